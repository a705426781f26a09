// MAC-grid stencil kernels (Sec. 3.2): the Stokes operator [[A, G], [-D, 0]],
// the pieces of the projection preconditioner P_S^-1 (Sec. 5.2,
// eq. P1_practical) and the explicit advection term of the unsteady step.
//
// Layout: field f of a vector lives at base + f*C, C = n^dim, x fastest.
// One thread per cell; blocks are remapped so each XCD walks a contiguous slab.
#include <type_traits>

#include "kernels.h"

namespace ibr {

namespace {

struct Nbr {
  int64_t m[3];  // c - e_a
  int64_t p[3];  // c + e_a
};

template <int DIM>
__device__ inline Nbr neighbours(int64_t c, int logn) {
  const int n = 1 << logn;
  const int mask = n - 1;
  Nbr r;
  int i = (int)(c & mask);
  r.m[0] = c - i + ((i - 1) & mask);
  r.p[0] = c - i + ((i + 1) & mask);
  int j = (int)((c >> logn) & mask);
  r.m[1] = c + ((int64_t)(((j - 1) & mask) - j) << logn);
  r.p[1] = c + ((int64_t)(((j + 1) & mask) - j) << logn);
  if (DIM == 3) {
    int k = (int)(c >> (2 * logn));
    r.m[2] = c + ((int64_t)(((k - 1) & mask) - k) << (2 * logn));
    r.p[2] = c + ((int64_t)(((k + 1) & mask) - k) << (2 * logn));
  } else {
    r.m[2] = r.p[2] = c;
  }
  return r;
}

// Natural (x fastest) storage of a cell lattice: cell <-> index.
template <int DIM>
struct Lat {
  int logn;
  __device__ void coords(int t, int& i, int& j, int& k) const {
    const int mask = (1 << logn) - 1;
    i = t & mask;
    j = (t >> logn) & mask;
    k = DIM == 3 ? (t >> (2 * logn)) : 0;
  }
  __device__ int index(int i, int j, int k) const { return natural_index<DIM>(i, j, k, logn); }
};

// yv = A v + G p + addc, yp = -D v.   A = c0 I - ch2 L,  G, D with 1/h.
// TI: storage type of the input, TO: of the output (arithmetic in TO).
// Natural storage, one thread per cell.
// walls: bit b set = no-slip walls at both ends of axis b.  Along a walled
// axis a tangential component's neighbour beyond a wall is its mirror image
// with the sign reversed (the cell itself, negated); the normal component's
// wall faces (index 0 along its own axis) hold 0 and are not equations
// (their rows are 0), and face n is the other wall.
template <typename TI, typename TO, int DIM>
__global__ void __launch_bounds__(256) k_stokes_apply(const TI* __restrict__ v, const TI* __restrict__ p,
                                                      TO* __restrict__ yv, TO* __restrict__ yp, int logn,
                                                      TO c0, TO ch2, TO inv_h,
                                                      const double* __restrict__ addc, int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t t64 = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (t64 >= C) return;
  const int t = (int)t64;
  const Lat<DIM> L{logn};
  int i, j, k;
  L.coords(t, i, j, k);
  const int co[3] = {i, j, k};
  int m[3], pl[3];
  m[0] = L.index(i - 1, j, k);
  pl[0] = L.index(i + 1, j, k);
  m[1] = L.index(i, j - 1, k);
  pl[1] = L.index(i, j + 1, k);
  m[2] = DIM == 3 ? L.index(i, j, k - 1) : t;
  pl[2] = DIM == 3 ? L.index(i, j, k + 1) : t;
  const TO pc = (TO)p[t];
  const int n = 1 << logn;
  TO div = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const TI* va = v + a * C;
    TO vc = (TO)va[t];
    TO nb[3][2];
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
      nb[q][0] = (TO)va[m[q]];
      nb[q][1] = (TO)va[pl[q]];
    }
    bool zero_row = false;
    if (walls) {
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        if (!((walls >> b) & 1)) continue;
        if (b == a) {
          if (co[b] == 0) {
            vc = TO(0);
            zero_row = true;
          }
          if (co[b] == 1) nb[b][0] = TO(0);
          if (co[b] == n - 1) nb[b][1] = TO(0);
        } else {
          if (co[b] == 0) nb[b][0] = -vc;
          if (co[b] == n - 1) nb[b][1] = -vc;
        }
      }
    }
    // the Laplacian as a sum of neighbour differences: each difference of two
    // nearby values is exact, so a smooth field keeps its digits (the form
    // sum - 2 dim vc loses about log10(n^2) of them to cancellation)
    TO lap = ((nb[0][0] - vc) + (nb[0][1] - vc)) + ((nb[1][0] - vc) + (nb[1][1] - vc));
    if (DIM == 3) lap += (nb[2][0] - vc) + (nb[2][1] - vc);
    TO out = c0 * vc - ch2 * lap + (pc - (TO)p[m[a]]) * inv_h;
    if (addc) out += (TO)addc[a];
    if (zero_row) out = TO(0);
    yv[a * C + t] = out;
    div += (nb[a][1] - vc) * inv_h;
  }
  yp[t] = -div;
}

// q = -D v - hp  (hp may be null), natural storage.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_div_q(const T* __restrict__ v, const T* __restrict__ hp,
                                               T* __restrict__ q, int logn, T inv_h) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t t64 = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (t64 >= C) return;
  const int t = (int)t64;
  const Lat<DIM> L{logn};
  int i, j, k;
  L.coords(t, i, j, k);
  const int pl[3] = {L.index(i + 1, j, k), L.index(i, j + 1, k), DIM == 3 ? L.index(i, j, k + 1) : t};
  T div = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) div += (v[a * C + pl[a]] - v[a * C + t]) * inv_h;
  q[t] = -div - (hp ? hp[t] : T(0));
}

// v <- v - vmean + h (phi_c - phi_{c-e_a});  pi = -c0 h^2 phi + eta q, natural
// storage; the normal components' wall faces stay 0 (walls: axis bits).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_ps_finish(T* __restrict__ v, const T* __restrict__ phi,
                                                   const T* __restrict__ q, T* __restrict__ pi, int logn,
                                                   T h, T c0h2, T eta, const double* __restrict__ vmean,
                                                   int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t t64 = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (t64 >= C) return;
  const int t = (int)t64;
  const Lat<DIM> L{logn};
  int i, j, k;
  L.coords(t, i, j, k);
  const int co[3] = {i, j, k};
  const int m[3] = {L.index(i - 1, j, k), L.index(i, j - 1, k), DIM == 3 ? L.index(i, j, k - 1) : t};
  const T ph = phi[t];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T mv = vmean ? (T)vmean[a] : T(0);
    const bool wall_face = ((walls >> a) & 1) && co[a] == 0;
    v[a * C + t] = wall_face ? T(0) : v[a * C + t] - mv + h * (ph - phi[m[a]]);
  }
  pi[t] = -c0h2 * ph + eta * q[t];
}

// ---------------------------------------------------------------- split storage, 4 cells per thread
// Each thread takes 4 consecutive cells of one colour in one row (split
// storage, see split_index): its own values and those of its neighbours come
// as 4-wide vectors of the other colour's rows, plus one x-neighbour beyond
// the group.  Arithmetic in the same order as the one-cell-per-thread kernels.
// Needs n >= 8.
template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T v[4];
};
template <typename T>
__device__ inline Q4<T> ld4(const T* p) {
  return *reinterpret_cast<const Q4<T>*>(p);
}
template <typename T>
__device__ inline void st4(T* p, const Q4<T>& q) {
  *reinterpret_cast<Q4<T>*>(p) = q;
}

// Offsets of a 4-cell group t (colour c, row (j, k), half-row offset m0) and
// of the rows and scalars its stencils read.
template <int DIM>
struct Group {
  int H, own, oth, xl, xr, ym, yp, zm, zp;
  int j, k;  // the group's row
  int i0;    // x coordinate of its first cell; cell u sits at i0 + 2u
  bool odd;  // the group's cells sit at i = 2m + 1
  __device__ Group(int t, int logn) {
    const int C = 1 << (DIM * logn);
    H = C >> 1;
    const int hl = logn - 1;
    const int mask = (1 << logn) - 1, hmask = (1 << hl) - 1;
    // the colours alternate every wavefront (lb = log2 of min(64, groups per
    // colour)), so one workgroup takes both colours of the same rows: what a
    // group reads of the other colour is what its neighbour wavefront owns,
    // still in cache, instead of a second pass over the field
    const int lb = DIM * logn - 3 < 6 ? DIM * logn - 3 : 6;
    const int c = (t >> lb) & 1;
    const int u = ((t >> (lb + 1)) << lb) | (t & ((1 << lb) - 1));
    const int m0 = (u & ((1 << (hl - 2)) - 1)) << 2;
    const int row = u >> (hl - 2);
    j = row & mask;
    k = DIM == 3 ? (row >> logn) : 0;
    odd = ((c + j + k) & 1) != 0;
    i0 = 2 * m0 + (odd ? 1 : 0);
    const int ob = (1 - c) * H;
    own = c * H + (row << hl) + m0;
    oth = ob + (row << hl) + m0;
    xl = ob + (row << hl) + ((m0 - 1) & hmask);
    xr = ob + (row << hl) + ((m0 + 4) & hmask);
    ym = ob + ((((j - 1) & mask) | (k << logn)) << hl) + m0;
    yp = ob + ((((j + 1) & mask) | (k << logn)) << hl) + m0;
    zm = DIM == 3 ? ob + ((j | (((k - 1) & mask) << logn)) << hl) + m0 : own;
    zp = DIM == 3 ? ob + ((j | (((k + 1) & mask) << logn)) << hl) + m0 : own;
  }
};

// (A v + G p, -D v) on split storage (the preconditioner's operator) for the
// 4-cell group g; out(f, off, q) receives field f's 4 values at storage
// offset off (f < DIM: velocity component f, f = DIM: the pressure row).
template <typename T, int DIM, typename Out>
__device__ inline void stokes_split4_group(const T* __restrict__ v, const T* __restrict__ p, int logn, T c0, T ch2,
                                           T inv_h, int walls, const Group<DIM>& g, Out&& out_fn) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const bool odd = g.odd;
  const Q4<T> pc = ld4(p + g.own);
  // p at c - e_a
  Q4<T> pm[3];
  {
    const Q4<T> po = ld4(p + g.oth);
    const T pe = p[g.xl];
#pragma unroll
    for (int u = 0; u < 4; ++u) pm[0].v[u] = odd ? po.v[u] : (u == 0 ? pe : po.v[u - 1]);
    pm[1] = ld4(p + g.ym);
    if (DIM == 3) pm[2] = ld4(p + g.zm);
  }
  T div[4] = {0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* va = v + a * C;
    Q4<T> vc = ld4(va + g.own);
    const Q4<T> vo = ld4(va + g.oth);
    const T ve = va[odd ? g.xr : g.xl];
    Q4<T> vym = ld4(va + g.ym), vyp = ld4(va + g.yp);
    Q4<T> vzm, vzp;
    if (DIM == 3) {
      vzm = ld4(va + g.zm);
      vzp = ld4(va + g.zp);
    }
    // walls (axis bits): along y and z the group's 4 cells share the
    // coordinate; along x each cell has its own
    const int n = 1 << logn;
    bool zero_rows = false;
    if (walls) {
#pragma unroll
      for (int b = 1; b < DIM; ++b) {
        if (!((walls >> b) & 1)) continue;
        const int cb = b == 1 ? g.j : g.k;
        Q4<T>& nm = b == 1 ? vym : vzm;
        Q4<T>& np = b == 1 ? vyp : vzp;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (b == a) {
            if (cb == 0) vc.v[u] = T(0);
            if (cb == 1) nm.v[u] = T(0);
            if (cb == n - 1) np.v[u] = T(0);
          } else {
            if (cb == 0) nm.v[u] = -vc.v[u];
            if (cb == n - 1) np.v[u] = -vc.v[u];
          }
        }
        if (b == a && cb == 0) zero_rows = true;
      }
    }
    Q4<T> out;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      T xl = odd ? vo.v[u] : (u == 0 ? ve : vo.v[u - 1]);
      T xr = odd ? (u == 3 ? ve : vo.v[u + 1]) : vo.v[u];
      T c = vc.v[u];
      bool zero_row = zero_rows;
      if (walls & 1) {
        const int iu = g.i0 + 2 * u;
        if (a == 0) {
          if (iu == 0) {
            c = T(0);
            zero_row = true;
          }
          if (iu == 1) xl = T(0);
          if (iu == n - 1) xr = T(0);
        } else {
          if (iu == 0) xl = -c;
          if (iu == n - 1) xr = -c;
        }
      }
      // neighbour differences (exact for nearby values; no cancellation of a sum)
      T lap = ((xl - c) + (xr - c)) + ((vym.v[u] - c) + (vyp.v[u] - c));
      if (DIM == 3) lap += (vzm.v[u] - c) + (vzp.v[u] - c);
      out.v[u] = zero_row ? T(0) : c0 * c - ch2 * lap + (pc.v[u] - pm[a].v[u]) * inv_h;
      const T vplus = a == 0 ? xr : (a == 1 ? vyp.v[u] : vzp.v[u]);
      div[u] += (vplus - c) * inv_h;
    }
    out_fn(a, g.own, out);
  }
  Q4<T> q;
#pragma unroll
  for (int u = 0; u < 4; ++u) q.v[u] = -div[u];
  out_fn(DIM, g.own, q);
}

// yv = A v + G p, yp = -D v on split storage.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_stokes_split4(const T* __restrict__ v, const T* __restrict__ p,
                                                       T* __restrict__ yv, T* __restrict__ yp, int logn, T c0, T ch2,
                                                       T inv_h, int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int t = (int)(xcd_block(gridDim.x) * blockDim.x + threadIdx.x);
  if (t >= (int)(C >> 2)) return;
  const Group<DIM> g(t, logn);
  stokes_split4_group<T, DIM>(v, p, logn, c0, ch2, inv_h, walls, g, [&](int f, int off, const Q4<T>& q) {
    if (f < DIM)
      st4(yv + f * C + off, q);
    else
      st4(yp + off, q);
  });
}

// The last column of a few-column least-squares problem formed on the fly:
// w = K (v, p) (as k_stokes_split4 computes it, rounded to T as it would be
// stored) is not written; instead each workgroup adds up, in fp64, its part
// of the normal equations of min_y || r - [W_0 .. W_{NS-2}, w] y || in the
// row order of the Gram reduction (upper triangle of the Gram matrix row by
// row, then the products with r).  W_b and r are stacked (DIM+1) C fluid
// vectors in split storage, W_b at stride ld.  part[q * gridDim.x + block].
template <typename T, int DIM, int NS>
__global__ void __launch_bounds__(256) k_stokes_gram4(const T* __restrict__ v, const T* __restrict__ p,
                                                      const T* __restrict__ W, int64_t ld, const T* __restrict__ r,
                                                      int logn, T c0, T ch2, T inv_h, int walls,
                                                      double* __restrict__ part) {
  constexpr int NQ = NS * (NS + 1) / 2 + NS;
  __shared__ double red[NQ][256 / kWave];
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int t = (int)(xcd_block(gridDim.x) * blockDim.x + threadIdx.x);
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (t < (int)(C >> 2)) {
    const Group<DIM> g(t, logn);
    stokes_split4_group<T, DIM>(v, p, logn, c0, ch2, inv_h, walls, g, [&](int f, int off, const Q4<T>& q4) {
      const int64_t o = f * C + off;
      const Q4<T> rr = ld4(r + o);
      Q4<T> wb[NS > 1 ? NS - 1 : 1];
#pragma unroll
      for (int b = 0; b < NS - 1; ++b) wb[b] = ld4(W + b * ld + o);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double w[NS];
#pragma unroll
        for (int b = 0; b < NS - 1; ++b) w[b] = (double)wb[b].v[u];
        w[NS - 1] = (double)q4.v[u];
        const double ri = (double)rr.v[u];
        int q = 0;
#pragma unroll
        for (int a = 0; a < NS; ++a)
#pragma unroll
          for (int b = a; b < NS; ++b) acc[q++] += w[a] * w[b];
#pragma unroll
        for (int a = 0; a < NS; ++a) acc[q++] += w[a] * ri;
      }
    });
  }
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) red[q][wv] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < NQ) {
    double s = 0;
    for (int u = 0; u < (int)(blockDim.x / kWave); ++u) s += red[threadIdx.x][u];
    part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// q = -D v - hp on split storage (hp may be null).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_div_q_split4(const T* __restrict__ v, const T* __restrict__ hp,
                                                      T* __restrict__ q, int logn, T inv_h) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int t = (int)(xcd_block(gridDim.x) * blockDim.x + threadIdx.x);
  if (t >= (int)(C >> 2)) return;
  const Group<DIM> g(t, logn);
  const bool odd = g.odd;
  T div[4] = {0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T* va = v + a * C;
    const Q4<T> vc = ld4(va + g.own);
    Q4<T> vp;
    if (a == 0) {
      const Q4<T> vo = ld4(va + g.oth);
      const T ve = va[g.xr];
#pragma unroll
      for (int u = 0; u < 4; ++u) vp.v[u] = odd ? (u == 3 ? ve : vo.v[u + 1]) : vo.v[u];
    } else {
      vp = ld4(va + (a == 1 ? g.yp : g.zp));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) div[u] += (vp.v[u] - vc.v[u]) * inv_h;
  }
  Q4<T> h4 = {{0, 0, 0, 0}};
  if (hp) h4 = ld4(hp + g.own);
  Q4<T> out;
#pragma unroll
  for (int u = 0; u < 4; ++u) out.v[u] = -div[u] - h4.v[u];
  st4(q + g.own, out);
}

// v <- v - vmean + h (phi_c - phi_{c-e_a});  pi = -c0 h^2 phi + eta q, split storage.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_ps_finish_split4(T* __restrict__ v, const T* __restrict__ phi,
                                                          const T* __restrict__ q, T* __restrict__ pi, int logn,
                                                          T h, T c0h2, T eta, const double* __restrict__ vmean,
                                                          int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int t = (int)(xcd_block(gridDim.x) * blockDim.x + threadIdx.x);
  if (t >= (int)(C >> 2)) return;
  const Group<DIM> g(t, logn);
  const bool odd = g.odd;
  const Q4<T> ph = ld4(phi + g.own);
  Q4<T> pm[3];
  {
    const Q4<T> po = ld4(phi + g.oth);
    const T pe = phi[g.xl];
#pragma unroll
    for (int u = 0; u < 4; ++u) pm[0].v[u] = odd ? po.v[u] : (u == 0 ? pe : po.v[u - 1]);
    pm[1] = ld4(phi + g.ym);
    if (DIM == 3) pm[2] = ld4(phi + g.zm);
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const T mv = vmean ? (T)vmean[a] : T(0);
    Q4<T> va = ld4(v + a * C + g.own);
    // the normal component's wall faces (index 0 along its own walled axis) stay 0
    const bool walled = (walls >> a) & 1;
    const bool row_face = walled && a > 0 && (a == 1 ? g.j : g.k) == 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool wall_face = row_face || (walled && a == 0 && g.i0 + 2 * u == 0);
      va.v[u] = wall_face ? T(0) : va.v[u] - mv + h * (ph.v[u] - pm[a].v[u]);
    }
    st4(v + a * C + g.own, va);
  }
  const Q4<T> qq = ld4(q + g.own);
  Q4<T> out;
#pragma unroll
  for (int u = 0; u < 4; ++u) out.v[u] = -c0h2 * ph.v[u] + eta * qq.v[u];
  st4(pi + g.own, out);
}

// Layout conversions between the public (natural) and the split storage of
// nf fields; one thread per natural cell.
template <typename TS, typename TD, int DIM>
__global__ void __launch_bounds__(256) k_to_split(const TS* __restrict__ src, TD* __restrict__ dst, int logn) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int64_t f = blockIdx.y;
  const int mask = (1 << logn) - 1;
  const int i = (int)c & mask, j = ((int)c >> logn) & mask, k = DIM == 3 ? ((int)c >> (2 * logn)) : 0;
  dst[f * C + split_index<DIM>(i, j, k, logn)] = (TD)src[f * C + c];
}

template <typename TS, typename TD, int DIM>
__global__ void __launch_bounds__(256) k_from_split(const TS* __restrict__ src, TD* __restrict__ dst, int logn) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int64_t f = blockIdx.y;
  const int mask = (1 << logn) - 1;
  const int i = (int)c & mask, j = ((int)c >> logn) & mask, k = DIM == 3 ? ((int)c >> (2 * logn)) : 0;
  dst[f * C + c] = (TD)src[f * C + split_index<DIM>(i, j, k, logn)];
}

// x (natural) = [x +] sum_j y[j] Z_j (split), fields f < nf of every Z_j.
template <typename TZ, typename TX, int DIM>
__global__ void __launch_bounds__(256) k_combine_from_split(const TZ* __restrict__ Z, int64_t ld, int kk,
                                                            const double* __restrict__ y, TX* __restrict__ x,
                                                            int logn, int assign) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int64_t f = blockIdx.y;
  const int mask = (1 << logn) - 1;
  const int i = (int)c & mask, j = ((int)c >> logn) & mask, k = DIM == 3 ? ((int)c >> (2 * logn)) : 0;
  const int64_t si = f * C + split_index<DIM>(i, j, k, logn);
  double acc = assign ? 0.0 : (double)x[f * C + c];
  for (int q = 0; q < kk; ++q) acc += y[q] * (double)Z[(int64_t)q * ld + si];
  x[f * C + c] = (TX)acc;
}

// Centred advective term N(v)^a = sum_b vbar^b (v^a_{c+e_b} - v^a_{c-e_b}) / (2h),
// vbar^b the average of the four b-faces around the a-face (b != a).
// walls (axis bits): along a walled axis a tangential component's neighbour
// beyond a wall is its negated self; the normal component's wall faces hold
// 0, so the averaged normal velocity and the normal component's own
// differences need no ghost, and its rows on the wall faces are 0.
template <int DIM>
__global__ void __launch_bounds__(256) k_advect(const double* __restrict__ v, double* __restrict__ N, int logn,
                                                double inv_2h, int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int n = 1 << logn;
  const int mask = n - 1;
  const Nbr nb = neighbours<DIM>(c, logn);
  const int co[3] = {(int)(c & mask), (int)((c >> logn) & mask), DIM == 3 ? (int)(c >> (2 * logn)) : 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double* va = v + a * C;
    if (((walls >> a) & 1) && co[a] == 0) {
      N[a * C + c] = 0.0;
      continue;
    }
    double acc = 0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      double vb;
      if (b == a) {
        vb = va[c];
      } else {
        const double* wv = v + b * C;
        const int64_t cm = nb.m[a];  // c - e_a
        // (c - e_a) + e_b
        const Nbr nm = neighbours<DIM>(cm, logn);
        vb = 0.25 * (wv[c] + wv[nb.p[b]] + wv[cm] + wv[nm.p[b]]);
      }
      double up = va[nb.p[b]], dn = va[nb.m[b]];
      if (((walls >> b) & 1) && a != b) {
        if (co[b] == n - 1) up = -va[c];
        if (co[b] == 0) dn = -va[c];
      }
      acc += vb * (up - dn) * inv_2h;
    }
    N[a * C + c] = acc;
  }
}

// Index and sign that lattice index j (any integer) reads along a walled
// axis through the mirror extension: repeated mirroring has period 2n.  A
// tangential component (cell-centred along the axis) is odd about each wall;
// the normal component is odd about the wall faces 0 and n, which hold 0.
__device__ inline int wall_fold(int j, int n, bool normal, double& sign) {
  const int jm = j & (2 * n - 1);
  if (normal) {
    if (jm == 0 || jm == n) {
      sign = 0.0;
      return 0;
    }
    if (jm < n) return jm;
    sign = -sign;
    return 2 * n - jm;
  }
  if (jm < n) return jm;
  sign = -sign;
  return 2 * n - 1 - jm;
}

// Semi-Lagrangian advection term N = (v - v_d) / dt.  Each a-face backtracks
// along the face velocity of the advective form (v^a itself and the four-face
// averages of the other components) to x - dt u, in lattice units the face
// index minus dtoh u, and v_d is v^a interpolated there multilinearly on the
// a-face lattice.  Periodic axes wrap with the power-of-two mask; along a
// walled axis the taps read through the mirror extension.  The displacement
// is clamped to +-2^20 cells so every index stays on the lattice whatever
// the velocity (a non-finite velocity still yields a non-finite N through
// v^a at the same face, or at the neighbour that carries it).
template <int DIM>
__global__ void __launch_bounds__(256) k_advect_sl(const double* __restrict__ v, double* __restrict__ N, int logn,
                                                   double dtoh, double inv_dt, int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = xcd_block(gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int n = 1 << logn;
  const int mask = n - 1;
  const Nbr nb = neighbours<DIM>(c, logn);
  int coord[3];
  coord[0] = (int)(c & mask);
  coord[1] = (int)((c >> logn) & mask);
  coord[2] = DIM == 3 ? (int)(c >> (2 * logn)) : 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double* va = v + a * C;
    if (((walls >> a) & 1) && coord[a] == 0) {
      N[a * C + c] = 0.0;
      continue;
    }
    int lo[3];
    double fr[3];
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      double ub;
      if (b == a) {
        ub = va[c];
      } else {
        const double* wv = v + b * C;
        const int64_t cm = nb.m[a];
        const Nbr nm = neighbours<DIM>(cm, logn);
        ub = 0.25 * (wv[c] + wv[nb.p[b]] + wv[cm] + wv[nm.p[b]]);
      }
      const double disp = fmin(fmax(dtoh * ub, -1048576.0), 1048576.0);
      const double sb = (double)coord[b] - disp;
      const double fl = floor(sb);
      lo[b] = (int)fl;
      fr[b] = sb - fl;
    }
    double acc = 0.0;
#pragma unroll
    for (int corner = 0; corner < (1 << DIM); ++corner) {
      double w = 1.0, sign = 1.0;
      int64_t idx = 0;
#pragma unroll
      for (int b = DIM - 1; b >= 0; --b) {
        const int o = (corner >> b) & 1;
        w *= o ? fr[b] : 1.0 - fr[b];
        int j = lo[b] + o;
        if ((walls >> b) & 1)
          j = wall_fold(j, n, a == b, sign);
        else
          j &= mask;
        idx = (idx << logn) | j;
      }
      acc += w * sign * va[idx];
    }
    N[a * C + c] = (va[c] - acc) * inv_dt;
  }
}

// Zero the normal components' wall faces (index 0 along a walled axis a of
// component a); natural storage, one thread per cell.
template <int DIM>
__global__ void __launch_bounds__(256) k_zero_wall_faces(double* __restrict__ v, int logn, int walls) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int mask = (1 << logn) - 1;
  const int co[3] = {(int)(c & mask), (int)((c >> logn) & mask), DIM == 3 ? (int)(c >> (2 * logn)) : 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (((walls >> a) & 1) && co[a] == 0) v[a * C + c] = 0.0;
}

// v += scale u_b, u_b the background flow of moving walls: component a is
// lo[a] + (hi[a] - lo[a]) z / l along the walled axis `axis` (z of the
// a-face: k h on the faces normal to that axis, (k + 1/2) h otherwise).
// Faces on the walls of the axes in `skip` keep their value: there the
// momentum rows are identities whose right-hand side must stay zero.
template <int DIM>
__global__ void __launch_bounds__(256) k_add_background(double* __restrict__ v, int logn, double h, double len,
                                                        int axis, WallVel wv, double scale, int skip) {
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int mask = (1 << logn) - 1;
  const int co[3] = {(int)(c & mask), (int)((c >> logn) & mask), DIM == 3 ? (int)(c >> (2 * logn)) : 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (((skip >> a) & 1) && co[a] == 0) continue;
    const double z = (co[axis] + (a == axis ? 0.0 : 0.5)) * h;
    v[a * C + c] += scale * (wv.lo[a] + (wv.hi[a] - wv.lo[a]) * z / len);
  }
}

// Vm[m] -= u_b(R_m): the background flow at the markers (the kernel
// interpolates linear fields exactly, mirror ghosts included).
__global__ void k_sub_background_markers(double* __restrict__ Vm, const double* __restrict__ R, int N, int dim,
                                         int axis, double len, WallVel wv) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const double z = R[(int64_t)m * dim + axis];
  for (int a = 0; a < dim; ++a) Vm[(int64_t)m * dim + a] -= wv.lo[a] + (wv.hi[a] - wv.lo[a]) * z / len;
}

// g = (rho/dt) v - rho (w1 N1 + w0 N0)   (N0 may be null)
__global__ void k_ns_rhs(const double* __restrict__ v, const double* __restrict__ N1,
                         const double* __restrict__ N0, double* __restrict__ g, int64_t len, double rdt,
                         double rho, double w1, double w0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = w1 * N1[i];
  if (N0) s += w0 * N0[i];
  g[i] = rdt * v[i] - rho * s;
}

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

}  // namespace

template <typename TI, typename TO>
void launch_stokes_apply(int dim, int logn, const TI* v, const TI* p, TO* yv, TO* yp, double c0, double ch2,
                         double inv_h, const double* addc, hipStream_t s, bool split, TimerEvents ev,
                         int walls) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (split) {
    // the preconditioner's operator: same storage type in and out, no added constant
    if constexpr (std::is_same<TI, TO>::value) {
      if (!addc) {
        if (dim == 3)
          hipLaunchKernelGGL((k_stokes_split4<TO, 3>), dim3(nblk(C / 4)), dim3(256), 0, s, v, p, yv, yp, logn,
                             (TO)c0, (TO)ch2, (TO)inv_h, walls);
        else
          hipLaunchKernelGGL((k_stokes_split4<TO, 2>), dim3(nblk(C / 4)), dim3(256), 0, s, v, p, yv, yp, logn,
                             (TO)c0, (TO)ch2, (TO)inv_h, walls);
        return;
      }
    }
    throw DeviceError("launch_stokes_apply: split storage needs equal input/output types and no added constant");
  }
  // natural storage (the outer operator): the one launch a timer samples
  if (dim == 3)
    hipExtLaunchKernelGGL(k_stokes_apply<TI, TO, 3>, dim3(nblk(C)), dim3(256), 0, s, ev.start, ev.stop, 0, v, p, yv,
                          yp, logn, (TO)c0, (TO)ch2, (TO)inv_h, addc, walls);
  else
    hipExtLaunchKernelGGL(k_stokes_apply<TI, TO, 2>, dim3(nblk(C)), dim3(256), 0, s, ev.start, ev.stop, 0, v, p, yv,
                          yp, logn, (TO)c0, (TO)ch2, (TO)inv_h, addc, walls);
}
template void launch_stokes_apply<double, double>(int, int, const double*, const double*, double*, double*,
                                                  double, double, double, const double*, hipStream_t, bool,
                                                  TimerEvents, int);
template void launch_stokes_apply<float, double>(int, int, const float*, const float*, double*, double*,
                                                 double, double, double, const double*, hipStream_t, bool,
                                                 TimerEvents, int);
template void launch_stokes_apply<float, float>(int, int, const float*, const float*, float*, float*, double,
                                                double, double, const double*, hipStream_t, bool, TimerEvents, int);

int stokes_gram_blocks(int dim, int logn) { return (int)nblk(((int64_t)1 << (dim * logn)) / 4); }

template <typename T>
void launch_stokes_gram(int dim, int logn, const T* v, const T* p, const T* W, int64_t ld, int ns, const T* r,
                        double c0, double ch2, double inv_h, int walls, double* part, hipStream_t s) {
  const dim3 grid(stokes_gram_blocks(dim, logn));
  switch (dim * 8 + ns) {
#define IBR_SG(D, NS)                                                                                           \
  case D * 8 + NS:                                                                                             \
    hipLaunchKernelGGL((k_stokes_gram4<T, D, NS>), grid, dim3(256), 0, s, v, p, W, ld, r, logn, (T)c0, (T)ch2, \
                       (T)inv_h, walls, part);                                                                 \
    break;
    IBR_SG(2, 1) IBR_SG(2, 2) IBR_SG(2, 3) IBR_SG(3, 1) IBR_SG(3, 2) IBR_SG(3, 3)
#undef IBR_SG
    default:
      throw DeviceError("launch_stokes_gram: n_s must be 1, 2 or 3");
  }
}
template void launch_stokes_gram<float>(int, int, const float*, const float*, const float*, int64_t, int,
                                        const float*, double, double, double, int, double*, hipStream_t);
template void launch_stokes_gram<double>(int, int, const double*, const double*, const double*, int64_t, int,
                                         const double*, double, double, double, int, double*, hipStream_t);

template <typename T>
void launch_div_q(int dim, int logn, const T* v, const T* hp, T* q, double inv_h, hipStream_t s, bool split) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (split) {
    if (dim == 3)
      hipLaunchKernelGGL((k_div_q_split4<T, 3>), dim3(nblk(C / 4)), dim3(256), 0, s, v, hp, q, logn, (T)inv_h);
    else
      hipLaunchKernelGGL((k_div_q_split4<T, 2>), dim3(nblk(C / 4)), dim3(256), 0, s, v, hp, q, logn, (T)inv_h);
    return;
  }
  if (dim == 3)
    hipLaunchKernelGGL((k_div_q<T, 3>), dim3(nblk(C)), dim3(256), 0, s, v, hp, q, logn, (T)inv_h);
  else
    hipLaunchKernelGGL((k_div_q<T, 2>), dim3(nblk(C)), dim3(256), 0, s, v, hp, q, logn, (T)inv_h);
}
template void launch_div_q<double>(int, int, const double*, const double*, double*, double, hipStream_t, bool);
template void launch_div_q<float>(int, int, const float*, const float*, float*, double, hipStream_t, bool);

template <typename T>
void launch_ps_finish(int dim, int logn, T* v, const T* phi, const T* q, T* pi, double h, double c0h2,
                      double eta, const double* vmean, hipStream_t s, bool split, int walls) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (split) {
    if (dim == 3)
      hipLaunchKernelGGL((k_ps_finish_split4<T, 3>), dim3(nblk(C / 4)), dim3(256), 0, s, v, phi, q, pi, logn, (T)h,
                         (T)c0h2, (T)eta, vmean, walls);
    else
      hipLaunchKernelGGL((k_ps_finish_split4<T, 2>), dim3(nblk(C / 4)), dim3(256), 0, s, v, phi, q, pi, logn, (T)h,
                         (T)c0h2, (T)eta, vmean, walls);
    return;
  }
  if (dim == 3)
    hipLaunchKernelGGL((k_ps_finish<T, 3>), dim3(nblk(C)), dim3(256), 0, s, v, phi, q, pi, logn, (T)h, (T)c0h2,
                       (T)eta, vmean, walls);
  else
    hipLaunchKernelGGL((k_ps_finish<T, 2>), dim3(nblk(C)), dim3(256), 0, s, v, phi, q, pi, logn, (T)h, (T)c0h2,
                       (T)eta, vmean, walls);
}
template void launch_ps_finish<double>(int, int, double*, const double*, const double*, double*, double, double,
                                       double, const double*, hipStream_t, bool, int);
template void launch_ps_finish<float>(int, int, float*, const float*, const float*, float*, double, double,
                                      double, const double*, hipStream_t, bool, int);

template <typename TS, typename TD>
void launch_to_split(int dim, int logn, const TS* src, TD* dst, int nf, hipStream_t s) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL((k_to_split<TS, TD, 3>), dim3(nblk(C), nf), dim3(256), 0, s, src, dst, logn);
  else
    hipLaunchKernelGGL((k_to_split<TS, TD, 2>), dim3(nblk(C), nf), dim3(256), 0, s, src, dst, logn);
}
template void launch_to_split<double, double>(int, int, const double*, double*, int, hipStream_t);
template void launch_to_split<double, float>(int, int, const double*, float*, int, hipStream_t);

template <typename TS, typename TD>
void launch_from_split(int dim, int logn, const TS* src, TD* dst, int nf, hipStream_t s) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL((k_from_split<TS, TD, 3>), dim3(nblk(C), nf), dim3(256), 0, s, src, dst, logn);
  else
    hipLaunchKernelGGL((k_from_split<TS, TD, 2>), dim3(nblk(C), nf), dim3(256), 0, s, src, dst, logn);
}
template void launch_from_split<double, double>(int, int, const double*, double*, int, hipStream_t);
template void launch_from_split<float, double>(int, int, const float*, double*, int, hipStream_t);

template <typename TZ, typename TX>
void launch_combine_from_split(int dim, int logn, const TZ* Z, int64_t ld, int k, const double* y, TX* x, int nf,
                               bool assign, hipStream_t s) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL((k_combine_from_split<TZ, TX, 3>), dim3(nblk(C), nf), dim3(256), 0, s, Z, ld, k, y, x, logn,
                       assign ? 1 : 0);
  else
    hipLaunchKernelGGL((k_combine_from_split<TZ, TX, 2>), dim3(nblk(C), nf), dim3(256), 0, s, Z, ld, k, y, x, logn,
                       assign ? 1 : 0);
}
template void launch_combine_from_split<double, double>(int, int, const double*, int64_t, int, const double*,
                                                        double*, int, bool, hipStream_t);
template void launch_combine_from_split<float, float>(int, int, const float*, int64_t, int, const double*, float*,
                                                      int, bool, hipStream_t);

void launch_add_background(int dim, int logn, double* v, double h, double len, int axis, WallVel wv, double scale,
                           int skip, hipStream_t s) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL(k_add_background<3>, dim3(nblk(C)), dim3(256), 0, s, v, logn, h, len, axis, wv, scale, skip);
  else
    hipLaunchKernelGGL(k_add_background<2>, dim3(nblk(C)), dim3(256), 0, s, v, logn, h, len, axis, wv, scale, skip);
}

void launch_sub_background_markers(double* Vm, const double* R, int N, int dim, int axis, double len, WallVel wv,
                                   hipStream_t s) {
  if (N > 0)
    hipLaunchKernelGGL(k_sub_background_markers, dim3(nblk(N)), dim3(256), 0, s, Vm, R, N, dim, axis, len, wv);
}

void launch_zero_wall_faces(int dim, int logn, double* v, int walls, hipStream_t s) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL(k_zero_wall_faces<3>, dim3(nblk(C)), dim3(256), 0, s, v, logn, walls);
  else
    hipLaunchKernelGGL(k_zero_wall_faces<2>, dim3(nblk(C)), dim3(256), 0, s, v, logn, walls);
}

void launch_advect(int dim, int logn, const double* v, double* N, double inv_2h, hipStream_t s, int walls) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL((k_advect<3>), dim3(nblk(C)), dim3(256), 0, s, v, N, logn, inv_2h, walls);
  else
    hipLaunchKernelGGL((k_advect<2>), dim3(nblk(C)), dim3(256), 0, s, v, N, logn, inv_2h, walls);
}

void launch_advect_sl(int dim, int logn, const double* v, double* N, double dtoh, double inv_dt, hipStream_t s,
                      int walls) {
  const int64_t C = (int64_t)1 << (dim * logn);
  if (dim == 3)
    hipLaunchKernelGGL((k_advect_sl<3>), dim3(nblk(C)), dim3(256), 0, s, v, N, logn, dtoh, inv_dt, walls);
  else
    hipLaunchKernelGGL((k_advect_sl<2>), dim3(nblk(C)), dim3(256), 0, s, v, N, logn, dtoh, inv_dt, walls);
}

void launch_ns_rhs(const double* v, const double* N1, const double* N0, double* g, int64_t len, double rdt,
                   double rho, double w1, double w0, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_rhs, dim3(nblk(len)), dim3(256), 0, s, v, N1, N0, g, len, rdt, rho, w1, w0);
}

}  // namespace ibr
