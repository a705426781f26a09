// Multigrid V-cycle with no-slip walls at both ends of any set of axes (the
// slit channel of Sec. 7 has them on the last axis; the box of Secs. 7.1 and
// 7.3 on every side), periodic along the others, with the boundary rules of
// the appendix on physical boundary conditions.
//
// Same cycle as the periodic one (red-black Gauss-Seidel, nu_pre sweeps from
// zero, residual restriction, rediscretised coarse operator c0 - (c1/4) L,
// prolongation, nu_post sweeps, nu_coarse sweeps on the 4^dim grid), with
// per field and axis one of four kinds:
//   periodic (no walls along the axis);
//   tangential velocity (cell-centred, mirror with the sign reversed) and the
//   pressure (cell-centred, mirror with the sign kept): a boundary cell's
//   ghost neighbour is the cell itself, so it moves into the diagonal
//   (c0 + (2 dim +- 1) c1); restriction averages the 2 children along the
//   axis; prolongation interpolates 3/4, 1/4 with the ghost coarse value;
//   normal velocity along its own axis (faces, the wall faces pinned to 0):
//   vertex-centred, so coarse face K sits on fine face 2K; restriction
//   weights the fine faces 2K-1, 2K, 2K+1 by 1/4, 1/2, 1/4; prolongation
//   copies coarse faces onto the even fine faces and averages neighbours onto
//   the odd ones (the wall faces get nothing).
// Transfers are tensor products of these one-dimensional rules.  The singular
// Neumann problem (pressure, c0 = 0) loses the mean of its coarsest
// right-hand side; its finest right-hand side has zero mean when it is a
// divergence, as in P_S^-1.
//
// Fields are in split (red half, black half) storage like the periodic
// hierarchy; these kernels take one cell per thread and address neighbours
// through split_index: the walls change the stencil only in the boundary
// layers, and this path is not the bandwidth-tuned periodic one.  From 4096
// cells (16^3, 64^2) down, the cycle runs in one workgroup per field with the
// levels in LDS (k_wvcycle_lds), on the same per-cell steps.
#include "kernels.h"

namespace ibr {

namespace {

enum WallKind : int { kPer = 0, kCellDir = 1, kFaceDir = 2, kCellNeu = 3 };

// Kinds of field f along the axes, two bits per axis (axis 0 lowest).
// mode 1: a velocity cycle (field f = component f); mode 2: the pressure
// cycle (one Neumann field).  wm: bit b = walls along axis b.
template <int DIM>
__device__ inline int field_kinds(int mode, int f, int wm) {
  int kinds = 0;
  for (int b = 0; b < DIM; ++b) {
    int k = kPer;
    if ((wm >> b) & 1) k = mode == 2 ? kCellNeu : (b == f ? kFaceDir : kCellDir);
    kinds |= k << (2 * b);
  }
  return kinds;
}

// Kind of axis b.  K >= 0: the kinds are the compile-time constant K (the
// per-cell steps below are instantiated for the combinations the slit and
// the box produce, so every per-axis branch folds away); K < 0: the run-time
// value `kinds`.
template <int K>
__device__ inline int kind_of(int kinds, int b) {
  return K >= 0 ? (K >> (2 * b)) & 3 : (kinds >> (2 * b)) & 3;
}

// Calls f(std::integral_constant<int, K>) with K = kinds for the field kinds
// of the slit channel and of the box (3D: walls on z, on every axis; 2D: on
// y, on both), K = -1 (run-time kinds) otherwise.
template <int DIM, typename F>
__device__ inline void with_kinds(int kinds, F&& f) {
  using std::integral_constant;
  if constexpr (DIM == 3) {
    switch (kinds) {
      case 16: f(integral_constant<int, 16>{}); return;  // slit: tangential velocity
      case 32: f(integral_constant<int, 32>{}); return;  // slit: normal velocity
      case 48: f(integral_constant<int, 48>{}); return;  // slit: pressure
      case 22: f(integral_constant<int, 22>{}); return;  // box: velocity along x
      case 25: f(integral_constant<int, 25>{}); return;  // box: velocity along y
      case 37: f(integral_constant<int, 37>{}); return;  // box: velocity along z
      case 63: f(integral_constant<int, 63>{}); return;  // box: pressure
      default: f(integral_constant<int, -1>{}); return;
    }
  } else {
    switch (kinds) {
      case 4: f(integral_constant<int, 4>{}); return;    // slit: tangential velocity
      case 8: f(integral_constant<int, 8>{}); return;    // slit: normal velocity
      case 12: f(integral_constant<int, 12>{}); return;  // slit: pressure
      case 6: f(integral_constant<int, 6>{}); return;    // box: velocity along x
      case 9: f(integral_constant<int, 9>{}); return;    // box: velocity along y
      case 15: f(integral_constant<int, 15>{}); return;  // box: pressure
      default: f(integral_constant<int, -1>{}); return;
    }
  }
}

// A wall face: index 0 along an axis of face kind.
template <int DIM, int K>
__device__ inline bool on_wall_face(const int* co, int kinds) {
  for (int b = 0; b < DIM; ++b)
    if (kind_of<K>(kinds, b) == kFaceDir && co[b] == 0) return true;
  return false;
}

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

// Cell of colour `color` with half-index t: natural coordinates.
template <int DIM>
__device__ inline void colour_cell(int t, int color, int logn, int* co) {
  const int hl = logn - 1;
  const int mask = (1 << logn) - 1;
  const int m = t & ((1 << hl) - 1);
  const int row = t >> hl;
  co[1] = row & mask;
  co[2] = DIM == 3 ? (row >> logn) : 0;
  co[0] = 2 * m + ((color + co[1] + co[2]) & 1);
}

template <typename T, int DIM>
__device__ inline T at(const T* x, const int* co, int logn) {
  return x[split_index<DIM>(co[0], co[1], co[2], logn)];
}

// Sum of the neighbours that are other unknowns, and the diagonal of
// (c0 - c1 L) at cell co.
template <typename T, int DIM, int K>
__device__ inline T nbr_sum(const T* x, const int* co, int logn, int kinds, T c0, T c1, T& diag) {
  const int n = 1 << logn;
  const int mask = n - 1;
  diag = c0 + T(2 * DIM) * c1;
  T sum = T(0);
#pragma unroll
  for (int b = DIM - 1; b >= 0; --b) {
    const int kind = kind_of<K>(kinds, b);
    int q[3] = {co[0], co[1], co[2]};
    T up = T(0), dn = T(0);
    if (kind == kPer) {
      q[b] = (co[b] + 1) & mask;
      up = at<T, DIM>(x, q, logn);
      q[b] = (co[b] - 1) & mask;
      dn = at<T, DIM>(x, q, logn);
    } else if (kind == kFaceDir) {
      // face n is the other wall (0); the wall face's own row is not an equation
      if (co[b] + 1 < n) {
        q[b] = co[b] + 1;
        up = at<T, DIM>(x, q, logn);
      }
      if (co[b] > 0) {
        q[b] = co[b] - 1;
        dn = at<T, DIM>(x, q, logn);
      }
    } else {
      const T s = kind == kCellDir ? T(1) : T(-1);
      if (co[b] + 1 < n) {
        q[b] = co[b] + 1;
        up = at<T, DIM>(x, q, logn);
      } else {
        diag += s * c1;
      }
      if (co[b] > 0) {
        q[b] = co[b] - 1;
        dn = at<T, DIM>(x, q, logn);
      } else {
        diag += s * c1;
      }
    }
    sum += up + dn;
  }
  return sum;
}

template <typename T, int DIM, int K>
__device__ inline T resid_at(const T* x, const T* b, const int* co, int logn, int kinds, T c0, T c1) {
  if (on_wall_face<DIM, K>(co, kinds)) return T(0);
  T diag;
  const T sum = nbr_sum<T, DIM, K>(x, co, logn, kinds, c0, c1, diag);
  return at<T, DIM>(b, co, logn) - (diag * at<T, DIM>(x, co, logn) - c1 * sum);
}

// ---- per-cell steps (global kernels: one cell per thread; the tail: loops)
// Half sweep at cell t of colour `color`.
template <typename T, int DIM, int K>
__device__ inline void wrb_cell(T* x, const T* b, int logn, T c0, T c1, int color, int t, int kinds) {
  const int C = 1 << (DIM * logn);
  int co[3];
  colour_cell<DIM>(t, color, logn, co);
  const int own = color * (C >> 1) + t;
  if (on_wall_face<DIM, K>(co, kinds)) {
    x[own] = T(0);
    return;
  }
  T diag;
  const T sum = nbr_sum<T, DIM, K>(x, co, logn, kinds, c0, c1, diag);
  x[own] = (b[own] + c1 * sum) / diag;
}

// Coarse right-hand side of coarse cell t (natural index) from the fine
// residual: its split index on the coarse level is returned in *at_c.  Per
// axis the fine points and weights of the one-dimensional restriction; the
// coarse value is their tensor product.
template <typename T, int DIM, int K>
__device__ inline T wrestrict_cell(const T* x, const T* b, int logn, T c0, T c1, int t, int kinds, int* at_c) {
  const int lognc = logn - 1;
  const int maskc = (1 << lognc) - 1;
  const int cc[3] = {t & maskc, (t >> lognc) & maskc, DIM == 3 ? (t >> (2 * lognc)) : 0};
  *at_c = split_index<DIM>(cc[0], cc[1], cc[2], lognc);
  int fi[3][3];
  T fw[3][3];
  int cnt[3] = {1, 1, 1};
  for (int a = 0; a < 3; ++a) {
    fi[a][0] = 0;
    fw[a][0] = T(1);
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (kind_of<K>(kinds, a) == kFaceDir) {
      if (cc[a] == 0) return T(0);  // the coarse wall face
      cnt[a] = 3;
      fi[a][0] = 2 * cc[a] - 1;
      fi[a][1] = 2 * cc[a];
      fi[a][2] = 2 * cc[a] + 1;
      fw[a][0] = T(0.25);
      fw[a][1] = T(0.5);
      fw[a][2] = T(0.25);
    } else {
      cnt[a] = 2;
      fi[a][0] = 2 * cc[a];
      fi[a][1] = 2 * cc[a] + 1;
      fw[a][0] = T(0.5);
      fw[a][1] = T(0.5);
    }
  }
  T out = T(0);
#pragma unroll
  for (int qz = 0; qz < 3; ++qz) {
    if (qz >= cnt[2]) break;
#pragma unroll
    for (int qy = 0; qy < 3; ++qy) {
      if (qy >= cnt[1]) break;
      T row = T(0);
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        if (qx >= cnt[0]) break;
        const int co[3] = {fi[0][qx], fi[1][qy], fi[2][qz]};
        row += fw[0][qx] * resid_at<T, DIM, K>(x, b, co, logn, kinds, c0, c1);
      }
      out += fw[1][qy] * fw[2][qz] * row;
    }
  }
  return out;
}

// x += P e at fine cell t (natural index).  Per axis the coarse points and
// weights of the one-dimensional interpolation (with a sign for a mirror
// ghost); the correction is their tensor product.
template <typename T, int DIM, int K>
__device__ inline void wprolong_cell(T* x, const T* e, int logn, int t, int kinds) {
  const int lognc = logn - 1;
  const int nc = 1 << lognc;
  const int mask = (1 << logn) - 1;
  const int co[3] = {t & mask, (t >> logn) & mask, DIM == 3 ? (t >> (2 * logn)) : 0};
  if (on_wall_face<DIM, K>(co, kinds)) return;
  int ci[3][2];
  T cw[3][2];
  int cnt[3] = {1, 1, 1};
  for (int a = 0; a < 3; ++a) {
    ci[a][0] = 0;
    cw[a][0] = T(1);
  }
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int kind = kind_of<K>(kinds, a);
    const int w = co[a], P = w >> 1;
    if (kind == kFaceDir) {
      // coarse face P on fine face 2P; odd faces average P and P + 1 (face nc is the wall)
      ci[a][0] = P;
      cw[a][0] = (w & 1) ? T(0.5) : T(1);
      cnt[a] = 1;
      if ((w & 1) && P + 1 < nc) {
        ci[a][1] = P + 1;
        cw[a][1] = T(0.5);
        cnt[a] = 2;
      }
    } else {
      int Q = (w & 1) ? P + 1 : P - 1;
      T s = T(1);
      if (kind == kPer) {
        Q &= nc - 1;
      } else if (Q < 0 || Q >= nc) {
        // beyond a wall: the boundary cell's mirror image
        Q = P;
        s = kind == kCellDir ? T(-1) : T(1);
      }
      ci[a][0] = P;
      cw[a][0] = T(0.75);
      ci[a][1] = Q;
      cw[a][1] = T(0.25) * s;
      cnt[a] = 2;
    }
  }
  T val = T(0);
#pragma unroll
  for (int qz = 0; qz < 2; ++qz) {
    if (qz >= cnt[2]) break;
#pragma unroll
    for (int qy = 0; qy < 2; ++qy) {
      if (qy >= cnt[1]) break;
      T row = T(0);
#pragma unroll
      for (int qx = 0; qx < 2; ++qx) {
        if (qx >= cnt[0]) break;
        const int cc[3] = {ci[0][qx], ci[1][qy], ci[2][qz]};
        row += cw[0][qx] * at<T, DIM>(e, cc, lognc);
      }
      val += cw[1][qy] * cw[2][qz] * row;
    }
  }
  x[split_index<DIM>(co[0], co[1], co[2], logn)] += val;
}

// ---- global kernels: fields in blockIdx.y
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wrb(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1,
                                             int color, int mode, int wm) {
  const int C = 1 << (DIM * logn);
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= (C >> 1)) return;
  const int f = blockIdx.y;
  const int kinds = field_kinds<DIM>(mode, f, wm);
  with_kinds<DIM>(kinds, [&](auto kc) {
    wrb_cell<T, DIM, decltype(kc)::value>(x + (int64_t)f * C, b + (int64_t)f * C, logn, c0, c1, color, t, kinds);
  });
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wresid_restrict(const T* __restrict__ x, const T* __restrict__ b,
                                                         T* __restrict__ bc, int logn, T c0, T c1, int mode,
                                                         int wm) {
  const int C = 1 << (DIM * logn), Cc = C >> DIM;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= Cc) return;
  const int f = blockIdx.y;
  const int kinds = field_kinds<DIM>(mode, f, wm);
  with_kinds<DIM>(kinds, [&](auto kc) {
    int at_c;
    const T r = wrestrict_cell<T, DIM, decltype(kc)::value>(x + (int64_t)f * C, b + (int64_t)f * C, logn, c0, c1,
                                                            t, kinds, &at_c);
    bc[(int64_t)f * Cc + at_c] = r;
  });
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wprolong(T* __restrict__ x, const T* __restrict__ e, int logn, int mode,
                                                  int wm) {
  const int C = 1 << (DIM * logn), Cc = C >> DIM;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= C) return;
  const int f = blockIdx.y;
  const int kinds = field_kinds<DIM>(mode, f, wm);
  with_kinds<DIM>(kinds, [&](auto kc) {
    wprolong_cell<T, DIM, decltype(kc)::value>(x + (int64_t)f * C, e + (int64_t)f * Cc, logn, t, kinds);
  });
}

// ---- the coarse tail in one workgroup per field
// Levels from the tail's entry (at most kWallTailCells cells) down to 4^dim
// run inside one workgroup with every level's x, and b below the entry, in
// LDS: the same per-cell steps as the global kernels, one launch instead of
// about eleven per level.
constexpr int kWallTailThreads = 512;
constexpr int kWallTailCells = 4096;
template <int DIM>
constexpr int wall_pyramid(int C) {
  int t = 0;
  for (int c = C; c >= (DIM == 3 ? 64 : 16); c >>= DIM) t += c;
  return t;
}

// Offset of level l in the tail's pyramid of levels (entry level 0 first).
template <int DIM>
__device__ inline int pyramid_off(int logn, int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += 1 << (DIM * (logn - i));
  return o;
}

// The tail's V-cycle for one field whose kinds are K (or the run-time kinds).
// xs: x of every level, entry level first; bs: b of the levels below the entry
// level (level l >= 1 at pyramid_off(l) - C0).
template <typename T, int DIM, int K>
__device__ inline void wvcycle_body(const T* __restrict__ b0, T* __restrict__ x0, T* xs, T* bs, T* red, int logn,
                                    T c0, T c1, int nu_pre, int nu_post, int nu_coarse, int mode, int kinds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int C0 = 1 << (DIM * logn);
  const int nlev = logn - 1;  // entry level down to n = 4
  auto xl = [&](int l) { return xs + pyramid_off<DIM>(logn, l); };
  auto bl = [&](int l) -> T* { return l == 0 ? nullptr : bs + (pyramid_off<DIM>(logn, l) - C0); };
  auto bread = [&](int l) -> const T* { return l == 0 ? b0 : bl(l); };
  T cl = c1;
  auto sweeps = [&](int l, T cc, int nsw) {
    const int lg = logn - l;
    const int H = 1 << (DIM * lg - 1);
    T* x = xl(l);
    const T* b = bread(l);
    for (int sw = 0; sw < nsw; ++sw)
      for (int color = 0; color < 2; ++color) {
        for (int t = tid; t < H; t += nt) wrb_cell<T, DIM, K>(x, b, lg, c0, cc, color, t, kinds);
        __syncthreads();
      }
  };
  for (int l = 0; l < nlev - 1; ++l) {
    const int lg = logn - l;
    const int Cl = 1 << (DIM * lg);
    T* x = xl(l);
    for (int c = tid; c < Cl; c += nt) x[c] = T(0);
    __syncthreads();
    sweeps(l, cl, nu_pre);
    const T* b = bread(l);
    T* bc = bl(l + 1);
    for (int t = tid; t < (Cl >> DIM); t += nt) {
      int at_c;
      const T r = wrestrict_cell<T, DIM, K>(x, b, lg, c0, cl, t, kinds, &at_c);
      bc[at_c] = r;
    }
    __syncthreads();
    cl = cl * T(0.25);
  }
  {
    const int l = nlev - 1;
    const int Cl = 1 << (DIM * (logn - l));
    if (mode == 2 && c0 == T(0)) {
      // the singular Neumann problem: the coarsest right-hand side loses its mean
      T* b = bl(l);
      T sm = T(0);
      for (int c = tid; c < Cl; c += nt) sm += b[c];
      sm = block_sum(sm, red);
      const T mean = sm / T(Cl);
      __syncthreads();
      for (int c = tid; c < Cl; c += nt) b[c] -= mean;
    }
    T* x = xl(l);
    for (int c = tid; c < Cl; c += nt) x[c] = T(0);
    __syncthreads();
    sweeps(l, cl, nu_coarse);
  }
  for (int l = nlev - 2; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const int Cl = 1 << (DIM * lg);
    T* x = xl(l);
    const T* xc = xl(l + 1);
    for (int t = tid; t < Cl; t += nt) wprolong_cell<T, DIM, K>(x, xc, lg, t, kinds);
    __syncthreads();
    sweeps(l, cl, nu_post);
  }
  for (int c = tid; c < C0; c += nt) x0[c] = xs[c];
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kWallTailThreads) k_wvcycle_lds(const T* __restrict__ bg, T* __restrict__ xg,
                                                                  int logn, T c0, T c1, int nu_pre, int nu_post,
                                                                  int nu_coarse, int mode, int wm) {
  constexpr int kX = wall_pyramid<DIM>(kWallTailCells);
  constexpr int kB = wall_pyramid<DIM>(kWallTailCells >> DIM) + 1;
  __shared__ T xs[kX];
  __shared__ T bs[kB];
  __shared__ T red[kWallTailThreads / kWave];
  const int f = blockIdx.x;
  const int kinds = field_kinds<DIM>(mode, f, wm);
  const int C0 = 1 << (DIM * logn);
  with_kinds<DIM>(kinds, [&](auto kc) {
    wvcycle_body<T, DIM, decltype(kc)::value>(bg + (int64_t)f * C0, xg + (int64_t)f * C0, xs, bs, red, logn, c0, c1,
                                             nu_pre, nu_post, nu_coarse, mode, kinds);
  });
}

}  // namespace

template <typename T>
void launch_wall_vcycle(int dim, int logn, int nf, const T* b, T* x, const std::vector<T*>& wx,
                        const std::vector<T*>& wb, double c0, double c1, int nu_pre, int nu_post, int nu_coarse,
                        int mode, int wm, hipStream_t s) {
  if (logn < 3) throw DeviceError("walls: grids need n >= 8");
  // levels above the tail run the global kernels; the tail starts at <= kWallTailCells cells
  int lt = 0;
  while (((int64_t)1 << (dim * (logn - lt))) > kWallTailCells) ++lt;
  if ((int)wx.size() <= lt || (int)wb.size() <= lt) throw DeviceError("walls: multigrid buffers missing");
  // the tail keeps b of its levels below the entry level in LDS: it needs at least two levels
  if (logn - lt < 3) throw DeviceError("walls: the multigrid tail needs an entry level of n >= 8");
  const bool three = dim == 3;
  const T tc0 = (T)c0;
  T cl = (T)c1;
  auto xl = [&](int l) { return l == 0 ? x : wx[l]; };
  auto bl = [&](int l) -> const T* { return l == 0 ? b : wb[l]; };
  auto half = [&](int l, int color) {
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    const dim3 g(nblk(Cl / 2), nf);
    // finest level: a live-timed class (algorithmic traffic as the periodic half sweep's)
    const TimerEvents ev = l == 0 ? timer_sample(kTimerWallRbFine, 1.5 * (double)Cl * nf * sizeof(T)) : TimerEvents();
    if (three)
      hipExtLaunchKernelGGL(k_wrb<T, 3>, g, dim3(256), 0, s, ev.start, ev.stop, 0, xl(l), bl(l), lg, tc0, cl, color,
                            mode, wm);
    else
      hipExtLaunchKernelGGL(k_wrb<T, 2>, g, dim3(256), 0, s, ev.start, ev.stop, 0, xl(l), bl(l), lg, tc0, cl, color,
                            mode, wm);
  };
  for (int l = 0; l < lt; ++l) {
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    launch_fill<T>(xl(l), Cl * nf, T(0), s);
    for (int sw = 0; sw < nu_pre; ++sw)
      for (int color = 0; color < 2; ++color) half(l, color);
    const dim3 g(nblk(Cl >> dim), nf);
    if (three)
      hipLaunchKernelGGL((k_wresid_restrict<T, 3>), g, dim3(256), 0, s, xl(l), bl(l), wb[l + 1], lg, tc0, cl, mode, wm);
    else
      hipLaunchKernelGGL((k_wresid_restrict<T, 2>), g, dim3(256), 0, s, xl(l), bl(l), wb[l + 1], lg, tc0, cl, mode, wm);
    cl = cl * T(0.25);
  }
  if (three)
    hipLaunchKernelGGL((k_wvcycle_lds<T, 3>), dim3(nf), dim3(kWallTailThreads), 0, s, bl(lt), xl(lt), logn - lt,
                       tc0, cl, nu_pre, nu_post, nu_coarse, mode, wm);
  else
    hipLaunchKernelGGL((k_wvcycle_lds<T, 2>), dim3(nf), dim3(kWallTailThreads), 0, s, bl(lt), xl(lt), logn - lt,
                       tc0, cl, nu_pre, nu_post, nu_coarse, mode, wm);
  for (int l = lt - 1; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    const dim3 g(nblk(Cl), nf);
    if (three)
      hipLaunchKernelGGL((k_wprolong<T, 3>), g, dim3(256), 0, s, xl(l), (const T*)xl(l + 1), lg, mode, wm);
    else
      hipLaunchKernelGGL((k_wprolong<T, 2>), g, dim3(256), 0, s, xl(l), (const T*)xl(l + 1), lg, mode, wm);
    for (int sw = 0; sw < nu_post; ++sw)
      for (int color = 0; color < 2; ++color) half(l, color);
  }
}

template void launch_wall_vcycle<double>(int, int, int, const double*, double*, const std::vector<double*>&,
                                         const std::vector<double*>&, double, double, int, int, int, int,
                                         int, hipStream_t);
template void launch_wall_vcycle<float>(int, int, int, const float*, float*, const std::vector<float*>&,
                                        const std::vector<float*>&, double, double, int, int, int, int,
                                        int, hipStream_t);

}  // namespace ibr
