// Fused multigrid level kernels for small 3D levels of the preconditioner's
// V-cycles (Sec. 5.2), in fp32 or fp64: temporal blocking in LDS.
//
// The unfused level runs one kernel per half sweep, one for the residual and
// restriction and one for the prolongation: nine dependent launches per level
// and cycle, each paying the kernel boundary (dispatch, drain, cache
// write-back between XCDs).  Here one workgroup owns an 8^3 tile of a level
// plus a halo of H = 2 nu cells, brings x and b of the whole block into LDS,
// runs every half sweep of one smoothing phase on a block that shrinks by
// one cell per half sweep (each half sweep reads the other colour one cell
// further out), and writes back only the interior, which is then exactly the
// result of the global sweeps.  Two kernels per level and cycle remain:
//   pre:  first sweep from x = 0, nu_pre - 1 more sweeps, residual, 2^3
//         averaging into the coarse right-hand side;
//   post: x += P e on the black cells (the first red half sweep overwrites the
//         red ones without reading them), nu_post sweeps.
// The arithmetic of every cell is that of the global kernels (same formulas,
// same order of the neighbour sum); the restriction uses the block identity
//   sum r = sum b - (diag - 3 c1) sum x + c1 (sum of outside face neighbours).
//
// LDS holds x and b of the block in split (red/black) storage: colour c,
// row = lj + E lk, half-row index li >> 1.  The block origin is even, so a
// cell's colour is the parity of its local coordinates.
#include "kernels.h"

namespace ibr {

namespace {

// Tile geometry: interior edge TT (8 or 16), halo H = 2 nu, block edge E;
// threads per workgroup scale with the block.
template <int NU, int TT>
struct FTile {
  static constexpr int T = TT;
  static constexpr int LT = TT == 16 ? 4 : 3;  // log2 TT
  static constexpr int H = 2 * NU;             // halo
  static constexpr int E = TT + 2 * H;         // block edge
  static constexpr int HR = E / 2;             // half-row
  static constexpr int HALF = E * E * HR;      // cells of one colour
  static constexpr int CE = E / 2 + 2;         // coarse block edge (post: e with one extra cell each side)
  static constexpr int NT = TT == 16 ? 1024 : 256;  // threads
};

__device__ inline int wrapm(int i, int mask) { return i & mask; }

// global split index of cell (i, j, k) (already wrapped) on a level of 2^logn
__device__ inline int gsplit(int i, int j, int k, int logn) {
  const int row = j | (k << logn);
  return (((i + j + k) & 1) << (3 * logn - 1)) | (row << (logn - 1)) | (i >> 1);
}

// Load a field of the block (E^3 cells around the tile at i0, j0, k0) into LDS.
// Every thread issues all of its global loads before its first LDS store, so
// they are in flight together.
template <typename V, int NU, int TT>
__device__ inline void load_block(V* s, const V* __restrict__ g, int i0, int j0, int k0, int logn) {
  using G = FTile<NU, TT>;
  constexpr int N = 2 * G::HALF;
  constexpr int PER = (N + G::NT - 1) / G::NT;
  const int mask = (1 << logn) - 1;
  V v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * G::NT;
    if (t < N) {
      const int c = t / G::HALF;
      const int r = t - c * G::HALF;
      const int row = r / G::HR;
      const int m = r - row * G::HR;
      const int lj = row % G::E, lk = row / G::E;
      const int li = 2 * m + ((c + lj + lk) & 1);
      const int i = wrapm(i0 - G::H + li, mask), j = wrapm(j0 - G::H + lj, mask), k = wrapm(k0 - G::H + lk, mask);
      v[u] = g[gsplit(i, j, k, logn)];
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * G::NT;
    if (t < N) s[t] = v[u];
  }
}

// Write the interior tile of x back to global memory.
template <typename V, int NU, int TT>
__device__ inline void store_interior(const V* s, V* __restrict__ g, int i0, int j0, int k0, int logn) {
  using G = FTile<NU, TT>;
  constexpr int IH = TT / 2;
  constexpr int N = TT * TT * TT;
  constexpr int PER = (N + G::NT - 1) / G::NT;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * G::NT;
    const int c = t / (TT * TT * IH);
    const int r = t - c * (TT * TT * IH);
    const int row = r / IH;
    const int m = r - row * IH;
    const int lj = G::H + row % TT, lk = G::H + row / TT;
    const int li = G::H + 2 * m + ((c + lj + lk) & 1);
    const int i = i0 - G::H + li, j = j0 - G::H + lj, k = k0 - G::H + lk;  // inside the level, no wrap
    g[gsplit(i, j, k, logn)] = s[c * G::HALF + (lj + G::E * lk) * G::HR + (li >> 1)];
  }
}

// One half sweep of colour C on the block [A, E - A)^3.  FIRST with C == 0:
// red cells from a zero guess (x = b / diag, no neighbours).  Each thread
// reads all of its cells' neighbours before it writes any result (the two
// colours never alias, but the compiler cannot tell), so the LDS reads of its
// cells overlap.
template <typename V, int NU, int TT, int A, int C, bool FIRST>
__device__ inline void block_half_sweep(V* xs, const V* bs, V c1, V inv_diag) {
  using G = FTile<NU, TT>;
  constexpr int W = G::E - 2 * A;
  constexpr int WH = W / 2;
  constexpr int CELLS = W * W * WH;
  constexpr int PER = (CELLS + G::NT - 1) / G::NT;
  const V* o = xs + (1 - C) * G::HALF;
  V* own = xs + C * G::HALF;
  const V* bo = bs + C * G::HALF;
  V res[PER];
  int at[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * G::NT;
    at[u] = -1;
    if (t < CELLS) {
      const int mp = t % WH;
      const int rw = t / WH;
      const int lj = A + rw % W, lk = A + rw / W;
      const int li = A + 2 * mp + ((C + lj + lk + A) & 1);
      const int row = lj + G::E * lk;
      const int self = row * G::HR + (li >> 1);
      at[u] = self;
      if (FIRST && C == 0) {
        res[u] = bo[self] * inv_diag;
      } else {
        V sum = o[row * G::HR + ((li - 1) >> 1)] + o[row * G::HR + ((li + 1) >> 1)] + o[self - G::HR] +
                    o[self + G::HR];
        sum += o[self - G::E * G::HR] + o[self + G::E * G::HR];
        res[u] = (bo[self] + c1 * sum) * inv_diag;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (at[u] >= 0) own[at[u]] = res[u];
}

template <typename V, int NU, int TT, int S>
__device__ inline void pre_sweeps(V* xs, const V* bs, V c1, V inv_diag) {
  if constexpr (S < NU) {
    block_half_sweep<V, NU, TT, 2 * S, 0, false>(xs, bs, c1, inv_diag);
    __syncthreads();
    block_half_sweep<V, NU, TT, 2 * S + 1, 1, false>(xs, bs, c1, inv_diag);
    __syncthreads();
    pre_sweeps<V, NU, TT, S + 1>(xs, bs, c1, inv_diag);
  }
}

template <typename V, int NU, int TT, int S>
__device__ inline void post_sweeps(V* xs, const V* bs, V c1, V inv_diag) {
  if constexpr (S < NU) {
    block_half_sweep<V, NU, TT, 2 * S + 1, 0, false>(xs, bs, c1, inv_diag);
    __syncthreads();
    block_half_sweep<V, NU, TT, 2 * S + 2, 1, false>(xs, bs, c1, inv_diag);
    __syncthreads();
    post_sweeps<V, NU, TT, S + 1>(xs, bs, c1, inv_diag);
  }
}

// Tile of workgroup: XCD-aware over the tiles of one field (neighbouring tiles,
// which share halo lines in L2, go to the same XCD), field in blockIdx.y.
template <int LT>
__device__ inline void tile_origin(int logn, int& i0, int& j0, int& k0) {
  const int tl = logn - LT;  // log2 tiles per axis
  const int t = (int)xcd_block(gridDim.x);
  i0 = (t & ((1 << tl) - 1)) << LT;
  j0 = ((t >> tl) & ((1 << tl) - 1)) << LT;
  k0 = (t >> (2 * tl)) << LT;
}

template <typename V, int NU, int TT>
__global__ void __launch_bounds__((FTile<NU, TT>::NT)) k_mg_pre(const V* __restrict__ b, V* __restrict__ x,
                                                          V* __restrict__ bc, int logn, V c0, V c1) {
  using G = FTile<NU, TT>;
  __shared__ V xs[2 * G::HALF];
  __shared__ V bs[2 * G::HALF];
  const int64_t C = (int64_t)1 << (3 * logn);
  const int64_t f = blockIdx.y;
  b += f * C;
  x += f * C;
  bc += f * (C >> 3);
  int i0, j0, k0;
  tile_origin<G::LT>(logn, i0, j0, k0);
  load_block<V, NU, TT>(bs, b, i0, j0, k0, logn);
  __syncthreads();
  const V diag = c0 + V(6) * c1;
  const V inv_diag = V(1) / diag;
  block_half_sweep<V, NU, TT, 0, 0, true>(xs, bs, c1, inv_diag);
  __syncthreads();
  block_half_sweep<V, NU, TT, 1, 1, true>(xs, bs, c1, inv_diag);
  __syncthreads();
  pre_sweeps<V, NU, TT, 1>(xs, bs, c1, inv_diag);
  store_interior<V, NU, TT>(xs, x, i0, j0, k0, logn);
  // residual summed over each 2^3 block of the tile, averaged into the coarse level
  constexpr int CT = TT / 2;
  constexpr int LC = G::LT - 1;
  const int lognc = logn - 1;
  for (int t = threadIdx.x; t < CT * CT * CT; t += blockDim.x) {
    const int ci = t & (CT - 1), cj = (t >> LC) & (CT - 1), ck = t >> (2 * LC);
    const int fi = G::H + 2 * ci, fj = G::H + 2 * cj, fk = G::H + 2 * ck;
    auto X = [&](int li, int lj, int lk) {
      return xs[((li + lj + lk) & 1) * G::HALF + (lj + G::E * lk) * G::HR + (li >> 1)];
    };
    auto B = [&](int li, int lj, int lk) {
      return bs[((li + lj + lk) & 1) * G::HALF + (lj + G::E * lk) * G::HR + (li >> 1)];
    };
    V sx = V(0), sb = V(0), sf = V(0);
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
      for (int dj = 0; dj < 2; ++dj) {
#pragma unroll
        for (int di = 0; di < 2; ++di) {
          sx += X(fi + di, fj + dj, fk + dk);
          sb += B(fi + di, fj + dj, fk + dk);
        }
        sf += X(fi - 1, fj + dj, fk + dk) + X(fi + 2, fj + dj, fk + dk);
      }
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
      for (int di = 0; di < 2; ++di) sf += X(fi + di, fj - 1, fk + dk) + X(fi + di, fj + 2, fk + dk);
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di) sf += X(fi + di, fj + dj, fk - 1) + X(fi + di, fj + dj, fk + 2);
    const V r = (sb - (diag - V(3) * c1) * sx + c1 * sf) * V(0.125);
    bc[gsplit((i0 >> 1) + ci, (j0 >> 1) + cj, (k0 >> 1) + ck, lognc)] = r;
  }
}

template <typename V, int NU, int TT>
__global__ void __launch_bounds__((FTile<NU, TT>::NT)) k_mg_post(const V* __restrict__ b,
                                                                 const V* __restrict__ xi,
                                                                 V* __restrict__ xo,
                                                                 const V* __restrict__ e, int logn, V c0,
                                                                 V c1) {
  using G = FTile<NU, TT>;
  __shared__ V xs[2 * G::HALF];
  __shared__ V bs[2 * G::HALF];
  __shared__ V es[G::CE * G::CE * G::CE];
  const int64_t C = (int64_t)1 << (3 * logn);
  const int64_t f = blockIdx.y;
  b += f * C;
  xi += f * C;
  xo += f * C;
  e += f * (C >> 3);
  int i0, j0, k0;
  tile_origin<G::LT>(logn, i0, j0, k0);
  load_block<V, NU, TT>(xs, xi, i0, j0, k0, logn);
  load_block<V, NU, TT>(bs, b, i0, j0, k0, logn);
  // coarse block: coarse cells (i0 - H)/2 - 1 ... + CE - 1 on each axis
  const int lognc = logn - 1;
  const int maskc = (1 << lognc) - 1;
  const int I0 = ((i0 - G::H) >> 1) - 1, J0 = ((j0 - G::H) >> 1) - 1, K0 = ((k0 - G::H) >> 1) - 1;
  {
    constexpr int NE = G::CE * G::CE * G::CE;
    constexpr int PER = (NE + G::NT - 1) / G::NT;
    V v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = threadIdx.x + u * G::NT;
      if (t < NE) {
        const int a = t % G::CE, rr = t / G::CE;
        const int bq = rr % G::CE, cq = rr / G::CE;
        v[u] = e[gsplit(wrapm(I0 + a, maskc), wrapm(J0 + bq, maskc), wrapm(K0 + cq, maskc), lognc)];
      }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = threadIdx.x + u * G::NT;
      if (t < NE) es[t] = v[u];
    }
  }
  __syncthreads();
  // x += P e on the black cells of the block (weights 3/4, 1/4 per axis; x, then y, then z)
  {
    const V w0 = V(0.75), w1 = V(0.25);
    V* xb = xs + G::HALF;
#pragma unroll 4
    for (int t = threadIdx.x; t < G::HALF; t += blockDim.x) {
      const int row = t / G::HR;
      const int m = t - row * G::HR;
      const int lj = row % G::E, lk = row / G::E;
      const int li = 2 * m + ((1 + lj + lk) & 1);
      // coarse cell of the fine cell and the side of its neighbours; the block
      // origin is even, so local and global parities agree
      const int ci = ((li - 0) >> 1) + 1, cj = (lj >> 1) + 1, ck = (lk >> 1) + 1;
      const int si = (li & 1) ? 1 : -1, sj = (lj & 1) ? 1 : -1, sk = (lk & 1) ? 1 : -1;
      auto Ec = [&](int a, int bq, int cq) { return es[a + G::CE * (bq + G::CE * cq)]; };
      const V a0 = w0 * Ec(ci, cj, ck) + w1 * Ec(ci + si, cj, ck);
      const V a1 = w0 * Ec(ci, cj + sj, ck) + w1 * Ec(ci + si, cj + sj, ck);
      const V a2 = w0 * Ec(ci, cj, ck + sk) + w1 * Ec(ci + si, cj, ck + sk);
      const V a3 = w0 * Ec(ci, cj + sj, ck + sk) + w1 * Ec(ci + si, cj + sj, ck + sk);
      const V b0 = w0 * a0 + w1 * a1;
      const V b1 = w0 * a2 + w1 * a3;
      xb[t] += w0 * b0 + w1 * b1;
    }
  }
  __syncthreads();
  const V inv_diag = V(1) / (c0 + V(6) * c1);
  post_sweeps<V, NU, TT, 0>(xs, bs, c1, inv_diag);
  store_interior<V, NU, TT>(xs, xo, i0, j0, k0, logn);
}


template <typename V, int TT>
static void pre_tt(const V* b, V* x, V* bc, int logn, int nf, V c0, V c1, int nu, hipStream_t s, TimerEvents ev) {
  const unsigned tiles = 1u << (3 * (logn - FTile<1, TT>::LT));
  if (nu == 2)
    hipExtLaunchKernelGGL((k_mg_pre<V, 2, TT>), dim3(tiles, nf), dim3(FTile<2, TT>::NT), 0, s, ev.start, ev.stop, 0,
                          b, x, bc, logn, c0, c1);
  else
    hipExtLaunchKernelGGL((k_mg_pre<V, 1, TT>), dim3(tiles, nf), dim3(FTile<1, TT>::NT), 0, s, ev.start, ev.stop, 0,
                          b, x, bc, logn, c0, c1);
}

template <typename V, int TT>
static void post_tt(const V* b, const V* xi, V* xo, const V* e, int logn, int nf, V c0, V c1, int nu, hipStream_t s,
                    TimerEvents ev) {
  const unsigned tiles = 1u << (3 * (logn - FTile<1, TT>::LT));
  if (nu == 2)
    hipExtLaunchKernelGGL((k_mg_post<V, 2, TT>), dim3(tiles, nf), dim3(FTile<2, TT>::NT), 0, s, ev.start, ev.stop, 0,
                          b, xi, xo, e, logn, c0, c1);
  else
    hipExtLaunchKernelGGL((k_mg_post<V, 1, TT>), dim3(tiles, nf), dim3(FTile<1, TT>::NT), 0, s, ev.start, ev.stop, 0,
                          b, xi, xo, e, logn, c0, c1);
}

}  // namespace

bool fused_level_ok(int dim, int logn, int nu) { return dim == 3 && logn >= 4 && (nu == 1 || nu == 2); }

// 8^3 tiles: 16^3 tiles (a 24^3 block, one workgroup of 1024 threads per
// compute unit) measured slower on every level, a block that large runs too
// long in one compute unit.
template <typename V>
void launch_mg_pre_fused(const V* b, V* x, V* bc, int logn, int nf, V c0, V c1, int nu, hipStream_t s,
                         TimerEvents ev) {
  pre_tt<V, 8>(b, x, bc, logn, nf, c0, c1, nu, s, ev);
}
template void launch_mg_pre_fused<float>(const float*, float*, float*, int, int, float, float, int, hipStream_t,
                                         TimerEvents);
template void launch_mg_pre_fused<double>(const double*, double*, double*, int, int, double, double, int,
                                          hipStream_t, TimerEvents);

template <typename V>
void launch_mg_post_fused(const V* b, const V* xi, V* xo, const V* e, int logn, int nf, V c0, V c1, int nu,
                          hipStream_t s, TimerEvents ev) {
  if (xi == xo) throw DeviceError("fused post-smoothing needs separate input and output x");
  post_tt<V, 8>(b, xi, xo, e, logn, nf, c0, c1, nu, s, ev);
}
template void launch_mg_post_fused<float>(const float*, const float*, float*, const float*, int, int, float, float,
                                          int, hipStream_t, TimerEvents);
template void launch_mg_post_fused<double>(const double*, const double*, double*, const double*, int, int, double,
                                           double, int, hipStream_t, TimerEvents);

}  // namespace ibr
