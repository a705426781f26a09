// Geometric multigrid V-cycle for (c0 - c1 L) x = b on periodic n^dim lattices
// (Sec. 5.2 approximates A^-1 and L_p^-1 by one V-cycle each).
//
// Cycle: red-black Gauss-Seidel (red = even i+j+k first), nu_pre sweeps from a
// zero guess, residual + 2^dim averaging, rediscretised coarse operator
// (c0 - c1/4 L), cell-centred multilinear prolongation (3/4, 1/4 per axis),
// nu_post sweeps, nu_coarse sweeps on the 4^dim grid.  Singular problems
// (c0 == 0) lose the mean of the coarsest right-hand side; the finest-level
// mean of x is removed by the caller.
//
// Fine levels run one kernel per step with nfields batched in blockIdx.y.
// The coarse tail of the cycle runs inside ONE workgroup per field
// (k_vcycle_lds) with every array of the tail levels in LDS: one launch
// instead of ~10 per level.  The tail starts at 4096 cells (16^3, 64^2): one
// compute unit sweeping a 32^3 level costs more than the launches it saves.
#include "kernels.h"

namespace ibr {

namespace {

constexpr int kLdsThreads = 1024;

// Largest level (cells) handled inside one workgroup, per precision and dimension.
template <typename T, int DIM>
constexpr int64_t lds_max_cells() {
  return 4096;
}
// Cells of all levels from C down to the 4^dim grid.
template <int DIM>
constexpr int64_t pyramid_cells(int64_t C) {
  int64_t t = 0;
  for (int64_t c = C; c >= (DIM == 3 ? 64 : 16); c >>= DIM) t += c;
  return t;
}
// The right-hand sides of tail levels with more cells than this stay in a
// global scratch array (written and re-read by the same workgroup).
template <typename T, int DIM>
constexpr int64_t lds_b_max_cells() {
  return lds_max_cells<T, DIM>() >> DIM;
}

// ---------------------------------------------------------------- helpers
// Indices inside one field are 32-bit (n^dim <= 2^27 for the grids accepted);
// field offsets are applied to the base pointers in 64-bit.
template <int DIM>
__device__ inline void cell_coords(int c, int logn, int& i, int& j, int& k) {
  const int mask = (1 << logn) - 1;
  i = c & mask;
  j = (c >> logn) & mask;
  k = DIM == 3 ? (c >> (2 * logn)) : 0;
}

template <int DIM>
__device__ inline int cell_index(int i, int j, int k, int logn) {
  const int mask = (1 << logn) - 1;
  int c = (i & mask) | ((j & mask) << logn);
  if (DIM == 3) c |= (k & mask) << (2 * logn);
  return c;
}

template <typename T, int DIM>
__device__ inline T nbr_sum(const T* x, int i, int j, int k, int logn) {
  T s = x[cell_index<DIM>(i - 1, j, k, logn)] + x[cell_index<DIM>(i + 1, j, k, logn)] +
        x[cell_index<DIM>(i, j - 1, k, logn)] + x[cell_index<DIM>(i, j + 1, k, logn)];
  if (DIM == 3) s += x[cell_index<DIM>(i, j, k - 1, logn)] + x[cell_index<DIM>(i, j, k + 1, logn)];
  return s;
}

// Cell of colour `color` with colour-local index t (half the cells): row-major
// pairs, the colour picks the parity inside each pair.
template <int DIM>
__device__ inline void colour_cell(int t, int logn, int color, int& i, int& j, int& k) {
  const int half_log = logn - 1;
  const int m = t & ((1 << half_log) - 1);
  const int row = t >> half_log;
  const int mask = (1 << logn) - 1;
  j = row & mask;
  k = DIM == 3 ? (row >> logn) : 0;
  i = 2 * m + ((j + k + color) & 1);
}

__device__ inline int flat_thread(unsigned nblocks) {
  return (int)xcd_block(nblocks) * (int)blockDim.x + (int)threadIdx.x;
}

// ---------------------------------------------------------------- fine-level kernels
// Four consecutive cells of one x-row, loaded and stored as one vector.
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T v[4];
};

// One red-black half sweep.  Each thread owns 4 consecutive cells of an
// x-row, 2 of them of the colour being updated: the row and its y/z
// neighbour rows are read as 4-wide vectors, plus the one x-neighbour outside
// the segment.  The 2 cells of the other colour are written back unchanged
// (no thread changes them during this half sweep).  FINE marks the finest
// level (same code; a separate symbol for profiling).  Needs n >= 4.
template <typename T, int DIM, bool FINE>
__global__ void __launch_bounds__(256) k_rb(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1,
                                            int color) {
  const int C = 1 << (DIM * logn);
  const int t = flat_thread(gridDim.x);
  if (t >= (C >> 2)) return;
  const int64_t f = blockIdx.y;
  x += f * C;
  b += f * C;
  const int mask = (1 << logn) - 1;
  const int qlog = logn - 2;  // segments per row = n/4
  const int i0 = (t & ((1 << qlog) - 1)) << 2;
  const int row = t >> qlog;
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const int p = (j + k + color) & 1;  // first cell of the colour in the segment
  const int o = (row << logn) + i0;
  Quad<T> xc = *reinterpret_cast<const Quad<T>*>(x + o);
  const Quad<T> bc = *reinterpret_cast<const Quad<T>*>(b + o);
  const int ry0 = (((j - 1) & mask) + (k << logn)) << logn, ry1 = (((j + 1) & mask) + (k << logn)) << logn;
  const Quad<T> ym = *reinterpret_cast<const Quad<T>*>(x + ry0 + i0);
  const Quad<T> yp = *reinterpret_cast<const Quad<T>*>(x + ry1 + i0);
  Quad<T> zm, zp;
  if (DIM == 3) {
    const int rz0 = (j + (((k - 1) & mask) << logn)) << logn, rz1 = (j + (((k + 1) & mask) << logn)) << logn;
    zm = *reinterpret_cast<const Quad<T>*>(x + rz0 + i0);
    zp = *reinterpret_cast<const Quad<T>*>(x + rz1 + i0);
  }
  // the x-neighbour outside the segment: left of cell 0 or right of cell 3
  const T ext = x[(row << logn) + ((p == 0 ? i0 - 1 : i0 + 4) & mask)];
  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  // the two cells of the colour are (0, 2) or (1, 3); static indices and a
  // select keep the four-cell vectors in registers
  const bool odd = p != 0;
  const T l0 = odd ? xc.v[0] : ext, r0 = odd ? xc.v[2] : xc.v[1];
  const T l1 = odd ? xc.v[2] : xc.v[1], r1 = odd ? ext : xc.v[3];
  T s0 = l0 + r0 + (odd ? ym.v[1] : ym.v[0]) + (odd ? yp.v[1] : yp.v[0]);
  T s1 = l1 + r1 + (odd ? ym.v[3] : ym.v[2]) + (odd ? yp.v[3] : yp.v[2]);
  if (DIM == 3) {
    s0 += (odd ? zm.v[1] : zm.v[0]) + (odd ? zp.v[1] : zp.v[0]);
    s1 += (odd ? zm.v[3] : zm.v[2]) + (odd ? zp.v[3] : zp.v[2]);
  }
  const T n0 = ((odd ? bc.v[1] : bc.v[0]) + c1 * s0) * inv_diag;
  const T n1 = ((odd ? bc.v[3] : bc.v[2]) + c1 * s1) * inv_diag;
  xc.v[0] = odd ? xc.v[0] : n0;
  xc.v[1] = odd ? n0 : xc.v[1];
  xc.v[2] = odd ? xc.v[2] : n1;
  xc.v[3] = odd ? n1 : xc.v[3];
  *reinterpret_cast<Quad<T>*>(x + o) = xc;
}

// The first red-black sweep from a zero guess in one pass: red cells take
// b/diag, black cells (all of whose neighbours are red) take
// (b + c1 * sum of the neighbours' b/diag)/diag.  Same arithmetic, in the same
// order, as a red then a black half sweep from x = 0.  Four cells of a row
// per thread, as in k_rb.
template <typename T, int DIM, bool FINE>
__global__ void __launch_bounds__(256) k_rb_first(T* __restrict__ x, const T* __restrict__ b, int logn, T c0,
                                                  T c1) {
  const int C = 1 << (DIM * logn);
  const int t = flat_thread(gridDim.x);
  if (t >= (C >> 2)) return;
  const int64_t f = blockIdx.y;
  x += f * C;
  b += f * C;
  const int mask = (1 << logn) - 1;
  const int qlog = logn - 2;
  const int i0 = (t & ((1 << qlog) - 1)) << 2;
  const int row = t >> qlog;
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const int p = (j + k + 1) & 1;  // first black cell of the segment
  const int o = (row << logn) + i0;
  const Quad<T> bc = *reinterpret_cast<const Quad<T>*>(b + o);
  const int ry0 = (((j - 1) & mask) + (k << logn)) << logn, ry1 = (((j + 1) & mask) + (k << logn)) << logn;
  const Quad<T> ym = *reinterpret_cast<const Quad<T>*>(b + ry0 + i0);
  const Quad<T> yp = *reinterpret_cast<const Quad<T>*>(b + ry1 + i0);
  Quad<T> zm, zp;
  if (DIM == 3) {
    const int rz0 = (j + (((k - 1) & mask) << logn)) << logn, rz1 = (j + (((k + 1) & mask) << logn)) << logn;
    zm = *reinterpret_cast<const Quad<T>*>(b + rz0 + i0);
    zp = *reinterpret_cast<const Quad<T>*>(b + rz1 + i0);
  }
  const T ext = b[(row << logn) + ((p == 0 ? i0 - 1 : i0 + 4) & mask)];
  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  // black cells are (0, 2) or (1, 3); static indices and a select keep the
  // four-cell vectors in registers
  const bool odd = p != 0;
  const T l0 = odd ? bc.v[0] : ext, r0 = odd ? bc.v[2] : bc.v[1];
  const T l1 = odd ? bc.v[2] : bc.v[1], r1 = odd ? ext : bc.v[3];
  T s0 = l0 * inv_diag + r0 * inv_diag + (odd ? ym.v[1] : ym.v[0]) * inv_diag +
         (odd ? yp.v[1] : yp.v[0]) * inv_diag;
  T s1 = l1 * inv_diag + r1 * inv_diag + (odd ? ym.v[3] : ym.v[2]) * inv_diag +
         (odd ? yp.v[3] : yp.v[2]) * inv_diag;
  if (DIM == 3) {
    s0 += (odd ? zm.v[1] : zm.v[0]) * inv_diag + (odd ? zp.v[1] : zp.v[0]) * inv_diag;
    s1 += (odd ? zm.v[3] : zm.v[2]) * inv_diag + (odd ? zp.v[3] : zp.v[2]) * inv_diag;
  }
  const T n0 = ((odd ? bc.v[1] : bc.v[0]) + c1 * s0) * inv_diag;
  const T n1 = ((odd ? bc.v[3] : bc.v[2]) + c1 * s1) * inv_diag;
  Quad<T> xo;
  xo.v[0] = odd ? bc.v[0] * inv_diag : n0;
  xo.v[1] = odd ? n0 : bc.v[1] * inv_diag;
  xo.v[2] = odd ? bc.v[2] * inv_diag : n1;
  xo.v[3] = odd ? n1 : bc.v[3] * inv_diag;
  *reinterpret_cast<Quad<T>*>(x + o) = xo;
}

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T v[2];
};

// Coarse right-hand side = average over the 2^dim children of the residual
// r = b - (diag x - c1 sum_nbr x).  Summed over a 2^dim block, each child's
// neighbour along each axis inside the block is a sibling, so
//   sum r = sum b - (diag - dim c1) sum x + c1 (sum of the 4^(dim-1) 2 dim
//           face neighbours outside the block).
// Each thread makes two coarse cells (four fine cells along x) from 4-wide
// row vectors.  Needs n >= 4.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_resid_restrict(const T* __restrict__ x, const T* __restrict__ b,
                                                        T* __restrict__ bc, int logn, T c0, T c1) {
  const int lognc = logn - 1;
  const int Cc = 1 << (DIM * lognc);
  const int C = 1 << (DIM * logn);
  const int t = flat_thread(gridDim.x);
  if (t >= (Cc >> 1)) return;
  const int64_t f = blockIdx.y;
  x += f * C;
  b += f * C;
  const int mask = (1 << logn) - 1;
  const int qlog = logn - 2;  // coarse-cell pairs per coarse row
  const int q = t & ((1 << qlog) - 1);
  const int rowc = t >> qlog;
  const int J = rowc & ((1 << lognc) - 1);
  const int K = DIM == 3 ? (rowc >> lognc) : 0;
  const int i0 = q << 2;
  T sx0 = 0, sx1 = 0, sb0 = 0, sb1 = 0, sf0 = 0, sf1 = 0;
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int ro = (((2 * J + dy) & mask) + (((2 * K + dz) & mask) << logn)) << logn;
      const Quad<T> xq = *reinterpret_cast<const Quad<T>*>(x + ro + i0);
      const Quad<T> bq = *reinterpret_cast<const Quad<T>*>(b + ro + i0);
      const T xl = x[ro + ((i0 - 1) & mask)], xr = x[ro + ((i0 + 4) & mask)];
      sx0 += xq.v[0] + xq.v[1];
      sx1 += xq.v[2] + xq.v[3];
      sb0 += bq.v[0] + bq.v[1];
      sb1 += bq.v[2] + bq.v[3];
      sf0 += xl + xq.v[2];
      sf1 += xq.v[1] + xr;
    }
  // y faces: rows 2J-1 and 2J+2
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int y = e == 0 ? 2 * J - 1 : 2 * J + 2;
      const int ro = ((y & mask) + (((2 * K + dz) & mask) << logn)) << logn;
      const Quad<T> yq = *reinterpret_cast<const Quad<T>*>(x + ro + i0);
      sf0 += yq.v[0] + yq.v[1];
      sf1 += yq.v[2] + yq.v[3];
    }
  if (DIM == 3) {
    // z faces: planes 2K-1 and 2K+2
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int z = e == 0 ? 2 * K - 1 : 2 * K + 2;
        const int ro = (((2 * J + dy) & mask) + ((z & mask) << logn)) << logn;
        const Quad<T> zq = *reinterpret_cast<const Quad<T>*>(x + ro + i0);
        sf0 += zq.v[0] + zq.v[1];
        sf1 += zq.v[2] + zq.v[3];
      }
  }
  const T diag = c0 + T(2 * DIM) * c1;
  const T inner = diag - T(DIM) * c1;
  const T avg = DIM == 3 ? T(0.125) : T(0.25);
  Pair<T> out;
  out.v[0] = (sb0 - inner * sx0 + c1 * sf0) * avg;
  out.v[1] = (sb1 - inner * sx1 + c1 * sf1) * avg;
  *reinterpret_cast<Pair<T>*>(bc + f * Cc + (rowc << lognc) + 2 * q) = out;
}

// x += P e (multilinear, cell-centred: weights 3/4 and 1/4 per axis).  Each
// thread owns four fine cells of an x-row; each of the 2^(dim-1) coarse rows
// it needs is interpolated along x once (a pair load and two scalars).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_prolong_add(T* __restrict__ x, const T* __restrict__ e, int logn) {
  const int C = 1 << (DIM * logn);
  const int lognc = logn - 1;
  const int Cc = 1 << (DIM * lognc);
  const int t = flat_thread(gridDim.x);
  if (t >= (C >> 2)) return;
  const int64_t f = blockIdx.y;
  x += f * C;
  e += f * Cc;
  const int mask = (1 << logn) - 1, maskc = (1 << lognc) - 1;
  const int qlog = logn - 2;
  const int i0 = (t & ((1 << qlog) - 1)) << 2;
  const int row = t >> qlog;
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const int J = j >> 1, K = k >> 1;
  const int sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
  const int I0 = i0 >> 1;
  const T w0 = T(0.75), w1 = T(0.25);
  T a[4][4];  // [coarse row: (J,K), (J+sj,K), (J,K+sk), (J+sj,K+sk)][fine cell]
#pragma unroll
  for (int r = 0; r < (DIM == 3 ? 4 : 2); ++r) {
    const int Jr = J + ((r & 1) ? sj : 0), Kr = K + ((r & 2) ? sk : 0);
    const int ro = ((Jr & maskc) + ((Kr & maskc) << lognc)) << lognc;
    const Pair<T> p = *reinterpret_cast<const Pair<T>*>(e + ro + I0);
    const T em = e[ro + ((I0 - 1) & maskc)], ep = e[ro + ((I0 + 2) & maskc)];
    a[r][0] = w0 * p.v[0] + w1 * em;
    a[r][1] = w0 * p.v[0] + w1 * p.v[1];
    a[r][2] = w0 * p.v[1] + w1 * p.v[0];
    a[r][3] = w0 * p.v[1] + w1 * ep;
  }
  Quad<T> xq = *reinterpret_cast<const Quad<T>*>(x + (row << logn) + i0);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    T v;
    if (DIM == 3) {
      const T b0 = w0 * a[0][u] + w1 * a[1][u];
      const T b1 = w0 * a[2][u] + w1 * a[3][u];
      v = w0 * b0 + w1 * b1;
    } else {
      v = w0 * a[0][u] + w1 * a[1][u];
    }
    xq.v[u] += v;
  }
  *reinterpret_cast<Quad<T>*>(x + (row << logn) + i0) = xq;
}

// ---------------------------------------------------------------- one-workgroup tail
template <typename T, int DIM>
__device__ void lds_rb_sweeps(T* x, const T* b, int logn, T c0, T c1, int sweeps, bool from_zero) {
  const int C = 1 << (DIM * logn);
  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  if (from_zero) {
    for (int c = threadIdx.x; c < C; c += blockDim.x) x[c] = T(0);
    __syncthreads();
  }
  for (int s = 0; s < sweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      for (int t = threadIdx.x; t < C / 2; t += blockDim.x) {
        int i, j, k;
        colour_cell<DIM>(t, logn, color, i, j, k);
        const int c = cell_index<DIM>(i, j, k, logn);
        x[c] = (b[c] + c1 * nbr_sum<T, DIM>(x, i, j, k, logn)) * inv_diag;
      }
      __syncthreads();
    }
  }
}

template <typename T, int DIM>
__device__ void lds_resid_restrict(const T* x, const T* b, T* bc, int logn, T c0, T c1) {
  const int lognc = logn - 1;
  const int Cc = 1 << (DIM * lognc);
  const T diag = c0 + T(2 * DIM) * c1;
  for (int t = threadIdx.x; t < Cc; t += blockDim.x) {
    int I, J, K;
    cell_coords<DIM>(t, lognc, I, J, K);
    T acc = 0;
    for (int dk = 0; dk < (DIM == 3 ? 2 : 1); ++dk)
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
          const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
          const int c = cell_index<DIM>(i, j, k, logn);
          acc += b[c] - (diag * x[c] - c1 * nbr_sum<T, DIM>(x, i, j, k, logn));
        }
    bc[t] = acc * (DIM == 3 ? T(0.125) : T(0.25));
  }
  __syncthreads();
}

template <typename T, int DIM>
__device__ void lds_prolong_add(T* x, const T* e, int logn) {
  const int C = 1 << (DIM * logn);
  const int lognc = logn - 1;
  const T w0 = T(0.75), w1 = T(0.25);
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    int i, j, k;
    cell_coords<DIM>(c, logn, i, j, k);
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
    T v;
    if (DIM == 3) {
      T a00 = w0 * e[cell_index<DIM>(I, J, K, lognc)] + w1 * e[cell_index<DIM>(I + si, J, K, lognc)];
      T a10 = w0 * e[cell_index<DIM>(I, J + sj, K, lognc)] + w1 * e[cell_index<DIM>(I + si, J + sj, K, lognc)];
      T a01 = w0 * e[cell_index<DIM>(I, J, K + sk, lognc)] + w1 * e[cell_index<DIM>(I + si, J, K + sk, lognc)];
      T a11 = w0 * e[cell_index<DIM>(I, J + sj, K + sk, lognc)] +
              w1 * e[cell_index<DIM>(I + si, J + sj, K + sk, lognc)];
      T b0 = w0 * a00 + w1 * a10;
      T b1 = w0 * a01 + w1 * a11;
      v = w0 * b0 + w1 * b1;
    } else {
      T a0 = w0 * e[cell_index<DIM>(I, J, 0, lognc)] + w1 * e[cell_index<DIM>(I + si, J, 0, lognc)];
      T a1 = w0 * e[cell_index<DIM>(I, J + sj, 0, lognc)] + w1 * e[cell_index<DIM>(I + si, J + sj, 0, lognc)];
      v = w0 * a0 + w1 * a1;
    }
    x[c] += v;
  }
  __syncthreads();
}

template <typename T>
__device__ void lds_remove_mean(T* b, int C, T* red) {
  T s = 0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) s += b[c];
  s = block_sum(s, red);
  const T m = s / T(C);
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) b[c] -= m;
  __syncthreads();
}

// V-cycle from a level of at most lds_max_cells cells down to n = 4, one field
// per workgroup.  The entry level's b is read from global memory (kept in L2),
// as are the right-hand sides too large for LDS (bscr, C/2^dim cells per
// field); every other array of the tail lives in LDS.  c1 is the coefficient
// at the entry level.
template <typename T, int DIM>
__global__ void __launch_bounds__(kLdsThreads) k_vcycle_lds(const T* __restrict__ bg, T* __restrict__ xg,
                                                            T* __restrict__ bscr, int logn, T c0, T c1, int nu_pre,
                                                            int nu_post, int nu_coarse) {
  constexpr int64_t kX = pyramid_cells<DIM>(lds_max_cells<T, DIM>()) + 64;
  constexpr int64_t kB = pyramid_cells<DIM>(lds_b_max_cells<T, DIM>()) + 64;
  // x of every level back to back (entry level first); b of the levels >= 1 that fit.
  __shared__ T xs[kX];
  __shared__ T bs[kB];
  __shared__ T red[kLdsThreads / kWave];
  const int C0 = 1 << (DIM * logn);
  const T* b0 = bg + (int64_t)blockIdx.x * C0;
  T* x0 = xg + (int64_t)blockIdx.x * C0;
  const bool singular = c0 == T(0);

  const int nlev = logn - 1;  // entry level down to n = 4
  int xoff[10];
  T* bptr[10];
  {
    int xo = 0, bo = 0;
    for (int l = 0; l < nlev; ++l) {
      const int Cl = 1 << (DIM * (logn - l));
      xoff[l] = xo;
      xo += Cl;
      bptr[l] = nullptr;
      if (l >= 1) {
        if (Cl <= lds_b_max_cells<T, DIM>()) {
          bptr[l] = bs + bo;
          bo += Cl;
        } else {
          bptr[l] = bscr + (int64_t)blockIdx.x * Cl;
        }
      }
    }
  }
  auto xlev = [&](int l) -> T* { return xs + xoff[l]; };

  // The entry level reads b from global memory.
  T cl = c1;
  for (int l = 0; l < nlev - 1; ++l) {
    const int lg = logn - l;
    const T* bl = l == 0 ? b0 : bptr[l];
    lds_rb_sweeps<T, DIM>(xlev(l), bl, lg, c0, cl, nu_pre, true);
    lds_resid_restrict<T, DIM>(xlev(l), bl, bptr[l + 1], lg, c0, cl);
    cl = cl * T(0.25);
  }
  {
    const int l = nlev - 1;
    const int lg = logn - l;
    T* bl = bptr[l];
    if (l == 0) {
      // whole cycle is the coarsest grid: copy b to LDS first
      bl = bs;  // C0 <= 64 here
      for (int c = threadIdx.x; c < C0; c += blockDim.x) bl[c] = b0[c];
      __syncthreads();
    }
    if (singular) lds_remove_mean<T>(bl, 1 << (DIM * lg), red);
    lds_rb_sweeps<T, DIM>(xlev(l), bl, lg, c0, cl, nu_coarse, true);
  }
  for (int l = nlev - 2; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const T* bl = l == 0 ? b0 : bptr[l];
    lds_prolong_add<T, DIM>(xlev(l), xlev(l + 1), lg);
    lds_rb_sweeps<T, DIM>(xlev(l), bl, lg, c0, cl, nu_post, false);
  }
  for (int c = threadIdx.x; c < C0; c += blockDim.x) x0[c] = xs[c];
}

// Per-field sums: partial[f][block] (deterministic two-pass reduction).
template <typename T>
__global__ void __launch_bounds__(256) k_field_partial(const T* __restrict__ x, int64_t C,
                                                       double* __restrict__ part) {
  __shared__ double red[256 / kWave];
  const int64_t f = blockIdx.y;
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < C; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[f * C + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[f * gridDim.x + blockIdx.x] = s;
}

__global__ void k_field_finish(const double* __restrict__ part, int nblocks, double scale,
                               double* __restrict__ out) {
  __shared__ double red[256 / kWave];
  const int f = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[f * nblocks + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[f] = s * scale;
}

template <typename T>
__global__ void k_sub_field_mean(T* __restrict__ x, int64_t C, const double* __restrict__ mean) {
  const int64_t f = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < C; i += (int64_t)gridDim.x * blockDim.x)
    x[f * C + i] -= (T)mean[f];
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, int64_t len, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

// The sweeps read and write 4 consecutive cells as one vector.
template <typename T>
void check_quad_aligned(const T* x, const T* b) {
  if (((uintptr_t)x | (uintptr_t)b) % (4 * sizeof(T)) != 0)
    throw DeviceError("multigrid: field arrays must be aligned to 4 elements");
}

}  // namespace


template <typename T>
void launch_fill(T* x, int64_t len, T v, hipStream_t s) {
  unsigned g = nblk(len);
  if (g > 8192) g = 8192;
  if (g == 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(256), 0, s, x, len, v);
}
template void launch_fill<double>(double*, int64_t, double, hipStream_t);
template void launch_fill<float>(float*, int64_t, float, hipStream_t);
template void launch_fill<int>(int*, int64_t, int, hipStream_t);

template <typename T>
void launch_field_means(const T* x, int nf, int64_t C, double* part, int part_blocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_field_partial<T>, dim3(part_blocks, nf), dim3(256), 0, s, x, C, part);
  hipLaunchKernelGGL(k_field_finish, dim3(nf), dim3(256), 0, s, part, part_blocks, 1.0 / (double)C, out);
}
template void launch_field_means<double>(const double*, int, int64_t, double*, int, double*, hipStream_t);
template void launch_field_means<float>(const float*, int, int64_t, double*, int, double*, hipStream_t);

template <typename T>
void launch_sub_field_mean(T* x, int nf, int64_t C, const double* mean, hipStream_t s) {
  unsigned g = nblk(C);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_sub_field_mean<T>, dim3(g, nf), dim3(256), 0, s, x, C, mean);
}
template void launch_sub_field_mean<double>(double*, int, int64_t, const double*, hipStream_t);
template void launch_sub_field_mean<float>(float*, int, int64_t, const double*, hipStream_t);

template <typename T>
void MGHier<T>::init(int dim_, int logn_, int maxf) {
  dim = dim_;
  logn = logn_;
  nfmax = maxf;
  levels.clear();
  // multi-kernel levels: while the level has more cells than one workgroup holds
  const int64_t cap = dim == 3 ? lds_max_cells<T, 3>() : lds_max_cells<T, 2>();
  int lg = logn;
  while (((int64_t)1 << (dim * lg)) > cap) {
    levels.push_back(lg);
    --lg;
  }
  lds_logn = lg;
  bufs_x.assign(levels.size() + 1, nullptr);
  bufs_b.assign(levels.size() + 1, nullptr);
  for (size_t l = 1; l <= levels.size(); ++l) {
    const int lgl = logn - (int)l;
    const int64_t Cl = (int64_t)1 << (dim * lgl);
    bufs_x[l] = dev_alloc<T>(Cl * nfmax);
    bufs_b[l] = dev_alloc<T>(Cl * nfmax);
  }
  // right-hand side of the tail's second level when it does not fit in LDS
  const int64_t bmax = dim == 3 ? lds_b_max_cells<T, 3>() : lds_b_max_cells<T, 2>();
  const int64_t c1 = lg >= 1 ? (int64_t)1 << (dim * (lg - 1)) : 0;
  tail_b = c1 > bmax ? dev_alloc<T>(c1 * nfmax) : nullptr;
}

template <typename T>
void MGHier<T>::release() {
  for (auto p : bufs_x) dev_free(p);
  for (auto p : bufs_b) dev_free(p);
  dev_free(tail_b);
  tail_b = nullptr;
  bufs_x.clear();
  bufs_b.clear();
}

template <typename T>
size_t MGHier<T>::bytes(int dim, int logn, int nf) {
  size_t tot = 0;
  const int64_t cap = dim == 3 ? lds_max_cells<T, 3>() : lds_max_cells<T, 2>();
  int lg = logn;
  while (((int64_t)1 << (dim * lg)) > cap) --lg;
  for (int l = logn - 1; l >= lg; --l) tot += 2 * ((size_t)1 << (dim * l)) * nf * sizeof(T);
  const int64_t bmax = dim == 3 ? lds_b_max_cells<T, 3>() : lds_b_max_cells<T, 2>();
  const int64_t c1 = lg >= 1 ? (int64_t)1 << (dim * (lg - 1)) : 0;
  if (c1 > bmax) tot += (size_t)c1 * nf * sizeof(T);
  return tot;
}

template <typename T>
void MGHier<T>::rb_half(T* x, const T* b, int lg, int nf, T c0, T c1, int color, bool fine, hipStream_t s) {
  const int64_t Cl = (int64_t)1 << (dim * lg);
  check_quad_aligned(x, b);
  const dim3 gh(nblk(Cl / 4), nf);
  if (fine) timer_begin(kTimerRbFine, s);
  if (dim == 3) {
    if (fine)
      hipLaunchKernelGGL((k_rb<T, 3, true>), gh, dim3(256), 0, s, x, b, lg, c0, c1, color);
    else
      hipLaunchKernelGGL((k_rb<T, 3, false>), gh, dim3(256), 0, s, x, b, lg, c0, c1, color);
  } else {
    if (fine)
      hipLaunchKernelGGL((k_rb<T, 2, true>), gh, dim3(256), 0, s, x, b, lg, c0, c1, color);
    else
      hipLaunchKernelGGL((k_rb<T, 2, false>), gh, dim3(256), 0, s, x, b, lg, c0, c1, color);
  }
  // algorithmic traffic of a half sweep: b and x of one colour, x of the other
  if (fine) timer_end(kTimerRbFine, s, 1.5 * (double)Cl * nf * sizeof(T));
}

template <typename T>
void MGHier<T>::rb_first(T* x, const T* b, int lg, int nf, T c0, T c1, bool fine, hipStream_t s) {
  const int64_t Cl = (int64_t)1 << (dim * lg);
  check_quad_aligned(x, b);
  const dim3 g(nblk(Cl / 4), nf);
  if (fine) timer_begin(kTimerRbFine, s);
  if (dim == 3) {
    if (fine)
      hipLaunchKernelGGL((k_rb_first<T, 3, true>), g, dim3(256), 0, s, x, b, lg, c0, c1);
    else
      hipLaunchKernelGGL((k_rb_first<T, 3, false>), g, dim3(256), 0, s, x, b, lg, c0, c1);
  } else {
    if (fine)
      hipLaunchKernelGGL((k_rb_first<T, 2, true>), g, dim3(256), 0, s, x, b, lg, c0, c1);
    else
      hipLaunchKernelGGL((k_rb_first<T, 2, false>), g, dim3(256), 0, s, x, b, lg, c0, c1);
  }
  // algorithmic traffic of the first sweep from zero: b read once, x written once
  if (fine) timer_end(kTimerRbFine, s, 2.0 * (double)Cl * nf * sizeof(T));
}

template <typename T>
void MGHier<T>::vcycle(int nf, const T* b, T* x, double c0, double c1, int nu_pre, int nu_post, int nu_coarse,
                       hipStream_t s) {
  const bool three = dim == 3;
  T cl = (T)c1;
  const T tc0 = (T)c0;
  const int nml = (int)levels.size();
  for (int l = 0; l < nml; ++l) {
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    T* xl = l == 0 ? x : bufs_x[l];
    const T* bl = l == 0 ? b : bufs_b[l];
    if (nu_pre <= 0)
      launch_fill<T>(xl, Cl * nf, T(0), s);
    else
      rb_first(xl, bl, lg, nf, tc0, cl, l == 0, s);
    for (int sw = 1; sw < nu_pre; ++sw)
      for (int color = 0; color < 2; ++color) rb_half(xl, bl, lg, nf, tc0, cl, color, l == 0, s);
    const int64_t Cc = Cl >> dim;
    if (three)
      hipLaunchKernelGGL((k_resid_restrict<T, 3>), dim3(nblk(Cc / 2), nf), dim3(256), 0, s, xl, bl, bufs_b[l + 1],
                         lg, tc0, cl);
    else
      hipLaunchKernelGGL((k_resid_restrict<T, 2>), dim3(nblk(Cc / 2), nf), dim3(256), 0, s, xl, bl, bufs_b[l + 1],
                         lg, tc0, cl);
    cl = cl * T(0.25);
  }
  {
    const T* bl = nml == 0 ? b : bufs_b[nml];
    T* xl = nml == 0 ? x : bufs_x[nml];
    if (three)
      hipLaunchKernelGGL((k_vcycle_lds<T, 3>), dim3(nf), dim3(kLdsThreads), 0, s, bl, xl, tail_b, lds_logn, tc0, cl,
                         nu_pre, nu_post, nu_coarse);
    else
      hipLaunchKernelGGL((k_vcycle_lds<T, 2>), dim3(nf), dim3(kLdsThreads), 0, s, bl, xl, tail_b, lds_logn, tc0, cl,
                         nu_pre, nu_post, nu_coarse);
  }
  for (int l = nml - 1; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    T* xl = l == 0 ? x : bufs_x[l];
    const T* bl = l == 0 ? b : bufs_b[l];
    if (three)
      hipLaunchKernelGGL((k_prolong_add<T, 3>), dim3(nblk(Cl / 4), nf), dim3(256), 0, s, xl, bufs_x[l + 1], lg);
    else
      hipLaunchKernelGGL((k_prolong_add<T, 2>), dim3(nblk(Cl / 4), nf), dim3(256), 0, s, xl, bufs_x[l + 1], lg);
    for (int sw = 0; sw < nu_post; ++sw)
      for (int color = 0; color < 2; ++color) rb_half(xl, bl, lg, nf, tc0, cl, color, l == 0, s);
  }
}

template struct MGHier<double>;
template struct MGHier<float>;

}  // namespace ibr
