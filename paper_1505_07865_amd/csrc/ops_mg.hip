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
// Every level stores its fields split by colour (red half, black half; see
// the split storage section).  Fine levels run one kernel per step with
// nfields batched in blockIdx.y.
// The coarse tail of the cycle runs inside ONE workgroup per field
// (k_vcycle_lds), on the same split storage and the same per-group code as
// the global levels, with every array of the tail levels in LDS: one launch
// instead of ~10 per level.  The tail starts at 4096 cells (16^3, 64^2).
#include "kernels.h"

namespace ibr {

namespace {

constexpr int kLdsThreads = 512;

// Largest level (cells) the one-workgroup tail starts from.  A 32^3 fp32
// pyramid would fit in LDS too, but one compute unit sweeping it is slower
// than the launches it saves.
constexpr int64_t kTailMaxCells = 4096;
// Levels above the tail whose fields (cells x fields) number at most this
// many run the fused LDS-tiled kernels in 3D: there the chain of small
// dependent launches costs more than one workgroup per tile doing a whole
// smoothing phase; on larger levels the per-step kernels stream HBM faster.
constexpr int64_t kFusedMaxWork = (int64_t)1 << 18;

template <typename T>
bool may_fuse(int dim, int lg) {
  return dim == 3 && lg >= 4 && ((int64_t)1 << (dim * lg)) <= kFusedMaxWork;
}
// Cells of all levels from C down to the 4^dim grid.
template <int DIM>
constexpr int64_t pyramid_cells(int64_t C) {
  int64_t t = 0;
  for (int64_t c = C; c >= (DIM == 3 ? 64 : 16); c >>= DIM) t += c;
  return t;
}

// ---------------------------------------------------------------- helpers
// Indices inside one field are 32-bit (n^dim <= 2^27 for the grids accepted);
// field offsets are applied to the base pointers in 64-bit.
__device__ inline int flat_thread(unsigned nblocks) {
  return (int)xcd_block(nblocks) * (int)blockDim.x + (int)threadIdx.x;
}

// ---------------------------------------------------------------- split (red/black) storage
// Every multigrid level stores each field as two halves: the red cells
// (i+j+k even) first, then the black cells, each half row-major over
// (row = j + k n, i >> 1).  A half sweep then streams exactly the cells it
// needs (one colour of x, the other colour's neighbours, one colour of b),
// with 4-wide vector loads of consecutive same-colour cells.
//   storage index = colour * C/2 + (row << (logn-1)) + (i >> 1)
// In a row of parity q = (j+k) & 1 the cell of colour c with half-row index
// m sits at i = 2m + ((c + q) & 1); its x-neighbours have the other colour
// (indices m-1, m if c+q is even, m, m+1 otherwise) and its y/z neighbours
// have the other colour at the same m.
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T v[4];
};
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T v[2];
};

template <typename T>
__device__ inline Quad<T> ldq(const T* p) {
  return *reinterpret_cast<const Quad<T>*>(p);
}
template <typename T>
__device__ inline void stq(T* p, const Quad<T>& q) {
  *reinterpret_cast<Quad<T>*>(p) = q;
}

// ---- per-group building blocks on one field (x, b already at that field) ----
// The global kernels below run one group per thread; the one-workgroup tail
// loops over the groups of a level with its 1024 threads.

// Half sweep of the 4 consecutive cells of colour `color` in group g of a row
// (H/4 groups).  Needs n >= 8.
template <typename T, int DIM>
__device__ inline void rb_group(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1, int color,
                                int g) {
  const int C = 1 << (DIM * logn);
  const int H = C >> 1;
  const int hl = logn - 1;  // log2 of the half-row length
  const int mask = (1 << logn) - 1, hmask = (1 << hl) - 1;
  const int m0 = (g & ((1 << (hl - 2)) - 1)) << 2;
  const int row = g >> (hl - 2);
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const bool odd = ((color + j + k) & 1) != 0;  // own cells at i = 2m + 1
  T* own = x + color * H;
  const T* oth = x + (1 - color) * H;
  const Quad<T> o = ldq(oth + (row << hl) + m0);
  const T ext = oth[(row << hl) + ((odd ? m0 + 4 : m0 - 1) & hmask)];
  const int ry0 = ((j - 1) & mask) | (k << logn), ry1 = ((j + 1) & mask) | (k << logn);
  const Quad<T> ym = ldq(oth + (ry0 << hl) + m0);
  const Quad<T> yp = ldq(oth + (ry1 << hl) + m0);
  Quad<T> zm, zp;
  if (DIM == 3) {
    const int rz0 = j | (((k - 1) & mask) << logn), rz1 = j | (((k + 1) & mask) << logn);
    zm = ldq(oth + (rz0 << hl) + m0);
    zp = ldq(oth + (rz1 << hl) + m0);
  }
  const Quad<T> bc = ldq(b + color * H + (row << hl) + m0);
  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  Quad<T> out;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const T xl = odd ? o.v[u] : (u == 0 ? ext : o.v[u - 1]);
    const T xr = odd ? (u == 3 ? ext : o.v[u + 1]) : o.v[u];
    T sum = xl + xr + ym.v[u] + yp.v[u];
    if (DIM == 3) sum += zm.v[u] + zp.v[u];
    out.v[u] = (bc.v[u] + c1 * sum) * inv_diag;
  }
  stq(own + (row << hl) + m0, out);
}

// The first red-black sweep from a zero guess in one pass: red cells take
// b/diag, black cells (all of whose neighbours are red) take
// (b + c1 * sum of the neighbours' b/diag)/diag.  Same arithmetic, in the same
// order, as a red then a black half sweep from x = 0.  Group g writes 4 red
// and 4 black cells of one row (H/4 groups).  Needs n >= 8.
template <typename T, int DIM>
__device__ inline void rb_first_group(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1, int g) {
  const int C = 1 << (DIM * logn);
  const int H = C >> 1;
  const int hl = logn - 1;
  const int mask = (1 << logn) - 1, hmask = (1 << hl) - 1;
  const int m0 = (g & ((1 << (hl - 2)) - 1)) << 2;
  const int row = g >> (hl - 2);
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const bool odd = ((1 + j + k) & 1) != 0;  // black cells at i = 2m + 1
  const T* bred = b;
  const T* bblk = b + H;
  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  const Quad<T> rr = ldq(bred + (row << hl) + m0);
  Quad<T> xr;
#pragma unroll
  for (int u = 0; u < 4; ++u) xr.v[u] = rr.v[u] * inv_diag;
  stq(x + (row << hl) + m0, xr);
  const T ext = bred[(row << hl) + ((odd ? m0 + 4 : m0 - 1) & hmask)];
  const int ry0 = ((j - 1) & mask) | (k << logn), ry1 = ((j + 1) & mask) | (k << logn);
  const Quad<T> ym = ldq(bred + (ry0 << hl) + m0);
  const Quad<T> yp = ldq(bred + (ry1 << hl) + m0);
  Quad<T> zm, zp;
  if (DIM == 3) {
    const int rz0 = j | (((k - 1) & mask) << logn), rz1 = j | (((k + 1) & mask) << logn);
    zm = ldq(bred + (rz0 << hl) + m0);
    zp = ldq(bred + (rz1 << hl) + m0);
  }
  const Quad<T> bb = ldq(bblk + (row << hl) + m0);
  Quad<T> xb;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const T xl = odd ? rr.v[u] : (u == 0 ? ext : rr.v[u - 1]);
    const T xrr = odd ? (u == 3 ? ext : rr.v[u + 1]) : rr.v[u];
    T sum = xl * inv_diag + xrr * inv_diag + ym.v[u] * inv_diag + yp.v[u] * inv_diag;
    if (DIM == 3) sum += zm.v[u] * inv_diag + zp.v[u] * inv_diag;
    xb.v[u] = (bb.v[u] + c1 * sum) * inv_diag;
  }
  stq(x + H + (row << hl) + m0, xb);
}

// Coarse right-hand side = average over the 2^dim children of the residual
// r = b - (diag x - c1 sum_nbr x).  Summed over a 2^dim block, each child's
// neighbour along each axis inside the block is a sibling, so
//   sum r = sum b - (diag - dim c1) sum x + c1 (sum of the face neighbours
//           outside the block).
// Group g makes 4 consecutive coarse cells of one coarse row (Cc/4 groups):
// in fine row (2J+dj, 2K+dk) the children 2I and 2I+1 are the two colours at
// half-row index I.  bc is the coarse field.  Needs n >= 8.
template <typename T, int DIM>
__device__ inline void restrict_group(const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ bc, int logn,
                                      T c0, T c1, int g) {
  const int lognc = logn - 1;
  const int C = 1 << (DIM * logn), H = C >> 1, hl = logn - 1;
  const int Cc = 1 << (DIM * lognc), Hc = Cc >> 1, hlc = lognc - 1;
  const int mask = (1 << logn) - 1, hmask = (1 << hl) - 1, maskc = (1 << lognc) - 1;
  const int qlog = lognc - 2;  // 4-cell groups per coarse row
  const int I0 = (g & ((1 << qlog) - 1)) << 2;
  const int rowc = g >> qlog;
  const int J = rowc & maskc;
  const int K = DIM == 3 ? (rowc >> lognc) : 0;
  T sx[4] = {0, 0, 0, 0}, sb[4] = {0, 0, 0, 0}, sf[4] = {0, 0, 0, 0};
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int row = ((2 * J + dy) & mask) | (((2 * K + dz) & mask) << logn);
      const int ev = (dy + dz) & 1;  // colour of the even children 2I
      const T* xe = x + ev * H + (row << hl);
      const T* xo = x + (1 - ev) * H + (row << hl);
      const Quad<T> A = ldq(xe + I0), B = ldq(xo + I0);
      const Quad<T> bA = ldq(b + ev * H + (row << hl) + I0), bB = ldq(b + (1 - ev) * H + (row << hl) + I0);
      const T left = xo[(I0 - 1) & hmask];   // fine 2 I0 - 1: odd child of coarse I0 - 1
      const T right = xe[(I0 + 4) & hmask];  // fine 2 I0 + 8: even child of coarse I0 + 4
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sx[u] += A.v[u] + B.v[u];
        sb[u] += bA.v[u] + bB.v[u];
        sf[u] += (u == 0 ? left : B.v[u - 1]) + (u == 3 ? right : A.v[u + 1]);
      }
    }
  // y faces: fine rows 2J-1 and 2J+2 (both children of every coarse cell)
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int y = e == 0 ? 2 * J - 1 : 2 * J + 2;
      const int row = (y & mask) | (((2 * K + dz) & mask) << logn);
      const Quad<T> P = ldq(x + (row << hl) + I0), Q = ldq(x + H + (row << hl) + I0);
#pragma unroll
      for (int u = 0; u < 4; ++u) sf[u] += P.v[u] + Q.v[u];
    }
  if (DIM == 3) {
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int z = e == 0 ? 2 * K - 1 : 2 * K + 2;
        const int row = ((2 * J + dy) & mask) | ((z & mask) << logn);
        const Quad<T> P = ldq(x + (row << hl) + I0), Q = ldq(x + H + (row << hl) + I0);
#pragma unroll
        for (int u = 0; u < 4; ++u) sf[u] += P.v[u] + Q.v[u];
      }
  }
  const T diag = c0 + T(2 * DIM) * c1;
  const T inner = diag - T(DIM) * c1;
  const T avg = DIM == 3 ? T(0.125) : T(0.25);
  T r[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) r[u] = (sb[u] - inner * sx[u] + c1 * sf[u]) * avg;
  // coarse cells I0, I0+2 have colour cp, I0+1, I0+3 the other, at half-row I0/2, I0/2+1
  const int cp = (J + K) & 1;
  const int o = (rowc << hlc) + (I0 >> 1);
  *reinterpret_cast<Pair<T>*>(bc + cp * Hc + o) = Pair<T>{{r[0], r[2]}};
  *reinterpret_cast<Pair<T>*>(bc + (1 - cp) * Hc + o) = Pair<T>{{r[1], r[3]}};
}

// x += P e (multilinear, cell-centred: weights 3/4 and 1/4 per axis).  Group
// g owns 8 consecutive fine cells of a row (4 of each colour; C/8 groups);
// each of the 2^(dim-1) coarse rows it needs is interpolated along x once
// from coarse cells I0-1 .. I0+4 (two pairs and two scalars).  BLACK_ONLY:
// only the black cells are corrected, for when a red half sweep follows (it
// overwrites the red cells without reading them), which leaves the result
// unchanged and halves the traffic.  Needs n >= 8.
template <typename T, int DIM, bool BLACK_ONLY>
__device__ inline void prolong_group(T* __restrict__ x, const T* __restrict__ e, int logn, int g) {
  const int C = 1 << (DIM * logn), H = C >> 1, hl = logn - 1;
  const int lognc = logn - 1;
  const int Cc = 1 << (DIM * lognc), Hc = Cc >> 1, hlc = lognc - 1;
  const int mask = (1 << logn) - 1, maskc = (1 << lognc) - 1, hmaskc = (1 << hlc) - 1;
  const int glog = logn - 3;  // 8-cell groups per fine row
  const int gi = g & ((1 << glog) - 1);
  const int row = g >> glog;
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const int J = j >> 1, K = k >> 1;
  const int sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
  const int I0 = gi << 2;     // first coarse cell; fine cells 2 I0 .. 2 I0 + 7
  const int mc = I0 >> 1;     // its half-row index
  const T w0 = T(0.75), w1 = T(0.25);
  T a[4][8];  // [coarse row: (J,K), (J+sj,K), (J,K+sk), (J+sj,K+sk)][fine cell]
#pragma unroll
  for (int r = 0; r < (DIM == 3 ? 4 : 2); ++r) {
    const int Jr = (J + ((r & 1) ? sj : 0)) & maskc, Kr = (K + ((r & 2) ? sk : 0)) & maskc;
    const int rowc = Jr | (Kr << lognc);
    const int cq = (Jr + Kr) & 1;  // colour of the even coarse cells I0, I0+2
    const T* ee = e + cq * Hc + (rowc << hlc);
    const T* eo = e + (1 - cq) * Hc + (rowc << hlc);
    const Pair<T> pe = *reinterpret_cast<const Pair<T>*>(ee + mc);
    const Pair<T> po = *reinterpret_cast<const Pair<T>*>(eo + mc);
    T E[6];  // coarse I0-1 .. I0+4
    E[0] = eo[(mc - 1) & hmaskc];
    E[1] = pe.v[0];
    E[2] = po.v[0];
    E[3] = pe.v[1];
    E[4] = po.v[1];
    E[5] = ee[(mc + 2) & hmaskc];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int ci = 1 + (v >> 1);  // position of coarse I in E
      a[r][v] = w0 * E[ci] + w1 * ((v & 1) ? E[ci + 1] : E[ci - 1]);
    }
  }
  // fine cells 2 I0 + v: colour fp for even v, the other for odd v; half-row index I0 + v/2
  const int fp = (j + k) & 1;
  T* xe = x + fp * H + (row << hl) + I0;
  T* xo = x + (1 - fp) * H + (row << hl) + I0;
  const bool even_black = fp == 1;  // black is colour 1
  Quad<T> qe, qo;
  if (!BLACK_ONLY || even_black) qe = ldq(xe);
  if (!BLACK_ONLY || !even_black) qo = ldq(xo);
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    T val;
    if (DIM == 3) {
      const T b0 = w0 * a[0][v] + w1 * a[1][v];
      const T b1 = w0 * a[2][v] + w1 * a[3][v];
      val = w0 * b0 + w1 * b1;
    } else {
      val = w0 * a[0][v] + w1 * a[1][v];
    }
    if (v & 1)
      qo.v[v >> 1] += val;
    else
      qe.v[v >> 1] += val;
  }
  if (!BLACK_ONLY || even_black) stq(xe, qe);
  if (!BLACK_ONLY || !even_black) stq(xo, qo);
}

// Coarse cells m0-1 .. m0+4 of coarse row (Jr, Kr) (wrapped), m0 a multiple
// of 4: the x-range that the fine cells 2 m0 - 1 .. 2 m0 + 8 interpolate from
// (as prolong_group loads them).
template <typename T, int DIM>
__device__ inline void coarse_row6(const T* __restrict__ e, int lognc, int Jr, int Kr, int m0, T E[6]) {
  const int Cc = 1 << (DIM * lognc), Hc = Cc >> 1, hlc = lognc - 1;
  const int maskc = (1 << lognc) - 1, hmaskc = (1 << hlc) - 1;
  Jr &= maskc;
  Kr = DIM == 3 ? (Kr & maskc) : 0;
  const int rowc = Jr | (Kr << lognc);
  const int cq = (Jr + Kr) & 1;  // colour of the even coarse cells
  const T* ee = e + cq * Hc + (rowc << hlc);
  const T* eo = e + (1 - cq) * Hc + (rowc << hlc);
  const int mc = m0 >> 1;
  const Pair<T> pe = *reinterpret_cast<const Pair<T>*>(ee + mc);
  const Pair<T> po = *reinterpret_cast<const Pair<T>*>(eo + mc);
  E[0] = eo[(mc - 1) & hmaskc];
  E[1] = pe.v[0];
  E[2] = po.v[0];
  E[3] = pe.v[1];
  E[4] = po.v[1];
  E[5] = ee[(mc + 2) & hmaskc];
}

// The first red half sweep after prolongation, with the prolongation folded
// in.  Post-smoothing corrects only the black cells (the red half sweep
// overwrites the red ones without reading them), and the black half sweep
// that follows overwrites the black ones from their red neighbours alone: so
// the corrected black values are read only here.  This red half sweep takes
// each black neighbour as x + P e, forming P e from the coarse e with the
// interpolation of prolong_group (per coarse row along x, then y, then z,
// weights 3/4 and 1/4), and leaves the black cells as they are.  The red cells
// of group g (rows (j, k)) read black cells in 5 fine rows, whose corrections
// come from 8 coarse rows in 3D (3 in 2D): Y in {J, J+sj, J-sj} x Z in
// {K, K+sk, K-sk}, sj and sk the side of the fine row within its coarse cell.
template <typename T, int DIM>
__device__ inline void rb_red_prolong_group(T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ e,
                                            int logn, T c0, T c1, int g) {
  const int C = 1 << (DIM * logn);
  const int H = C >> 1;
  const int hl = logn - 1;
  const int mask = (1 << logn) - 1, hmask = (1 << hl) - 1;
  const int m0 = (g & ((1 << (hl - 2)) - 1)) << 2;
  const int row = g >> (hl - 2);
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const bool odd = ((j + k) & 1) != 0;  // red cells at i = 2m + 1 (black at 2m), else the other way
  const T* oth = x + H;
  Quad<T> o = ldq(oth + (row << hl) + m0);
  T ext = oth[(row << hl) + ((odd ? m0 + 4 : m0 - 1) & hmask)];
  const int ry0 = ((j - 1) & mask) | (k << logn), ry1 = ((j + 1) & mask) | (k << logn);
  Quad<T> ym = ldq(oth + (ry0 << hl) + m0);
  Quad<T> yp = ldq(oth + (ry1 << hl) + m0);
  Quad<T> zm, zp;
  if (DIM == 3) {
    const int rz0 = j | (((k - 1) & mask) << logn), rz1 = j | (((k + 1) & mask) << logn);
    zm = ldq(oth + (rz0 << hl) + m0);
    zp = ldq(oth + (rz1 << hl) + m0);
  }
  const Quad<T> bc = ldq(b + (row << hl) + m0);

  // Coarse rows by (Y, Z) offset from the fine row's own coarse cell (J, K):
  // r0 (0,0), r1 (sj,0), r2 (0,sk), r3 (sj,sk), r4 (-sj,0), r5 (-sj,sk),
  // r6 (0,-sk), r7 (sj,-sk) (2D: r0, r1, r4).  Each fine row combines 4 of
  // them as prolong_group does, b0 = w0 a(near Y) + w1 a(far Y) in its own Z
  // row, b1 likewise in the other Z row, P e = w0 b0 + w1 b1:
  //   own row (j, k): r0 r1 | r2 r3      far y row (j+sj): r1 r0 | r3 r2
  //   near y row (j-sj): r0 r4 | r2 r5   far z row (k+sk): r2 r3 | r0 r1
  //   near z row (k-sk): r0 r1 | r6 r7
  // The rows come in pairs and each combination is finished as soon as its
  // rows are in, so only a few partial sums stay live.  a = the x-interpolation
  // of one coarse row at the 4 black cells of the fine row (parity pb0 for the
  // own row, the other parity for the 4 neighbour rows); both parities are
  // formed and chosen by value (a choice between array elements would keep
  // the row in memory).
  const int lognc = logn - 1;
  const int J = j >> 1, K = k >> 1;
  const int sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
  const T w0 = T(0.75), w1 = T(0.25);
  const bool pb0 = !odd;  // black cells of the own row at fine x = 2m + pb0
  // own-parity (q) and neighbour-parity (p) interpolations of a coarse row,
  // and the own row's cell beyond the group (xg)
  auto lerps = [&](int dy, int dz, Quad<T>& q, Quad<T>& p, T& xg) {
    T E[6];
    coarse_row6<T, DIM>(e, lognc, J + dy, K + dz, m0, E);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T lo = w0 * E[1 + u] + w1 * E[u];
      const T hi = w0 * E[1 + u] + w1 * E[2 + u];
      q.v[u] = pb0 ? hi : lo;
      p.v[u] = pb0 ? lo : hi;
    }
    const T xo = w0 * E[0] + w1 * E[1];  // coarse m0-1 (odd fine x)
    const T xe = w0 * E[5] + w1 * E[4];  // coarse m0+4 (even fine x)
    xg = pb0 ? xo : xe;
  };
  Quad<T> q0, p0, q1, p1, own_b0, yfar_b0, zfar_b1;
  T x0, x1, xg_b0;
  lerps(0, 0, q0, p0, x0);
  lerps(sj, 0, q1, p1, x1);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    own_b0.v[u] = w0 * q0.v[u] + w1 * q1.v[u];
    yfar_b0.v[u] = w0 * p1.v[u] + w1 * p0.v[u];
    zfar_b1.v[u] = w0 * p0.v[u] + w1 * p1.v[u];  // also the near z row's b0
  }
  xg_b0 = w0 * x0 + w1 * x1;
  if constexpr (DIM == 3) {
    Quad<T> q2, p2, q3, p3;
    T x2, x3;
    lerps(0, sk, q2, p2, x2);
    lerps(sj, sk, q3, p3, x3);
    Quad<T> yfar, zfar;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T own_b1 = w0 * q2.v[u] + w1 * q3.v[u];
      o.v[u] += w0 * own_b0.v[u] + w1 * own_b1;
      const T yfar_b1 = w0 * p3.v[u] + w1 * p2.v[u];
      yfar.v[u] = w0 * yfar_b0.v[u] + w1 * yfar_b1;
      const T zfar_b0 = w0 * p2.v[u] + w1 * p3.v[u];
      zfar.v[u] = w0 * zfar_b0 + w1 * zfar_b1.v[u];
    }
    ext += w0 * xg_b0 + w1 * (w0 * x2 + w1 * x3);
    Quad<T> q4, p4, q5, p5, ynear;
    T x4, x5;
    lerps(-sj, 0, q4, p4, x4);
    lerps(-sj, sk, q5, p5, x5);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T b0 = w0 * p0.v[u] + w1 * p4.v[u];
      const T b1 = w0 * p2.v[u] + w1 * p5.v[u];
      ynear.v[u] = w0 * b0 + w1 * b1;
    }
    Quad<T> q6, p6, q7, p7;
    T x6, x7;
    lerps(0, -sk, q6, p6, x6);
    lerps(sj, -sk, q7, p7, x7);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T b1 = w0 * p6.v[u] + w1 * p7.v[u];
      const T znear = w0 * zfar_b1.v[u] + w1 * b1;
      ym.v[u] += sj < 0 ? yfar.v[u] : ynear.v[u];
      yp.v[u] += sj < 0 ? ynear.v[u] : yfar.v[u];
      zm.v[u] += sk < 0 ? zfar.v[u] : znear;
      zp.v[u] += sk < 0 ? znear : zfar.v[u];
    }
  } else {
    Quad<T> q4, p4;
    T x4;
    lerps(-sj, 0, q4, p4, x4);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      o.v[u] += own_b0.v[u];
      const T ynear = w0 * p0.v[u] + w1 * p4.v[u];
      ym.v[u] += sj < 0 ? yfar_b0.v[u] : ynear;
      yp.v[u] += sj < 0 ? ynear : yfar_b0.v[u];
    }
    ext += xg_b0;
  }

  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  Quad<T> out;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const T xl = odd ? o.v[u] : (u == 0 ? ext : o.v[u - 1]);
    const T xr = odd ? (u == 3 ? ext : o.v[u + 1]) : o.v[u];
    T sum = xl + xr + ym.v[u] + yp.v[u];
    if (DIM == 3) sum += zm.v[u] + zp.v[u];
    out.v[u] = (bc.v[u] + c1 * sum) * inv_diag;
  }
  stq(x + (row << hl) + m0, out);
}

// Half sweep of one cell of colour `color` (t < C/2), for the 4^dim coarsest
// grid, whose half rows (2 cells) are shorter than a 4-cell group.
template <typename T, int DIM>
__device__ inline void rb_cell(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1, int color, int t) {
  const int C = 1 << (DIM * logn);
  const int H = C >> 1;
  const int hl = logn - 1;
  const int mask = (1 << logn) - 1, hmask = (1 << hl) - 1;
  const int m = t & hmask;
  const int row = t >> hl;
  const int j = row & mask;
  const int k = DIM == 3 ? (row >> logn) : 0;
  const int i = 2 * m + ((color + j + k) & 1);
  const T* oth = x + (1 - color) * H;
  const int ry0 = ((j - 1) & mask) | (k << logn), ry1 = ((j + 1) & mask) | (k << logn);
  T sum = oth[(row << hl) + (((i - 1) & mask) >> 1)] + oth[(row << hl) + (((i + 1) & mask) >> 1)] +
          oth[(ry0 << hl) + m] + oth[(ry1 << hl) + m];
  if (DIM == 3) {
    const int rz0 = j | (((k - 1) & mask) << logn), rz1 = j | (((k + 1) & mask) << logn);
    sum += oth[(rz0 << hl) + m] + oth[(rz1 << hl) + m];
  }
  const T inv_diag = T(1) / (c0 + T(2 * DIM) * c1);
  x[color * H + (row << hl) + m] = (b[color * H + (row << hl) + m] + c1 * sum) * inv_diag;
}

// ---------------------------------------------------------------- level kernels
// One group per thread, nfields batched in blockIdx.y.  FINE marks the finest
// level (same code; a separate symbol for profiling).
template <typename T, int DIM, bool FINE>
__global__ void __launch_bounds__(256) k_rb(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1,
                                            int color) {
  const int C = 1 << (DIM * logn);
  const int g = flat_thread(gridDim.x);
  if (g >= (C >> 3)) return;
  const int64_t f = blockIdx.y;
  rb_group<T, DIM>(x + f * C, b + f * C, logn, c0, c1, color, g);
}

template <typename T, int DIM, bool FINE>
__global__ void __launch_bounds__(256) k_rb_first(T* __restrict__ x, const T* __restrict__ b, int logn, T c0,
                                                  T c1) {
  const int C = 1 << (DIM * logn);
  const int g = flat_thread(gridDim.x);
  if (g >= (C >> 3)) return;
  const int64_t f = blockIdx.y;
  rb_first_group<T, DIM>(x + f * C, b + f * C, logn, c0, c1, g);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_resid_restrict(const T* __restrict__ x, const T* __restrict__ b,
                                                        T* __restrict__ bc, int logn, T c0, T c1) {
  const int C = 1 << (DIM * logn);
  const int Cc = C >> DIM;
  const int g = flat_thread(gridDim.x);
  if (g >= (Cc >> 2)) return;
  const int64_t f = blockIdx.y;
  restrict_group<T, DIM>(x + f * C, b + f * C, bc + f * Cc, logn, c0, c1, g);
}

template <typename T, int DIM, bool BLACK_ONLY>
__global__ void __launch_bounds__(256) k_prolong_add(T* __restrict__ x, const T* __restrict__ e, int logn) {
  const int C = 1 << (DIM * logn);
  const int Cc = C >> DIM;
  const int g = flat_thread(gridDim.x);
  if (g >= (C >> 3)) return;
  const int64_t f = blockIdx.y;
  prolong_group<T, DIM, BLACK_ONLY>(x + f * C, e + f * Cc, logn, g);
}

// Post-smoothing's first red half sweep with the black cells' prolongation
// folded in (rb_red_prolong_group); FINE marks the finest level.
template <typename T, int DIM, bool FINE>
__global__ void __launch_bounds__(256) k_rb_red_prolong(T* __restrict__ x, const T* __restrict__ b,
                                                        const T* __restrict__ e, int logn, T c0, T c1) {
  const int C = 1 << (DIM * logn);
  const int Cc = C >> DIM;
  const int g = flat_thread(gridDim.x);
  if (g >= (C >> 3)) return;
  const int64_t f = blockIdx.y;
  rb_red_prolong_group<T, DIM>(x + f * C, b + f * C, e + f * Cc, logn, c0, c1, g);
}

// ---------------------------------------------------------------- one-workgroup tail
// Tail levels of at most this many cells run in wavefront 0 alone (at most
// two items per lane and phase, 3D 8^3 and 2D 32^2 down): each phase then
// ends with a wavefront-level ordering instead of a workgroup barrier, whose
// cost dominates phases that small.
constexpr int kWaveCells = 1024;

// One level's pre-smoothing from zero and restriction of its residual into
// the next level's b.  Items t = i0, i0 + st, ...; sync() ends each phase.
template <typename T, int DIM, typename Sync>
__device__ inline void tail_pre(T* x, const T* b, T* bc, int lg, T c0, T cl, int nu_pre, int i0, int st, Sync sync) {
  const int Cl = 1 << (DIM * lg);
  if (nu_pre > 0) {
    for (int g = i0; g < (Cl >> 3); g += st) rb_first_group<T, DIM>(x, b, lg, c0, cl, g);
    sync();
    for (int sw = 1; sw < nu_pre; ++sw)
      for (int color = 0; color < 2; ++color) {
        for (int g = i0; g < (Cl >> 3); g += st) rb_group<T, DIM>(x, b, lg, c0, cl, color, g);
        sync();
      }
  } else {
    for (int c = i0; c < Cl; c += st) x[c] = T(0);
    sync();
  }
  for (int g = i0; g < ((Cl >> DIM) >> 2); g += st) restrict_group<T, DIM>(x, b, bc, lg, c0, cl, g);
  sync();
}

// One level's prolongation of the coarse correction xc and post-smoothing.
template <typename T, int DIM, typename Sync>
__device__ inline void tail_post(T* x, const T* xc, const T* b, int lg, T c0, T cl, int nu_post, int i0, int st,
                                 Sync sync) {
  const int Cl = 1 << (DIM * lg);
  if (nu_post > 0) {
    for (int g = i0; g < (Cl >> 3); g += st) prolong_group<T, DIM, true>(x, xc, lg, g);
  } else {
    for (int g = i0; g < (Cl >> 3); g += st) prolong_group<T, DIM, false>(x, xc, lg, g);
  }
  sync();
  for (int sw = 0; sw < nu_post; ++sw)
    for (int color = 0; color < 2; ++color) {
      for (int g = i0; g < (Cl >> 3); g += st) rb_group<T, DIM>(x, b, lg, c0, cl, color, g);
      sync();
    }
}

// V-cycle from the tail's entry level down to n = 4, one field per workgroup
// of kLdsThreads threads, on split storage like the global levels: the
// iterates of every tail level and the right-hand sides below the entry level
// live in LDS; the entry level's right-hand side is read from global memory.
// Levels above kWaveCells cells use the whole workgroup, the smaller ones
// wavefront 0 (the others wait at the workgroup barrier after them).  c1 is
// the coefficient at the entry level; level l uses c1 / 4^l (exact).
template <typename T, int DIM>
__global__ void __launch_bounds__(kLdsThreads) k_vcycle_lds(const T* __restrict__ bg, T* __restrict__ xg, int logn,
                                                            T c0, T c1, int nu_pre, int nu_post, int nu_coarse) {
  constexpr int kX = (int)pyramid_cells<DIM>(kTailMaxCells) + 64;
  constexpr int kB = (int)pyramid_cells<DIM>(kTailMaxCells >> DIM) + 64;
  __shared__ Quad<T> xs4[kX / 4];  // x of every level back to back, entry level first
  __shared__ Quad<T> bs4[kB / 4];  // b of the levels below the entry level
  T* xs = &xs4[0].v[0];
  T* bs = &bs4[0].v[0];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int C0 = 1 << (DIM * logn);
  const T* b0 = bg + (int64_t)blockIdx.x * C0;
  T* x0 = xg + (int64_t)blockIdx.x * C0;
  const bool singular = c0 == T(0);

  const int nlev = logn - 1;  // entry level down to n = 4
  int off[10];
  T* bl[10];
  {
    int xo = 0, bo = 0;
    for (int l = 0; l < nlev; ++l) {
      const int Cl = 1 << (DIM * (logn - l));
      off[l] = xo;
      xo += Cl;
      bl[l] = nullptr;
      if (l == 0 && nlev > 1) continue;  // the entry level reads b0
      bl[l] = bs + bo;
      bo += Cl;
    }
  }
  if (nlev == 1) {
    // the whole cycle is the coarsest grid: its b is modified (mean removal), take a copy
    for (int c = tid; c < C0; c += nt) bl[0][c] = b0[c];
    __syncthreads();
  }
  auto level_b = [&](int l) -> const T* { return l == 0 ? b0 : bl[l]; };
  auto coef = [&](int l) { return c1 / T(1 << (2 * l)); };
  auto block_sync = [] { __syncthreads(); };
  auto wsync = [] { wave_sync(); };

  // first level small enough for one wavefront (the coarsest always is)
  int lw = 0;
  while (lw < nlev - 1 && (1 << (DIM * (logn - lw))) > kWaveCells) ++lw;
  for (int l = 0; l < lw; ++l)
    tail_pre<T, DIM>(xs + off[l], level_b(l), bl[l + 1], logn - l, c0, coef(l), nu_pre, tid, nt, block_sync);
  if (tid < kWave) {
    const int lane = tid;
    for (int l = lw; l < nlev - 1; ++l)
      tail_pre<T, DIM>(xs + off[l], level_b(l), bl[l + 1], logn - l, c0, coef(l), nu_pre, lane, kWave, wsync);
    {
      // coarsest grid (n = 4): nu_coarse sweeps from zero
      const int l = nlev - 1;
      const int lg = logn - l;
      const int Cl = 1 << (DIM * lg);
      const T cl = coef(l);
      T* x = xs + off[l];
      T* b = bl[l];
      if (singular) {
        T sm = 0;
        for (int c = lane; c < Cl; c += kWave) sm += b[c];
        const T m = wave_sum(sm) / T(Cl);
        for (int c = lane; c < Cl; c += kWave) b[c] -= m;
      }
      for (int c = lane; c < Cl; c += kWave) x[c] = T(0);
      wsync();
      for (int sw = 0; sw < nu_coarse; ++sw)
        for (int color = 0; color < 2; ++color) {
          for (int t = lane; t < (Cl >> 1); t += kWave) rb_cell<T, DIM>(x, b, lg, c0, cl, color, t);
          wsync();
        }
    }
    for (int l = nlev - 2; l >= lw; --l)
      tail_post<T, DIM>(xs + off[l], xs + off[l + 1], level_b(l), logn - l, c0, coef(l), nu_post, lane, kWave,
                        wsync);
  }
  __syncthreads();
  for (int l = lw - 1; l >= 0; --l)
    tail_post<T, DIM>(xs + off[l], xs + off[l + 1], level_b(l), logn - l, c0, coef(l), nu_post, tid, nt,
                      block_sync);
  for (int q = tid; q < (C0 >> 2); q += nt) stq(x0 + 4 * q, ldq(xs + 4 * q));
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
void MGHier<T>::init(int dim_, int logn_, int maxf, int wall_mask_) {
  dim = dim_;
  wall_mask = wall_mask_;
  logn = logn_;
  nfmax = maxf;
  levels.clear();
  // multi-kernel levels: while the level has more cells than the tail starts from
  int lg = logn;
  while (((int64_t)1 << (dim * lg)) > kTailMaxCells) {
    levels.push_back(lg);
    --lg;
  }
  lds_logn = lg;
  bufs_x.assign(levels.size() + 1, nullptr);
  bufs_b.assign(levels.size() + 1, nullptr);
  bufs_xo.assign(levels.size() + 1, nullptr);
  for (size_t l = 1; l <= levels.size(); ++l) {
    const int lgl = logn - (int)l;
    const int64_t Cl = (int64_t)1 << (dim * lgl);
    bufs_x[l] = dev_alloc<T>(Cl * nfmax);
    bufs_b[l] = dev_alloc<T>(Cl * nfmax);
    if (l < levels.size() && may_fuse<T>(dim, lgl)) bufs_xo[l] = dev_alloc<T>(Cl * nfmax);
  }
  x0_tmp = (!levels.empty() && may_fuse<T>(dim, logn)) ? dev_alloc<T>(((int64_t)1 << (dim * logn)) * nfmax) : nullptr;
  wall_x.assign(logn > 2 ? logn - 1 : 1, nullptr);
  wall_b.assign(logn > 2 ? logn - 1 : 1, nullptr);
  if (wall_mask)
    for (int l = 1; l <= logn - 2; ++l) {
      const int64_t Cl = (int64_t)1 << (dim * (logn - l));
      wall_x[l] = dev_alloc<T>(Cl * nfmax);
      wall_b[l] = dev_alloc<T>(Cl * nfmax);
    }
}

template <typename T>
bool MGHier<T>::fused(int lg, int nu, int nf) const {
  return may_fuse<T>(dim, lg) && fused_level_ok(dim, lg, nu) && ((int64_t)nf << (dim * lg)) <= kFusedMaxWork;
}

template <typename T>
void MGHier<T>::release() {
  for (auto p : bufs_x) dev_free(p);
  for (auto p : bufs_b) dev_free(p);
  for (auto p : bufs_xo) dev_free(p);
  dev_free(x0_tmp);
  x0_tmp = nullptr;
  for (auto p : wall_x) dev_free(p);
  for (auto p : wall_b) dev_free(p);
  wall_x.clear();
  wall_b.clear();
  bufs_x.clear();
  bufs_b.clear();
  bufs_xo.clear();
}

template <typename T>
size_t MGHier<T>::bytes(int dim, int logn, int nf, bool walls) {
  size_t tot = 0;
  if (walls)
    for (int l = logn - 1; l >= 2; --l) tot += 2 * ((size_t)1 << (dim * l)) * nf * sizeof(T);
  int lg = logn;
  while (((int64_t)1 << (dim * lg)) > kTailMaxCells) --lg;
  for (int l = logn - 1; l >= lg; --l) tot += 2 * ((size_t)1 << (dim * l)) * nf * sizeof(T);
  for (int l = logn - 1; l > lg; --l)
    if (may_fuse<T>(dim, l)) tot += ((size_t)1 << (dim * l)) * nf * sizeof(T);
  if (logn > lg && may_fuse<T>(dim, logn)) tot += ((size_t)1 << (dim * logn)) * nf * sizeof(T);
  return tot;
}

template <typename T>
void MGHier<T>::rb_half(T* x, const T* b, int lg, int nf, T c0, T c1, int color, bool fine, hipStream_t s) {
  const int64_t Cl = (int64_t)1 << (dim * lg);
  check_quad_aligned(x, b);
  const dim3 gh(nblk(Cl / 8), nf);
  // algorithmic traffic of a half sweep: x of one colour written, x of the other and b of this colour read
  const TimerEvents ev = fine ? timer_sample(kTimerRbFine, 1.5 * (double)Cl * nf * sizeof(T)) : TimerEvents();
  if (dim == 3) {
    if (fine)
      hipExtLaunchKernelGGL(k_rb<T, 3, true>, gh, dim3(256), 0, s, ev.start, ev.stop, 0, x, b, lg, c0, c1, color);
    else
      hipLaunchKernelGGL((k_rb<T, 3, false>), gh, dim3(256), 0, s, x, b, lg, c0, c1, color);
  } else {
    if (fine)
      hipExtLaunchKernelGGL(k_rb<T, 2, true>, gh, dim3(256), 0, s, ev.start, ev.stop, 0, x, b, lg, c0, c1, color);
    else
      hipLaunchKernelGGL((k_rb<T, 2, false>), gh, dim3(256), 0, s, x, b, lg, c0, c1, color);
  }
}

template <typename T>
void MGHier<T>::rb_red_prolong(T* x, const T* b, const T* e, int lg, int nf, T c0, T c1, bool fine,
                               hipStream_t s) {
  const int64_t Cl = (int64_t)1 << (dim * lg);
  check_quad_aligned(x, b);
  const dim3 g(nblk(Cl / 8), nf);
  // algorithmic traffic: a half sweep's plus the coarse correction read once
  const TimerEvents ev =
      fine ? timer_sample(kTimerRbRedProlong, (1.5 + 1.0 / (1 << dim)) * (double)Cl * nf * sizeof(T)) : TimerEvents();
  if (dim == 3) {
    if (fine)
      hipExtLaunchKernelGGL(k_rb_red_prolong<T, 3, true>, g, dim3(256), 0, s, ev.start, ev.stop, 0, x, b, e, lg, c0,
                            c1);
    else
      hipLaunchKernelGGL((k_rb_red_prolong<T, 3, false>), g, dim3(256), 0, s, x, b, e, lg, c0, c1);
  } else {
    if (fine)
      hipExtLaunchKernelGGL(k_rb_red_prolong<T, 2, true>, g, dim3(256), 0, s, ev.start, ev.stop, 0, x, b, e, lg, c0,
                            c1);
    else
      hipLaunchKernelGGL((k_rb_red_prolong<T, 2, false>), g, dim3(256), 0, s, x, b, e, lg, c0, c1);
  }
}

template <typename T>
void MGHier<T>::rb_first(T* x, const T* b, int lg, int nf, T c0, T c1, bool fine, hipStream_t s) {
  const int64_t Cl = (int64_t)1 << (dim * lg);
  check_quad_aligned(x, b);
  const dim3 g(nblk(Cl / 8), nf);
  // algorithmic traffic of the first sweep from zero: b read once, x written once
  const TimerEvents ev = fine ? timer_sample(kTimerRbFine, 2.0 * (double)Cl * nf * sizeof(T)) : TimerEvents();
  if (dim == 3) {
    if (fine)
      hipExtLaunchKernelGGL(k_rb_first<T, 3, true>, g, dim3(256), 0, s, ev.start, ev.stop, 0, x, b, lg, c0, c1);
    else
      hipLaunchKernelGGL((k_rb_first<T, 3, false>), g, dim3(256), 0, s, x, b, lg, c0, c1);
  } else {
    if (fine)
      hipExtLaunchKernelGGL(k_rb_first<T, 2, true>, g, dim3(256), 0, s, ev.start, ev.stop, 0, x, b, lg, c0, c1);
    else
      hipLaunchKernelGGL((k_rb_first<T, 2, false>), g, dim3(256), 0, s, x, b, lg, c0, c1);
  }
}

template <typename T>
void MGHier<T>::vcycle(int nf, const T* b, T* x, double c0, double c1, int nu_pre, int nu_post, int nu_coarse,
                       hipStream_t s, int wall_mode) {
  if (wall_mode != 0) {
    launch_wall_vcycle<T>(dim, logn, nf, b, x, wall_x, wall_b, c0, c1, nu_pre, nu_post, nu_coarse, wall_mode,
                          wall_mask, s);
    return;
  }
  const bool three = dim == 3;
  T cl = (T)c1;
  const T tc0 = (T)c0;
  const int nml = (int)levels.size();
  // Where each level keeps x: xin (pre-smoothing result, input of the
  // post-smoothing) and xout (the level's result, the correction the finer
  // level interpolates).  They differ only on levels whose post-smoothing runs
  // the fused kernel, which cannot update x in place.
  // whole-cycle timer; algorithmic bytes: per level of C cells and field the
  // per-step kernels' (first sweep 2, each further sweep 3, residual and
  // restriction 2 + 1/8, the coarse correction read by the first red half
  // sweep 1/8, words of w per cell), over the levels about 8/7 of the finest one
  const double words_per_cell =
      2.0 + 3.0 * (nu_pre > 0 ? nu_pre - 1 : 0) + 2.125 + (nu_post > 0 ? 0.125 + 3.0 * nu_post : 1.125);
  const TimerEvents evc =
      timer_sample(kTimerVcycle, words_per_cell * 8.0 / 7.0 * (double)((int64_t)1 << (dim * logn)) * nf * sizeof(T));
  if (evc.start) IBR_HIP(hipEventRecord(evc.start, s));
  auto post_fused = [&](int l) { return nu_post > 0 && fused(logn - l, nu_post, nf); };
  auto xin = [&](int l) -> T* {
    if (l == 0) return post_fused(0) ? x0_tmp : x;
    return bufs_x[l];
  };
  auto xout = [&](int l) -> T* {
    if (l == nml) return nml == 0 ? x : bufs_x[l];
    if (l == 0) return x;
    return post_fused(l) ? bufs_xo[l] : bufs_x[l];
  };
  for (int l = 0; l < nml; ++l) {
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    T* xl = xin(l);
    const T* bl = l == 0 ? b : bufs_b[l];
    if (fused(lg, nu_pre, nf)) {
      check_quad_aligned(xl, bl);
      launch_mg_pre_fused<T>(bl, xl, bufs_b[l + 1], lg, nf, tc0, cl, nu_pre, s,
                             l == 0 ? timer_sample(kTimerRbFine, 2.125 * (double)Cl * nf * sizeof(T)) : TimerEvents());
      cl = cl * T(0.25);
      continue;
    }
    if (nu_pre <= 0)
      launch_fill<T>(xl, Cl * nf, T(0), s);
    else
      rb_first(xl, bl, lg, nf, tc0, cl, l == 0, s);
    for (int sw = 1; sw < nu_pre; ++sw)
      for (int color = 0; color < 2; ++color) rb_half(xl, bl, lg, nf, tc0, cl, color, l == 0, s);
    const int64_t Cc = Cl >> dim;
    if (three)
      hipLaunchKernelGGL((k_resid_restrict<T, 3>), dim3(nblk(Cc / 4), nf), dim3(256), 0, s, xl, bl, bufs_b[l + 1],
                         lg, tc0, cl);
    else
      hipLaunchKernelGGL((k_resid_restrict<T, 2>), dim3(nblk(Cc / 4), nf), dim3(256), 0, s, xl, bl, bufs_b[l + 1],
                         lg, tc0, cl);
    cl = cl * T(0.25);
  }
  {
    const T* bl = nml == 0 ? b : bufs_b[nml];
    T* xl = xout(nml);
    if (three)
      hipLaunchKernelGGL((k_vcycle_lds<T, 3>), dim3(nf), dim3(kLdsThreads), 0, s, bl, xl, lds_logn, tc0, cl, nu_pre,
                         nu_post, nu_coarse);
    else
      hipLaunchKernelGGL((k_vcycle_lds<T, 2>), dim3(nf), dim3(kLdsThreads), 0, s, bl, xl, lds_logn, tc0, cl, nu_pre,
                         nu_post, nu_coarse);
  }
  for (int l = nml - 1; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    const T* bl = l == 0 ? b : bufs_b[l];
    const T* e = xout(l + 1);
    if (post_fused(l)) {
      launch_mg_post_fused<T>(bl, xin(l), xout(l), e, lg, nf, tc0, cl, nu_post, s,
                              l == 0 ? timer_sample(kTimerRbFine, 3.125 * (double)Cl * nf * sizeof(T)) : TimerEvents());
      continue;
    }
    T* xl = xin(l);  // == xout(l): updated in place
    if (nu_post > 0) {
      // the prolongation folded into the first red half sweep (which alone
      // reads the corrected black cells; the black half sweep rewrites them)
      rb_red_prolong(xl, bl, e, lg, nf, tc0, cl, l == 0, s);
      rb_half(xl, bl, lg, nf, tc0, cl, 1, l == 0, s);
      for (int sw = 1; sw < nu_post; ++sw)
        for (int color = 0; color < 2; ++color) rb_half(xl, bl, lg, nf, tc0, cl, color, l == 0, s);
    } else {
      const dim3 gp(nblk(Cl / 8), nf);
      if (three)
        hipLaunchKernelGGL((k_prolong_add<T, 3, false>), gp, dim3(256), 0, s, xl, e, lg);
      else
        hipLaunchKernelGGL((k_prolong_add<T, 2, false>), gp, dim3(256), 0, s, xl, e, lg);
    }
  }
  if (evc.stop) IBR_HIP(hipEventRecord(evc.stop, s));
}

template struct MGHier<double>;
template struct MGHier<float>;

}  // namespace ibr
