// Krylov building blocks (Sec. 5): block Gram-Schmidt passes, norms, basis
// combination and the Givens-rotation Hessenberg least squares of GMRES.
// All reductions are two-pass with a fixed partition, so results are
// bitwise reproducible run to run.
#include <algorithm>

#include "kernels.h"

namespace ibr {

namespace {

constexpr int kDotCols = 8;  // basis vectors per multi-dot block

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

// part[j * nblocks + block] = partial <w, V_j> for j in this block's column chunk.
template <typename TV, typename TW>
__global__ void __launch_bounds__(256) k_multi_dot(const TV* __restrict__ V, int64_t ld, int k,
                                                   const TW* __restrict__ w, int64_t len, double* __restrict__ part,
                                                   const int* __restrict__ cond) {
  if (cond && cond[0] == 0) return;
  __shared__ double red[kDotCols][256 / kWave];
  const int j0 = blockIdx.y * kDotCols;
  const int nj = min(kDotCols, k - j0);
  double acc[kDotCols];
#pragma unroll
  for (int q = 0; q < kDotCols; ++q) acc[q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    const double wi = (double)w[i];
#pragma unroll
    for (int q = 0; q < kDotCols; ++q)
      if (q < nj) acc[q] += (double)V[(int64_t)(j0 + q) * ld + i] * wi;
  }
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < kDotCols; ++q) {
    double s = wave_sum(acc[q]);
    if (lane == 0) red[q][wv] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < nj) {
    double s = 0;
    for (int u = 0; u < (int)(blockDim.x / kWave); ++u) s += red[threadIdx.x][u];
    part[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_dot_finish(const double* __restrict__ part, int nblocks, double* __restrict__ h, int accumulate,
                             const int* __restrict__ cond) {
  if (cond && cond[0] == 0) return;
  __shared__ double red[256 / kWave];
  const int j = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[(int64_t)j * nblocks + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) h[j] = accumulate ? h[j] + s : s;
}

template <typename TV, typename TW>
__global__ void __launch_bounds__(256) k_multi_axpy(const TV* __restrict__ V, int64_t ld, int k,
                                                    const double* __restrict__ h, TW* __restrict__ w, int64_t len,
                                                    double* __restrict__ norm_part, const int* __restrict__ cond) {
  if (cond && cond[0] == 0) return;
  __shared__ double red[256 / kWave];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double ss = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    double acc = (double)w[i];
    for (int j = 0; j < k; ++j) acc -= h[j] * (double)V[(int64_t)j * ld + i];
    const TW o = (TW)acc;
    w[i] = o;
    ss += (double)o * (double)o;
  }
  if (norm_part) {
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) norm_part[blockIdx.x] = ss;
  }
}

template <typename TZ, typename TX>
__global__ void __launch_bounds__(256) k_combine(const TZ* __restrict__ Z, int64_t ld, int k,
                                                 const double* __restrict__ y, TX* __restrict__ x, int64_t len,
                                                 int assign, const double* __restrict__ zmean, int64_t C, int dim) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    double acc = assign ? 0.0 : (double)x[i];
    for (int j = 0; j < k; ++j) acc += y[j] * (double)Z[(int64_t)j * ld + i];
    if (zmean && i < dim * C) {
      const int a = (int)(i >= C) + (int)(i >= 2 * C);
      double sh = 0.0;
      for (int j = 0; j < k; ++j) sh += y[j] * zmean[4 * j + a];
      acc -= sh;
    }
    x[i] = (TX)acc;
  }
}

// Normal equations of min_y || r - W y || for a few columns W_0..W_{NS-1}:
// part holds nblocks per-workgroup partial sums, in fp64, of each product in
// the order (upper triangle of W^T W row by row, then W^T r), row q at
// part[q * nblocks].  Sums the rows (one wavefront per row, fixed order) and
// solves (W^T W) y = W^T r by Cholesky.  A column that is numerically in the
// span of the earlier ones (squared pivot <= drop * its squared norm) is
// dropped and gets y = 0, so a zero or rank-deficient W still yields a finite
// minimiser.
template <int NS>
__global__ void __launch_bounds__(1024) k_gram_solve(const double* __restrict__ part, int nblocks,
                                                     double* __restrict__ y, double drop) {
  constexpr int NQ = NS * (NS + 1) / 2 + NS;
  __shared__ double tot[NQ];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int q = wv; q < NQ; q += (int)(blockDim.x / kWave)) {
    const double* pr = part + (int64_t)q * nblocks;
    double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    int i = lane;
    for (; i + 3 * kWave < nblocks; i += 4 * kWave) {
      v0 += pr[i];
      v1 += pr[i + kWave];
      v2 += pr[i + 2 * kWave];
      v3 += pr[i + 3 * kWave];
    }
    for (; i < nblocks; i += kWave) v0 += pr[i];
    const double v = wave_sum((v0 + v1) + (v2 + v3));
    if (lane == 0) tot[q] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double G[NS][NS], L[NS][NS], rhs[NS], z[NS];
  bool keep[NS];
  int q = 0;
  for (int a = 0; a < NS; ++a)
    for (int b = a; b < NS; ++b) {
      G[a][b] = tot[q];
      G[b][a] = tot[q];
      ++q;
    }
  for (int a = 0; a < NS; ++a) rhs[a] = tot[q++];
  for (int k = 0; k < NS; ++k) {
    double d = G[k][k];
    for (int m = 0; m < k; ++m)
      if (keep[m]) d -= L[k][m] * L[k][m];
    keep[k] = G[k][k] > 0.0 && d > drop * G[k][k];
    L[k][k] = keep[k] ? sqrt(d) : 1.0;
    for (int i = k + 1; i < NS; ++i) {
      double v = G[i][k];
      for (int m = 0; m < k; ++m)
        if (keep[m]) v -= L[i][m] * L[k][m];
      L[i][k] = keep[k] ? v / L[k][k] : 0.0;
    }
  }
  for (int k = 0; k < NS; ++k) {
    double v = rhs[k];
    for (int m = 0; m < k; ++m)
      if (keep[m]) v -= L[k][m] * z[m];
    z[k] = keep[k] ? v / L[k][k] : 0.0;
  }
  for (int k = NS - 1; k >= 0; --k) {
    double v = z[k];
    for (int m = k + 1; m < NS; ++m)
      if (keep[m]) v -= L[m][k] * y[m];
    y[k] = keep[k] ? v / L[k][k] : 0.0;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_sumsq(const T* __restrict__ w, int64_t len, double* __restrict__ part) {
  __shared__ double red[256 / kWave];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double ss = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    const double v = (double)w[i];
    ss += v * v;
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

__global__ void k_norm_finish(const double* __restrict__ part, int nblocks, double* __restrict__ out) {
  __shared__ double red[256 / kWave];
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

template <typename TS, typename TD>
__global__ void k_scale_copy(const TS* __restrict__ src, TD* __restrict__ dst, int64_t len,
                             const double* __restrict__ nrm) {
  const double nv = nrm[0];
  const double sc = nv > 0.0 ? 1.0 / nv : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    dst[i] = (TD)((double)src[i] * sc);
}

template <typename TS, typename TD>
__global__ void k_copy(const TS* __restrict__ src, TD* __restrict__ dst, int64_t len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) dst[i] = (TD)src[i];
}

__global__ void k_axpby(const double* __restrict__ x, double* __restrict__ y, int64_t len, double a, double b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) y[i] = a * x[i] + b * y[i];
}

// Daniel-Gragg-Kaufman-Stewart test after one Gram-Schmidt pass: hcol[k+1]
// holds ||w||^2 before the pass, part1 the partial sums of ||w||^2 after it.
// Re-orthogonalise (flag = 1) when the norm dropped below 1/sqrt(2) of its
// value; otherwise store the final norm in hcol[k+1].
__global__ void k_dgks_decide(double* __restrict__ hcol, int k, const double* __restrict__ part1, int nblocks,
                              int* __restrict__ flag) {
  __shared__ double red[256 / kWave];
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part1[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double before = hcol[k + 1];
    const int f = s < 0.5 * before ? 1 : 0;
    flag[0] = f;
    if (!f) hcol[k + 1] = sqrt(s);
  }
}

// After the second pass: hcol[0..k] += h2, hcol[k+1] = ||w||.
__global__ void k_dgks_finish(double* __restrict__ hcol, int k, const double* __restrict__ h2,
                              const double* __restrict__ part2, int nblocks, const int* __restrict__ flag) {
  if (flag[0] == 0) return;
  __shared__ double red[256 / kWave];
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part2[i];
  s = block_sum(s, red);
  for (int i = threadIdx.x; i <= k; i += blockDim.x) hcol[i] += h2[i];
  if (threadIdx.x == 0) hcol[k + 1] = sqrt(s);
}

// ---------------------------------------------------------------- delayed CGS2 (outer Arnoldi)
// Basis layout V_0..V_{k+1} with stride ld.  On entry to iteration k, V_k is
// the "pending" vector (one Gram-Schmidt pass, not normalised) and V_{k+1} = w
// = K z_k.  One reduction computes <V_j, V_k> and <V_j, w> for all j; one
// update pass re-orthogonalises and normalises V_k and projects w; w stays
// pending for the next iteration.  Same stability as two-pass CGS with half
// the passes over the basis.

// part[(2 j + r) * nblocks + block]: r = 0 against V_k, r = 1 against w.
// Up to kDualCols basis vectors per workgroup row (blockIdx.y), so the two
// vectors being orthogonalised are read once per chunk.  Element offsets are
// 32-bit (len < 2^28) on top of uniform column base addresses.
constexpr int kDualCols = 16;
// (4 waves per SIMD: room for all the loads of one element in flight)
template <typename T, int NJ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) k_dual_dot(const T* __restrict__ V, int64_t ld, int j0, int kx, int len,
                                                  double* __restrict__ part) {
  __shared__ double red[2 * NJ][256 / kWave];
  const T* __restrict__ x1 = V + (int64_t)kx * ld;
  const T* __restrict__ x2 = x1 + ld;
  const T* __restrict__ Vj = V + (int64_t)j0 * ld;
  double a1[NJ], a2[NJ];
#pragma unroll
  for (int q = 0; q < NJ; ++q) a1[q] = a2[q] = 0.0;
  const unsigned stride = gridDim.x * blockDim.x;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < (unsigned)len; i += stride) {
    double v[NJ];
    // the basis columns are streamed once per pass (a basis of 15 columns is
    // about 1 GB at 128^3, beyond every cache): non-temporal loads keep them
    // from evicting the two vectors the next pass reads again
#pragma unroll
    for (int q = 0; q < NJ; ++q) v[q] = (double)__builtin_nontemporal_load(&Vj[(int64_t)q * ld + i]);
    const double u = (double)x1[i], w = (double)x2[i];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
      a1[q] += v[q] * u;
      a2[q] += v[q] * w;
    }
  }
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NJ; ++q) {
    const double s1 = wave_sum(a1[q]);
    const double s2 = wave_sum(a2[q]);
    if (lane == 0) {
      red[2 * q][wv] = s1;
      red[2 * q + 1][wv] = s2;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * NJ) {
    double t = 0;
    for (int u = 0; u < (int)(blockDim.x / kWave); ++u) t += red[threadIdx.x][u];
    part[(int64_t)(2 * j0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
  }
}

// Sums the 2(k+2) rows of partials (one wavefront per row, rows round-robin
// over the 4 wavefronts, fixed order) into G, then computes the coefficients
// of the delayed step.  G[2j] = <V_j, V_k>, G[2j+1] = <V_j, w>.
// coef[0..k) = s (re-orthogonalisation of V_k), coef[k] = nu, coef[k+1 .. 2k+1] = c.
// Column k-1 of H is corrected (its pending vector is now resolved) and the
// provisional column k is written.
__global__ void __launch_bounds__(1024) k_dcgs2_coef(const double* __restrict__ part, int nblocks,
                                                     double* __restrict__ G, int k, double* __restrict__ H, int ldh,
                                                     double* __restrict__ coef) {
  const int rows = 2 * (k + 2);
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int r = wv; r < rows; r += (int)(blockDim.x / kWave)) {
    const double* pr = part + (int64_t)r * nblocks;
    double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    int i = lane;
    for (; i + 3 * kWave < nblocks; i += 4 * kWave) {
      v0 += pr[i];
      v1 += pr[i + kWave];
      v2 += pr[i + 2 * kWave];
      v3 += pr[i + 3 * kWave];
    }
    for (; i < nblocks; i += kWave) v0 += pr[i];
    const double v = wave_sum((v0 + v1) + (v2 + v3));
    if (lane == 0) G[r] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* colk = H + (int64_t)k * ldh;
  if (k == 0) {
    coef[0] = 1.0;
    coef[1] = G[1];
    colk[0] = G[1];
    return;
  }
  double ss = 0.0, sg = 0.0;
  for (int j = 0; j < k; ++j) {
    const double sj = G[2 * j];
    coef[j] = sj;
    ss += sj * sj;
    sg += sj * G[2 * j + 1];
  }
  const double alpha = G[2 * k];
  double nu2 = alpha - ss;
  if (!(nu2 > 0.0)) nu2 = alpha > 0.0 ? alpha * 1e-30 : 1e-300;
  const double nu = sqrt(nu2);
  coef[k] = nu;
  double* colp = H + (int64_t)(k - 1) * ldh;
  for (int j = 0; j < k; ++j) colp[j] += coef[j];
  colp[k] = nu;
  for (int j = 0; j < k; ++j) {
    coef[k + 1 + j] = G[2 * j + 1];
    colk[j] = G[2 * j + 1];
  }
  const double ck = (G[2 * k + 1] - sg) / nu;
  coef[2 * k + 1] = ck;
  colk[k] = ck;
}

// Copy of the new pending vector's first nsplit entries (its velocity and
// pressure fields, C cells each) into split storage in TS: the next outer
// iteration preconditions exactly this vector, so the copy saves that
// iteration a pass over it.
template <typename TS>
struct SplitOut {
  TS* dst;  // null: no copy
  int dim, logn;
  int64_t nsplit;
};

template <typename TS>
__device__ inline void split_store(const SplitOut<TS>& so, int64_t i, double v) {
  const int lc = so.dim * so.logn;
  const int64_t f = i >> lc;
  const int c = (int)(i & (((int64_t)1 << lc) - 1));
  const int mask = (1 << so.logn) - 1;
  const int x = c & mask, y = (c >> so.logn) & mask;
  const int pos = so.dim == 3 ? split_index<3>(x, y, c >> (2 * so.logn), so.logn) : split_index<2>(x, y, 0, so.logn);
  so.dst[(f << lc) + pos] = (TS)v;
}

// V_k <- (V_k - sum_{j<k} s_j V_j) / nu ;  w <- w - sum_{j<k} c_j V_j - c_k V_k(new).
// part[block] = partial sums of the new w^2.
template <typename T, typename TS>
__global__ void __launch_bounds__(256) k_dcgs2_axpy(T* __restrict__ V, int64_t ld, int k,
                                                    const double* __restrict__ coef, int len,
                                                    double* __restrict__ part, SplitOut<TS> so) {
  __shared__ double red[256 / kWave];
  const unsigned stride = gridDim.x * blockDim.x;
  T* __restrict__ vk = V + (int64_t)k * ld;
  T* __restrict__ w = vk + ld;
  const double inv_nu = 1.0 / coef[k];
  const double* c = coef + k + 1;
  double ss = 0.0;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < (unsigned)len; i += stride) {
    double q = (double)vk[i];
    double a = (double)w[i];
    int j = 0;
    // 4 columns per chunk: measured a little faster than 8 or 16 (occupancy)
    for (; j + 4 <= k; j += 4) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (double)__builtin_nontemporal_load(&V[(int64_t)(j + u) * ld + i]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q -= coef[j + u] * v[u];
        a -= c[j + u] * v[u];
      }
    }
    for (; j < k; ++j) {
      const double v = (double)__builtin_nontemporal_load(&V[(int64_t)j * ld + i]);
      q -= coef[j] * v;
      a -= c[j] * v;
    }
    if (k > 0) {
      q *= inv_nu;
      vk[i] = (T)q;
    }
    a -= c[k] * q;
    const T o = (T)a;
    w[i] = o;
    if (so.dst && (int64_t)i < so.nsplit) split_store(so, i, (double)o);
    ss += (double)o * (double)o;
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

// Provisional h_{k+1,k} = ||w||; finish the Givens rotation of column k-1
// (final now) and estimate the residual with a temporary rotation of column k.
__global__ void k_dcgs2_finish(const double* __restrict__ part, int nblocks, double* __restrict__ H, int ldh,
                               int k, double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                               double* __restrict__ resid) {
  __shared__ double red[256 / kWave];
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x != 0) return;
  double* colk = H + (int64_t)k * ldh;
  colk[k + 1] = sqrt(s);
  if (k > 0) {
    double* col = H + (int64_t)(k - 1) * ldh;
    const int kk = k - 1;
    for (int i = 0; i < kk; ++i) {
      const double t = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
      col[i] = t;
    }
    const double a = col[kk], b = col[kk + 1];
    const double r = hypot(a, b);
    double cc = 1.0, sv = 0.0;
    if (r > 0.0) {
      cc = a / r;
      sv = b / r;
    }
    cs[kk] = cc;
    sn[kk] = sv;
    col[kk] = r;
    col[kk + 1] = 0.0;
    const double gk = g[kk];
    g[kk] = cc * gk;
    g[kk + 1] = -sv * gk;
  }
  // residual estimate: rotations 0..k-1 applied to a copy of column k; only
  // the rotated entry k and h_{k+1,k} matter for the new rotation.
  double t0 = colk[0];
  for (int i = 0; i < k; ++i) t0 = -sn[i] * t0 + cs[i] * colk[i + 1];
  const double t1 = colk[k + 1];
  const double r = hypot(t0, t1);
  const double sv = r > 0.0 ? t1 / r : 0.0;
  resid[0] = fabs(sv * g[k]);
}

// Apply the previous rotations to column k of H, build rotation k, update g.
__global__ void k_givens_step(double* __restrict__ H, int ldh, int k, double* __restrict__ cs,
                              double* __restrict__ sn, double* __restrict__ g, double* __restrict__ resid) {
  if (threadIdx.x != 0) return;
  double* col = H + (int64_t)k * ldh;
  for (int i = 0; i < k; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[k], b = col[k + 1];
  const double r = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (r > 0.0) {
    c = a / r;
    s = b / r;
  }
  cs[k] = c;
  sn[k] = s;
  col[k] = r;
  col[k + 1] = 0.0;
  const double gk = g[k];
  g[k] = c * gk;
  g[k + 1] = -s * gk;
  resid[0] = fabs(g[k + 1]);
}

// Back substitution R y = g for the first k columns of the rotated H.
__global__ void k_lsq_solve(const double* __restrict__ H, int ldh, int k, const double* __restrict__ g,
                            double* __restrict__ y) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[(int64_t)j * ldh + i] * y[j];
    const double d = H[(int64_t)i * ldh + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

__global__ void k_init_g(double* __restrict__ g, int len, const double* __restrict__ beta) {
  for (int i = threadIdx.x; i < len; i += blockDim.x) g[i] = i == 0 ? beta[0] : 0.0;
}

}  // namespace

int krylov_dot_blocks(int64_t len) {
  int64_t b = (len + 256 * 8 - 1) / (256 * 8);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename TV, typename TW>
void launch_multi_dot(const TV* V, int64_t ld, int k, const TW* w, int64_t len, double* part, int nblocks,
                      double* h, bool accumulate, hipStream_t s, const int* cond) {
  if (k <= 0) return;
  const int nchunk = (k + kDotCols - 1) / kDotCols;
  hipLaunchKernelGGL((k_multi_dot<TV, TW>), dim3(nblocks, nchunk), dim3(256), 0, s, V, ld, k, w, len, part, cond);
  hipLaunchKernelGGL(k_dot_finish, dim3(k), dim3(256), 0, s, part, nblocks, h, accumulate ? 1 : 0, cond);
}
template void launch_multi_dot<double, double>(const double*, int64_t, int, const double*, int64_t, double*, int,
                                               double*, bool, hipStream_t, const int*);
template void launch_multi_dot<float, float>(const float*, int64_t, int, const float*, int64_t, double*, int,
                                             double*, bool, hipStream_t, const int*);

template <typename TV, typename TW>
void launch_multi_axpy(const TV* V, int64_t ld, int k, const double* h, TW* w, int64_t len, double* norm_part,
                       int nblocks, hipStream_t s, const int* cond) {
  hipLaunchKernelGGL((k_multi_axpy<TV, TW>), dim3(nblocks), dim3(256), 0, s, V, ld, k, h, w, len, norm_part,
                     cond);
}
template void launch_multi_axpy<double, double>(const double*, int64_t, int, const double*, double*, int64_t,
                                                double*, int, hipStream_t, const int*);
template void launch_multi_axpy<float, float>(const float*, int64_t, int, const double*, float*, int64_t, double*,
                                              int, hipStream_t, const int*);

template <typename T>
void arnoldi_step(const T* V, int64_t ld, int k, double* hcol, double* h2, double* part1, double* part2,
                  int nblocks, int* flag, hipStream_t s, bool timed, bool reorth) {
  T* w = const_cast<T*>(V) + (int64_t)(k + 1) * ld;
  (void)timed;  // the inner Arnoldi passes are not a timed class
  // pass 1: columns 0..k+1 (the last one is w itself, giving ||w||^2 in hcol[k+1])
  launch_multi_dot<T, T>(V, ld, k + 2, w, ld, part1, nblocks, hcol, false, s, nullptr);
  launch_multi_axpy<T, T>(V, ld, k + 1, hcol, w, ld, part1, nblocks, s, nullptr);
  if (!reorth) {
    launch_norm_finish(part1, nblocks, hcol + k + 1, s);
    return;
  }
  hipLaunchKernelGGL(k_dgks_decide, dim3(1), dim3(256), 0, s, hcol, k, part1, nblocks, flag);
  // pass 2 only when the DGKS test asks for it
  launch_multi_dot<T, T>(V, ld, k + 1, w, ld, part2, nblocks, h2, false, s, flag);
  launch_multi_axpy<T, T>(V, ld, k + 1, h2, w, ld, part2, nblocks, s, flag);
  hipLaunchKernelGGL(k_dgks_finish, dim3(1), dim3(256), 0, s, hcol, k, h2, part2, nblocks, flag);
}
template void arnoldi_step<double>(const double*, int64_t, int, double*, double*, double*, double*, int, int*,
                                   hipStream_t, bool, bool);
template void arnoldi_step<float>(const float*, int64_t, int, double*, double*, double*, double*, int, int*,
                                  hipStream_t, bool, bool);

template <typename TZ, typename TX>
void launch_combine(const TZ* Z, int64_t ld, int k, const double* y, TX* x, int64_t len, hipStream_t s,
                    bool assign, const double* zmean, int64_t C, int dim) {
  if (k <= 0) return;
  unsigned g = nblk(len);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL((k_combine<TZ, TX>), dim3(g), dim3(256), 0, s, Z, ld, k, y, x, len, assign ? 1 : 0, zmean, C,
                     dim);
}
template void launch_combine<double, double>(const double*, int64_t, int, const double*, double*, int64_t,
                                             hipStream_t, bool, const double*, int64_t, int);
template void launch_combine<float, double>(const float*, int64_t, int, const double*, double*, int64_t,
                                            hipStream_t, bool, const double*, int64_t, int);
template void launch_combine<float, float>(const float*, int64_t, int, const double*, float*, int64_t,
                                           hipStream_t, bool, const double*, int64_t, int);

// A column whose squared distance from the span of the previous ones is
// below this fraction of its squared norm is dropped (rounding level of T).
template <typename T>
constexpr double gram_drop() {
  return sizeof(T) == 4 ? 1e-5 : 1e-13;
}

template <typename T>
void launch_gram_finish(const double* part, int nblocks, int ns, double* y, hipStream_t s) {
  const double drop = gram_drop<T>();
  switch (ns) {
    case 1:
      hipLaunchKernelGGL((k_gram_solve<1>), dim3(1), dim3(1024), 0, s, part, nblocks, y, drop);
      break;
    case 2:
      hipLaunchKernelGGL((k_gram_solve<2>), dim3(1), dim3(1024), 0, s, part, nblocks, y, drop);
      break;
    case 3:
      hipLaunchKernelGGL((k_gram_solve<3>), dim3(1), dim3(1024), 0, s, part, nblocks, y, drop);
      break;
    default:
      throw DeviceError("launch_gram_finish: n_s must be 1, 2 or 3");
  }
}
template void launch_gram_finish<double>(const double*, int, int, double*, hipStream_t);
template void launch_gram_finish<float>(const double*, int, int, double*, hipStream_t);

void launch_norm_finish(const double* part, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(256), 0, s, part, nblocks, out);
}

template <typename T>
void launch_sumsq_partial(const T* w, int64_t len, double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq<T>, dim3(nblocks), dim3(256), 0, s, w, len, part);
}
template void launch_sumsq_partial<double>(const double*, int64_t, double*, int, hipStream_t);
template void launch_sumsq_partial<float>(const float*, int64_t, double*, int, hipStream_t);

template <typename TS, typename TD>
void launch_scale_copy(const TS* src, TD* dst, int64_t len, const double* nrm, hipStream_t s) {
  unsigned g = nblk(len);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL((k_scale_copy<TS, TD>), dim3(g), dim3(256), 0, s, src, dst, len, nrm);
}
template void launch_scale_copy<double, double>(const double*, double*, int64_t, const double*, hipStream_t);
template void launch_scale_copy<double, float>(const double*, float*, int64_t, const double*, hipStream_t);
template void launch_scale_copy<float, float>(const float*, float*, int64_t, const double*, hipStream_t);

template <typename TS, typename TD>
void launch_copy(const TS* src, TD* dst, int64_t len, hipStream_t s) {
  if (len <= 0) return;
  unsigned g = nblk(len);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL((k_copy<TS, TD>), dim3(g), dim3(256), 0, s, src, dst, len);
}
template void launch_copy<double, double>(const double*, double*, int64_t, hipStream_t);
template void launch_copy<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_copy<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_copy<float, float>(const float*, float*, int64_t, hipStream_t);

void launch_axpby(const double* x, double* y, int64_t len, double a, double b, hipStream_t s) {
  unsigned g = nblk(len);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_axpby, dim3(g), dim3(256), 0, s, x, y, len, a, b);
}

template <typename T, typename TS>
void dcgs2_step(T* V, int64_t ld, int64_t len, int k, double* H, int ldh, double* G, double* coef, double* part,
                int nblocks, double* cs, double* sn, double* g, double* resid, hipStream_t s, bool timed,
                TS* split, int dim, int logn, int64_t nsplit) {
  if (len >= ((int64_t)1 << 28)) throw DeviceError("dcgs2_step: vectors longer than 2^28 entries");
  const int ncols = k + 2;
  const double vb = (double)len * sizeof(T);
  // the reduction's algorithmic bytes (all chunks): the k+2 columns once, plus
  // the two vectors being orthogonalised once per extra chunk; the first chunk
  // carries the start event, the last the stop event
  const TimerEvents evd =
      timed ? timer_sample(kTimerOrthoDot, (ncols + 2 * ((ncols - 1) / kDualCols)) * vb) : TimerEvents();
  for (int j0 = 0; j0 < ncols; j0 += kDualCols) {
    const int nj = std::min(kDualCols, ncols - j0);
    const hipEvent_t e0 = j0 == 0 ? evd.start : nullptr;
    const hipEvent_t e1 = j0 + kDualCols >= ncols ? evd.stop : nullptr;
    switch (nj) {
#define IBR_DUAL(NJ)                                                                                          \
  case NJ:                                                                                                    \
    hipExtLaunchKernelGGL(k_dual_dot<T, NJ>, dim3(nblocks), dim3(256), 0, s, e0, e1, 0, (const T*)V, ld, j0, k, \
                          (int)len, part);                                                                    \
    break;
      IBR_DUAL(1) IBR_DUAL(2) IBR_DUAL(3) IBR_DUAL(4) IBR_DUAL(5) IBR_DUAL(6) IBR_DUAL(7) IBR_DUAL(8)
      IBR_DUAL(9) IBR_DUAL(10) IBR_DUAL(11) IBR_DUAL(12) IBR_DUAL(13) IBR_DUAL(14) IBR_DUAL(15) IBR_DUAL(16)
#undef IBR_DUAL
    }
  }
  hipLaunchKernelGGL(k_dcgs2_coef, dim3(1), dim3(1024), 0, s, part, nblocks, G, k, H, ldh, coef);
  if (split && (nsplit > len || nsplit != ((int64_t)(dim + 1) << (dim * logn))))
    throw DeviceError("dcgs2_step: split copy does not cover the fluid fields of the vectors");
  const SplitOut<TS> so{split, dim, logn, split ? nsplit : 0};
  const double sb = split ? (double)nsplit * sizeof(TS) : 0.0;
  const TimerEvents eva = timed ? timer_sample(kTimerOrthoAxpy, (ncols + 2) * vb + sb) : TimerEvents();
  hipExtLaunchKernelGGL((k_dcgs2_axpy<T, TS>), dim3(nblocks), dim3(256), 0, s, eva.start, eva.stop, 0, V, ld, k,
                        (const double*)coef, (int)len, part, so);
  hipLaunchKernelGGL(k_dcgs2_finish, dim3(1), dim3(256), 0, s, part, nblocks, H, ldh, k, cs, sn, g, resid);
}
template void dcgs2_step<double, float>(double*, int64_t, int64_t, int, double*, int, double*, double*, double*,
                                        int, double*, double*, double*, double*, hipStream_t, bool, float*, int, int,
                                        int64_t);
template void dcgs2_step<double, double>(double*, int64_t, int64_t, int, double*, int, double*, double*, double*,
                                         int, double*, double*, double*, double*, hipStream_t, bool, double*, int, int,
                                         int64_t);

void launch_givens_step(double* H, int ldh, int k, double* cs, double* sn, double* g, double* resid,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_givens_step, dim3(1), dim3(64), 0, s, H, ldh, k, cs, sn, g, resid);
}

void launch_lsq_solve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq_solve, dim3(1), dim3(64), 0, s, H, ldh, k, g, y);
}

void launch_init_g(double* g, int len, const double* beta, hipStream_t s) {
  hipLaunchKernelGGL(k_init_g, dim3(1), dim3(128), 0, s, g, len, beta);
}

}  // namespace ibr
