// Per-body approximate mobility blocks (Sec. 4, eq. M_tilde_ij) and their
// dense solve (Sec. 5.3).  Each body's block is assembled from f(r), g(r),
// factored by Cholesky (shifted by s f(0) I when it is not positive definite)
// and turned into an explicit inverse, so that every preconditioner
// application is one batched matrix-vector product.
//
// Block p is row-major dN_p x dN_p at M + moff[p].
#include "kernels.h"

namespace ibr {

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ void brinkmanlet(double r, double alpha, double eta, double& f, double& g) {
  const double ar = alpha * r;
  const double e = exp(-ar) / (4.0 * kPi * eta * r);
  const double far = 1.0 / (4.0 * kPi * eta * alpha * alpha * r * r * r);
  f = e * (1.0 / (ar * ar) + 1.0 / ar + 1.0) - far;
  g = -e * (3.0 / (ar * ar) + 3.0 / ar + 1.0) + 3.0 * far;
}

__device__ void fb_far(double r, const MobParams& p, double& f, double& g) {
  if (p.dim == 3) {
    brinkmanlet(r, p.alpha, p.eta, f, g);
  } else {
    f = -p.dt_rho / (2.0 * kPi * r * r);
    g = p.dt_rho / (kPi * r * r);
  }
}

// f(r), g(r) of the approximate mobility (same forms as the documented reading
// of Sec. 4 / Appendices A and B).
__device__ void mob_fg(double r, const MobParams& p, double& f, double& g) {
  const double a = p.a;
  if (p.steady) {
    if (p.dim == 3) {
      const double c = 1.0 / (6.0 * kPi * p.eta * a);
      if (r > 2.0 * a) {
        const double q = a / r;
        f = c * (0.75 * q + 0.5 * q * q * q);
        g = c * (0.75 * q - 1.5 * q * q * q);
      } else {
        f = c * (1.0 - 9.0 * r / (32.0 * a));
        g = c * (3.0 * r / (32.0 * a));
      }
      f -= p.periodic_shift;
    } else {
      const double c = 1.0 / (4.0 * kPi * p.eta);
      f = p.finf0 - 0.5 * c * log1p(r * r / (a * a));
      g = c * r * r / (r * r + a * a);
    }
    return;
  }
  const double r2a = 2.0 * a;
  if (r < r2a) {
    double f2, g2;
    fb_far(r2a, p, f2, g2);
    const double t = r / r2a;
    f = p.f00 + t * (f2 - p.f00);
    g = t * g2;
  } else {
    fb_far(r, p, f, g);
  }
}

__global__ void k_mob_assemble(int dim, const int* __restrict__ off, const int64_t* __restrict__ moff,
                               const double* __restrict__ R, MobParams p, double* __restrict__ M) {
  const int b = blockIdx.y;
  const int lo = off[b];
  const int np = off[b + 1] - lo;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)np * np) return;
  const int i = (int)(t / np), j = (int)(t - (int64_t)i * np);
  double dr[3] = {0, 0, 0};
  double r2 = 0;
  for (int a = 0; a < dim; ++a) {
    double d = R[(lo + i) * dim + a] - R[(lo + j) * dim + a];
    d -= p.L * rint(d / p.L);
    dr[a] = d;
    r2 += d * d;
  }
  const double r = sqrt(r2);
  double f, g;
  mob_fg(r, p, f, g);
  const int ld = (dim * np + 15) & ~15;
  double* blk = M + moff[b];
  for (int a = 0; a < dim; ++a)
    for (int c = 0; c < dim; ++c) {
      const double ra = r > 0 ? dr[a] / r : 0.0, rc = r > 0 ? dr[c] / r : 0.0;
      blk[(int64_t)(dim * i + a) * ld + (dim * j + c)] = (a == c ? f : 0.0) + g * ra * rc;
    }
}

// ---------------------------------------------------------------- fp64 MFMA block factorisation
// Blocks are stored row-major with a leading dimension ld = n rounded up to a
// multiple of 16 (the padding is an identity block, so the padded matrix
// factors with the same leading n x n factor).
//
// v_mfma_f64_16x16x4f64 operand layout (lane l of a wave64):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   C/D:       lane l, register r holds D[4 r + l / 16][l % 16]
typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ inline int pad16(int n) { return (n + 15) & ~15; }

// Batched blocked right-looking Cholesky of M_p + shift_p f0 I over all
// bodies, 16x16 tiles.  Per 16-column panel p two launches cover every body:
//   panel:  one wavefront per (row tile I > p, body) factors the diagonal
//           tile in registers (lane r holds row r, shuffles broadcast the
//           pivot column) and solves L_Ip L_pp^T = A_Ip row by row (lane
//           r < 16 owns row r of the tile);
//   update: one wavefront per lower tile (I, J), p < J <= I, of every body:
//           L_IJ -= L_Ip L_Jp^T on fp64 MFMA 16x16x4; one more per body
//           writes the factored diagonal tile (after the panel launch has
//           read the unfactored one).
// So the work of a panel spreads over every compute unit instead of one
// workgroup per body walking all panels.  A pivot <= pivot_tol f0 marks the
// body failed (it is factored again with a larger shift).

// L = lower(M) + shift on the diagonal, identity on the padding rows.
__global__ void __launch_bounds__(64) k_chol_init(const int* __restrict__ off, int dim,
                                                  const int64_t* __restrict__ moff, const double* __restrict__ M,
                                                  double* __restrict__ Lf, const int* __restrict__ active,
                                                  const double* __restrict__ shift, double f0, int* __restrict__ fail) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int i = blockIdx.x;
  if (i >= ld) return;
  if (i == 0 && threadIdx.x == 0) fail[b] = 0;
  const double* A = M + moff[b];
  double* L = Lf + moff[b];
  const double sh = shift[b] * f0;
  for (int j = threadIdx.x; j < ld; j += blockDim.x) {
    double v = 0.0;
    if (j <= i) {
      if (i < n) v = A[(int64_t)i * ld + j] + (i == j ? sh : 0.0);
      else if (i == j) v = 1.0;
    }
    L[(int64_t)i * ld + j] = v;
  }
}

// The diagonal tile (p, p) factored in registers: lane r (mod 16) holds row
// r; shuffles within each group of 16 lanes broadcast the pivot column.
// bad = some pivot <= pivot_tol f0.
__device__ inline void factor_diag_tile(const double* L, int ld, int c0, double row[16], bool& bad, double f0,
                                        double pivot_tol) {
  const int r = threadIdx.x & 15;
#pragma unroll
  for (int c = 0; c < 16; ++c) row[c] = (c <= r) ? L[(int64_t)(c0 + r) * ld + c0 + c] : 0.0;
  bad = false;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double d = __shfl(row[j], j, 16);
    bad = bad || !(d > pivot_tol * f0);
    const double sd = sqrt(d > 0.0 ? d : 1.0);
    if (r == j) row[j] = sd;
    else if (r > j) row[j] = row[j] / sd;
#pragma unroll
    for (int c = j + 1; c < 16; ++c) {
      const double lc = __shfl(row[j], c, 16);  // L[c][j]
      if (r >= c) row[c] -= row[j] * lc;
    }
  }
}

// Row tiles I > p of the panel: L_Ip = A_Ip L_pp^-T.  Every workgroup factors
// the diagonal tile itself from the still unfactored L_pp (it is written back
// by the update launch, after all of them have read it).
__global__ void __launch_bounds__(64) k_chol_panel(const int* __restrict__ off, int dim,
                                                   const int64_t* __restrict__ moff, double* __restrict__ Lf,
                                                   const int* __restrict__ active, int p, double f0, double pivot_tol) {
  __shared__ double D[16][17];
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int nt = ld / 16;
  const int I = p + 1 + blockIdx.x;
  if (I >= nt) return;
  double* L = Lf + moff[b];
  const int lane = threadIdx.x;
  const int r = lane & 15;
  const int c0 = 16 * p;
  double row[16];
  bool bad;
  factor_diag_tile(L, ld, c0, row, bad, f0, pivot_tol);
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) D[r][c] = row[c];
  }
  __syncthreads();
  if (lane >= 16) return;
  // row r of tile I: x L_pp^T = a, forward substitution over the 16 columns
  double* Lr = L + (int64_t)(16 * I + r) * ld + c0;
  double x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = Lr[c];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double t = x[c];
#pragma unroll
    for (int k = 0; k < c; ++k) t -= x[k] * D[c][k];
    x[c] = t / D[c][c];
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) Lr[c] = x[c];
}

// Block 0: write the factored diagonal tile (p, p) and the pivot verdict.
// Blocks 1..: the trailing tiles (I, J), p < J <= I: L_IJ -= L_Ip L_Jp^T.
__global__ void __launch_bounds__(64) k_chol_update(const int* __restrict__ off, int dim,
                                                    const int64_t* __restrict__ moff, double* __restrict__ Lf,
                                                    const int* __restrict__ active, int p, double f0,
                                                    double pivot_tol, int* __restrict__ fail) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int nt = ld / 16;
  if (p >= nt) return;
  double* L = Lf + moff[b];
  const int c0 = 16 * p;
  const int lane = threadIdx.x;
  if (blockIdx.x == 0) {
    double row[16];
    bool bad;
    factor_diag_tile(L, ld, c0, row, bad, f0, pivot_tol);
    if (lane < 16) {
      const int r = lane;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c <= r) L[(int64_t)(c0 + r) * ld + c0 + c] = row[c];
    }
    if (lane == 0 && bad) fail[b] = 1;
    return;
  }
  const int T = nt - p - 1;
  const int t = blockIdx.x - 1;
  if (t >= T * (T + 1) / 2) return;
  // unrank t -> (I, J) in row-major lower-triangular order
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int r0 = 16 * (p + 1 + I), q0 = 16 * (p + 1 + J);
  const int ci = lane & 15, rq = lane >> 4;
  dvec4 acc;
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = L[(int64_t)(r0 + 4 * k + rq) * ld + q0 + ci];
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const double a = -L[(int64_t)(r0 + ci) * ld + c0 + k0 + rq];
    const double bb = L[(int64_t)(q0 + ci) * ld + c0 + k0 + rq];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int row = r0 + 4 * k + rq, cc = q0 + ci;
    if (I != J || cc <= row) L[(int64_t)row * ld + cc] = acc[k];
  }
}

// X = L^-1 (L lower triangular, 16x16 tiles).  First every diagonal tile is
// inverted (one wavefront per tile, lane c < 16 solves for column c), then
// each 16-column block J is filled by block forward substitution,
//   X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ,   I = J+1, J+2, ...
// with one workgroup per (J, body): its four wavefronts split the K-sum
// (fp64 MFMA 16x16x4 tiles) and one of them applies -X_II.
__global__ void __launch_bounds__(64) k_diag_inv(const int* __restrict__ off, int dim,
                                                 const int64_t* __restrict__ moff, const double* __restrict__ Lf,
                                                 double* __restrict__ X) {
  const int b = blockIdx.y;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int I = blockIdx.x;
  if (16 * I >= ld) return;
  const double* L = Lf + moff[b];
  double* Xb = X + moff[b];
  const int r0 = 16 * I;
  const int c = threadIdx.x;
  if (c >= 16) return;
  double col[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double v = i == c ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[(int64_t)(r0 + i) * ld + r0 + k] * col[k];  // col[k] = 0 for k < c
    col[i] = i < c ? 0.0 : v / L[(int64_t)(r0 + i) * ld + r0 + i];
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) Xb[(int64_t)(r0 + i) * ld + r0 + c] = col[i];
}

__global__ void __launch_bounds__(256) k_tri_inv_cols(const int* __restrict__ off, int dim,
                                                      const int64_t* __restrict__ moff,
                                                      const double* __restrict__ Lf, double* __restrict__ X) {
  const int b = blockIdx.y;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int nt = ld / 16;
  const int J = blockIdx.x;
  if (J >= nt) return;
  const double* L = Lf + moff[b];
  double* Xb = X + moff[b];
  __shared__ double part[4][16][17];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int ci = lane & 15, rq = lane >> 4;
  const int j0 = 16 * J;
  for (int I = J + 1; I < nt; ++I) {
    const int i0 = 16 * I;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int K = J + wv; K < I; K += 4) {
      const int k0 = 16 * K;
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const double a = L[(int64_t)(i0 + ci) * ld + k0 + kk + rq];
        const double bb = Xb[(int64_t)(k0 + kk + rq) * ld + j0 + ci];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wv][4 * r + rq][ci] = acc[r];
    __syncthreads();
    if (wv == 0) {
      dvec4 res = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const double a = -Xb[(int64_t)(i0 + ci) * ld + i0 + kk + rq];
        const int sr = kk + rq;
        const double bb = ((part[0][sr][ci] + part[1][sr][ci]) + part[2][sr][ci]) + part[3][sr][ci];
        res = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, res, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Xb[(int64_t)(i0 + 4 * r + rq) * ld + j0 + ci] = res[r];
    }
    __syncthreads();
  }
}

// Minv = X^T X for X = L^-1 lower triangular: one wave per 16x16 tile (I >= J),
// fp64 MFMA over 4-row slabs of X, mirrored into the upper triangle.
__global__ void __launch_bounds__(64) k_xtx(const int* __restrict__ off, int dim, const int64_t* __restrict__ moff,
                                            const double* __restrict__ X, double* __restrict__ Minv) {
  const int b = blockIdx.z;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int I = blockIdx.y, J = blockIdx.x;
  if (16 * I >= ld || J > I) return;
  const double* Xb = X + moff[b];
  const int lane = threadIdx.x;
  const int ci = lane & 15, rq = lane >> 4;
  const int i0 = 16 * I, j0 = 16 * J;
  dvec4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = i0; k0 < ld; k0 += 4) {
    const double a = Xb[(int64_t)(k0 + rq) * ld + i0 + ci];
    const double bb = Xb[(int64_t)(k0 + rq) * ld + j0 + ci];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
  }
  double* Mb = Minv + moff[b];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = i0 + 4 * r + rq, col = j0 + ci;
    Mb[(int64_t)row * ld + col] = acc[r];
    Mb[(int64_t)col * ld + row] = acc[r];
  }
}

// lam_p = Minv_p dU_p: one wavefront per row.
__global__ void __launch_bounds__(256) k_mob_apply(const int* __restrict__ off, int dim,
                                                   const int64_t* __restrict__ moff, const double* __restrict__ Minv,
                                                   const double* __restrict__ dU, double* __restrict__ lam) {
  const int b = blockIdx.y;
  const int lo = off[b];
  const int n = dim * (off[b + 1] - lo);
  const int ld = pad16(n);
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  const double* Mr = Minv + moff[b] + (int64_t)row * ld;
  const double* u = dU + (int64_t)lo * dim;
  double acc = 0;
  for (int k = lane; k < n; k += kWave) acc += Mr[k] * u[k];
  acc = wave_sum(acc);
  if (lane == 0) lam[(int64_t)lo * dim + row] = acc;
}

}  // namespace

void launch_mob_assemble(int dim, int nb, const int* offsets, const int64_t* moff, const double* R, MobParams p,
                         double* M, int max_np, hipStream_t s) {
  const int64_t pairs = (int64_t)max_np * max_np;
  hipLaunchKernelGGL(k_mob_assemble, dim3((unsigned)((pairs + 255) / 256), nb), dim3(256), 0, s, dim, offsets,
                     moff, R, p, M);
}

void launch_chol(int nb, const int* offsets, int dim, const int64_t* moff, const double* M, double* Lf,
                 const int* active, const double* shift, double f0, double pivot_tol, int* fail, int max_rows,
                 hipStream_t s) {
  const int ldmax = (max_rows + 15) & ~15;
  const int ntmax = ldmax / 16;
  hipLaunchKernelGGL(k_chol_init, dim3(ldmax, nb), dim3(64), 0, s, offsets, dim, moff, M, Lf, active, shift, f0,
                     fail);
  for (int p = 0; p < ntmax; ++p) {
    const int T = ntmax - p - 1;
    if (T > 0)
      hipLaunchKernelGGL(k_chol_panel, dim3(T, nb), dim3(64), 0, s, offsets, dim, moff, Lf, active, p, f0,
                         pivot_tol);
    hipLaunchKernelGGL(k_chol_update, dim3(T * (T + 1) / 2 + 1, nb), dim3(64), 0, s, offsets, dim, moff, Lf, active,
                       p, f0, pivot_tol, fail);
  }
}

void launch_chol_inverse(int nb, const int* offsets, int dim, const int64_t* moff, double* Lf, double* Minv,
                         double* X, int max_n, hipStream_t s) {
  const unsigned t = (unsigned)((max_n + 15) / 16);
  hipLaunchKernelGGL(k_diag_inv, dim3(t, nb), dim3(64), 0, s, offsets, dim, moff, Lf, X);
  hipLaunchKernelGGL(k_tri_inv_cols, dim3(t, nb), dim3(256), 0, s, offsets, dim, moff, Lf, X);
  hipLaunchKernelGGL(k_xtx, dim3(t, t, nb), dim3(64), 0, s, offsets, dim, moff, X, Minv);
}

void launch_mob_apply(int nb, const int* offsets, int dim, const int64_t* moff, const double* Minv,
                      const double* dU, double* lam, int max_rows, hipStream_t s) {
  const unsigned g = (unsigned)((max_rows + 3) / 4);
  hipLaunchKernelGGL(k_mob_apply, dim3(g, nb), dim3(256), 0, s, offsets, dim, moff, Minv, dU, lam);
}

}  // namespace ibr
