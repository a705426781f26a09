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

constexpr int kCholThreads = 256;

// Blocked right-looking Cholesky of M_p + shift_p f0 I, one workgroup per body:
// 16-column panels factored with scalar code, trailing updates
// C -= P_I P_J^T as 16x16 fp64 MFMA tiles spread over the waves.
__global__ void __launch_bounds__(kCholThreads) k_chol(const int* __restrict__ off, int dim,
                                                       const int64_t* __restrict__ moff, const double* __restrict__ M,
                                                       double* __restrict__ Lf, const int* __restrict__ active,
                                                       const double* __restrict__ shift, double f0, double pivot_tol,
                                                       int* __restrict__ fail) {
  const int b = blockIdx.x;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int nt = ld / 16;
  const double* A = M + moff[b];
  double* L = Lf + moff[b];
  const double sh = shift[b] * f0;
  for (int64_t q = threadIdx.x; q < (int64_t)ld * ld; q += blockDim.x) {
    const int i = (int)(q / ld), j = (int)(q - (int64_t)i * ld);
    double v = 0.0;
    if (j <= i) {
      if (i < n) v = A[q] + (i == j ? sh : 0.0);
      else if (i == j) v = 1.0;
    }
    L[q] = v;
  }
  __shared__ double s_piv;
  __shared__ int s_fail;
  if (threadIdx.x == 0) s_fail = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int p = 0; p < nt; ++p) {
    const int c0 = 16 * p;
    // panel: columns c0..c0+15, rows c0..ld-1, unblocked right-looking
    for (int jj = 0; jj < 16; ++jj) {
      const int col = c0 + jj;
      if (threadIdx.x == 0) {
        const double d = L[(int64_t)col * ld + col];
        if (!(d > pivot_tol * f0)) s_fail = 1;
        s_piv = sqrt(d > 0 ? d : 1.0);
        L[(int64_t)col * ld + col] = s_piv;
      }
      __syncthreads();
      if (s_fail) break;
      const double inv = 1.0 / s_piv;
      for (int i = col + 1 + threadIdx.x; i < ld; i += blockDim.x) L[(int64_t)i * ld + col] *= inv;
      __syncthreads();
      const int ncol = 15 - jj;  // remaining panel columns
      if (ncol > 0) {
        const int nrow = ld - col - 1;
        for (int q = threadIdx.x; q < nrow * ncol; q += blockDim.x) {
          const int i = col + 1 + q / ncol;
          const int c = col + 1 + q % ncol;
          if (c <= i) L[(int64_t)i * ld + c] -= L[(int64_t)i * ld + col] * L[(int64_t)c * ld + col];
        }
      }
      __syncthreads();
    }
    if (s_fail) break;
    // trailing update of the lower tiles (I, J), p < J <= I < nt
    const int T = nt - p - 1;
    const int ntiles = T * (T + 1) / 2;
    for (int t = wv; t < ntiles; t += nw) {
      // unrank t -> (I, J) in row-major lower-triangular order
      int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      while (I * (I + 1) / 2 > t) --I;
      const int J = t - I * (I + 1) / 2;
      const int r0 = 16 * (p + 1 + I), q0 = 16 * (p + 1 + J);
      dvec4 acc;
      const int ci = lane & 15, rq = lane >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = L[(int64_t)(r0 + 4 * r + rq) * ld + q0 + ci];
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4) {
        const double a = -L[(int64_t)(r0 + ci) * ld + c0 + k0 + rq];
        const double bb = L[(int64_t)(q0 + ci) * ld + c0 + k0 + rq];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 4 * r + rq, cc = q0 + ci;
        if (I != J || cc <= row) L[(int64_t)row * ld + cc] = acc[r];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) fail[b] = s_fail;
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
                 const int* active, const double* shift, double f0, double pivot_tol, int* fail, hipStream_t s) {
  hipLaunchKernelGGL(k_chol, dim3(nb), dim3(kCholThreads), 0, s, offsets, dim, moff, M, Lf, active, shift, f0,
                     pivot_tol, fail);
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
