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
  const int n = dim * np;
  double* blk = M + moff[b];
  for (int a = 0; a < dim; ++a)
    for (int c = 0; c < dim; ++c) {
      const double ra = r > 0 ? dr[a] / r : 0.0, rc = r > 0 ? dr[c] / r : 0.0;
      blk[(int64_t)(dim * i + a) * n + (dim * j + c)] = (a == c ? f : 0.0) + g * ra * rc;
    }
}

// Right-looking Cholesky of M_p + shift_p f0 I into Lf (lower triangle,
// row-major), one workgroup per body.  Bodies with active[p] == 0 are skipped.
// fail[p] = 1 when a pivot is not above pivot_tol * f0.
constexpr int kCholThreads = 512;

__global__ void __launch_bounds__(kCholThreads) k_chol(const int* __restrict__ off, int dim,
                                                       const int64_t* __restrict__ moff, const double* __restrict__ M,
                                                       double* __restrict__ Lf, const int* __restrict__ active,
                                                       const double* __restrict__ shift, double f0, double pivot_tol,
                                                       int* __restrict__ fail) {
  const int b = blockIdx.x;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const double* A = M + moff[b];
  double* L = Lf + moff[b];
  const double sh = shift[b] * f0;
  for (int64_t q = threadIdx.x; q < (int64_t)n * n; q += blockDim.x) {
    const int i = (int)(q / n), j = (int)(q - (int64_t)i * n);
    L[q] = j <= i ? A[q] + (i == j ? sh : 0.0) : 0.0;
  }
  __shared__ double col[1024 * 3];  // column j below the diagonal (n <= 3072)
  __shared__ double s_piv;
  __shared__ int s_fail;
  if (threadIdx.x == 0) s_fail = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double d = L[(int64_t)j * n + j];
      if (!(d > pivot_tol * f0)) s_fail = 1;
      s_piv = sqrt(d > 0 ? d : 1.0);
      L[(int64_t)j * n + j] = s_piv;
    }
    __syncthreads();
    if (s_fail) break;
    const double inv = 1.0 / s_piv;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
      const double v = L[(int64_t)i * n + j] * inv;
      L[(int64_t)i * n + j] = v;
      col[i] = v;
    }
    __syncthreads();
    for (int i = j + 1 + wv; i < n; i += nw) {
      const double lij = col[i];
      double* row = L + (int64_t)i * n;
      for (int k = j + 1 + lane; k <= i; k += kWave) row[k] -= lij * col[k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) fail[b] = s_fail;
}

// X = L^-1 (lower triangular), one workgroup per body, one column per thread.
__global__ void __launch_bounds__(256) k_tri_inv(const int* __restrict__ off, int dim,
                                                 const int64_t* __restrict__ moff, const double* __restrict__ Lf,
                                                 double* __restrict__ X) {
  const int b = blockIdx.x;
  const int n = dim * (off[b + 1] - off[b]);
  const double* L = Lf + moff[b];
  double* Xb = X + moff[b];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    for (int i = 0; i < j; ++i) Xb[(int64_t)i * n + j] = 0.0;
    for (int i = j; i < n; ++i) {
      double s = i == j ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= L[(int64_t)i * n + k] * Xb[(int64_t)k * n + j];
      Xb[(int64_t)i * n + j] = s / L[(int64_t)i * n + i];
    }
  }
}

// Minv = X^T X  (X lower triangular), 16x16 output tiles, LDS-staged.
__global__ void __launch_bounds__(256) k_xtx(const int* __restrict__ off, int dim, const int64_t* __restrict__ moff,
                                             const double* __restrict__ X, double* __restrict__ Minv) {
  const int b = blockIdx.z;
  const int n = dim * (off[b + 1] - off[b]);
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  if (i0 >= n || j0 >= n) return;
  const double* Xb = X + moff[b];
  __shared__ double ti[16][17], tj[16][17];
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  const int i = i0 + ty, j = j0 + tx;
  double acc = 0;
  const int kstart = (i0 > j0 ? i0 : j0);
  for (int k0 = kstart - (kstart % 16); k0 < n; k0 += 16) {
    // rows k0..k0+15 of X, columns i0.. and j0..
    const int kr = k0 + ty;
    ti[ty][tx] = (kr < n && i0 + tx < n) ? Xb[(int64_t)kr * n + i0 + tx] : 0.0;
    tj[ty][tx] = (kr < n && j0 + tx < n) ? Xb[(int64_t)kr * n + j0 + tx] : 0.0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += ti[q][ty] * tj[q][tx];
    __syncthreads();
  }
  if (i < n && j < n) Minv[moff[b] + (int64_t)i * n + j] = acc;
}

// lam_p = Minv_p dU_p: one wavefront per row.
__global__ void __launch_bounds__(256) k_mob_apply(const int* __restrict__ off, int dim,
                                                   const int64_t* __restrict__ moff, const double* __restrict__ Minv,
                                                   const double* __restrict__ dU, double* __restrict__ lam) {
  const int b = blockIdx.y;
  const int lo = off[b];
  const int n = dim * (off[b + 1] - lo);
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  const double* Mr = Minv + moff[b] + (int64_t)row * n;
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
  hipLaunchKernelGGL(k_tri_inv, dim3(nb), dim3(256), 0, s, offsets, dim, moff, Lf, X);
  const unsigned t = (unsigned)((max_n + 15) / 16);
  hipLaunchKernelGGL(k_xtx, dim3(t, t, nb), dim3(256), 0, s, offsets, dim, moff, X, Minv);
}

void launch_mob_apply(int nb, const int* offsets, int dim, const int64_t* moff, const double* Minv,
                      const double* dU, double* lam, int max_rows, hipStream_t s) {
  const unsigned g = (unsigned)((max_rows + 3) / 4);
  hipLaunchKernelGGL(k_mob_apply, dim3(g, nb), dim3(256), 0, s, offsets, dim, moff, Minv, dU, lam);
}

}  // namespace ibr
