// Free kinematics: rigid bodies moving under an applied force and torque
// (Sec. 2 poses the problem; Sec. 8 names the enlarged saddle-point system
// and its body mobility N = (K* M^-1 K)^-1, approximated per body).
//
// Once some body is free the stacked vector gains a body block after Lambda:
// the linear velocities U[nb][dim], then the angular velocities
// Omega[nb][1 or 3] (the layout of the body force and torque).  Rows:
//   markers of free bodies:  -J v + K U   (K U = u_p + omega_p x (R_i - X_p))
//   free bodies:             K* Lambda    (sum Lambda_i, sum (R_i - X_p) x Lambda_i)
//   prescribed bodies:       the unknown itself (an identity row; their motion
//                            is in the marker right-hand side instead)
// The preconditioner's per-body step solves, for every free body,
//   M~ Lambda - K U = dU,  K* Lambda = r_U
// as U = N~ (r_U - K* M~^-1 dU), Lambda = M~^-1 dU + Y U, with Y = M~^-1 K
// and N~ = (K* Y)^-1 formed once per set of bodies (one workgroup per body).
#include "kernels.h"

namespace ibr {

namespace {

__device__ inline int pad16f(int n) { return (n + 15) & ~15; }

__device__ inline void rel_pos(int dim, const double* R, const double* X, int m, int b, double L, double r[3]) {
  r[0] = r[1] = r[2] = 0.0;
  for (int a = 0; a < dim; ++a) {
    double d = R[m * dim + a] - X[b * dim + a];
    d -= L * rint(d / L);
    r[a] = d;
  }
}

// Column `col` of the rigid map at marker component a with arm r: a unit
// translation along col (col < dim) or a unit rotation about axis col - dim
// (the z axis in 2D).
__device__ inline double rigid_entry(int dim, int a, int col, const double r[3]) {
  if (col < dim) return a == col ? 1.0 : 0.0;
  if (dim == 2) return a == 0 ? -r[1] : r[0];
  const int e = col - 3;  // (e_e x r)_a
  if (e == 0) return a == 1 ? -r[2] : (a == 2 ? r[1] : 0.0);
  if (e == 1) return a == 0 ? r[2] : (a == 2 ? -r[0] : 0.0);
  return a == 0 ? -r[1] : (a == 1 ? r[0] : 0.0);
}

template <typename TI>
__global__ void k_free_rigid_add(int dim, int N, const double* __restrict__ R, const int* __restrict__ body,
                                 const double* __restrict__ X, double L, const int* __restrict__ free_b,
                                 const TI* __restrict__ xu, const TI* __restrict__ xo, double* __restrict__ yl) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int b = body[m];
  if (!free_b[b]) return;
  double r[3];
  rel_pos(dim, R, X, m, b, L, r);
  if (dim == 2) {
    const double w = (double)xo[b];
    yl[m * 2 + 0] += (double)xu[b * 2 + 0] - w * r[1];
    yl[m * 2 + 1] += (double)xu[b * 2 + 1] + w * r[0];
  } else {
    const double w0 = (double)xo[b * 3 + 0], w1 = (double)xo[b * 3 + 1], w2 = (double)xo[b * 3 + 2];
    yl[m * 3 + 0] += (double)xu[b * 3 + 0] + (w1 * r[2] - w2 * r[1]);
    yl[m * 3 + 1] += (double)xu[b * 3 + 1] + (w2 * r[0] - w0 * r[2]);
    yl[m * 3 + 2] += (double)xu[b * 3 + 2] + (w0 * r[1] - w1 * r[0]);
  }
}

// Sums of one body's marker forces: f = sum lam_i, t = sum r_i x lam_i (all threads get them).
__device__ inline void body_sums(int dim, const int* off, const double* R, const double* X, double L,
                                 const double* lam, int b, double* red, double f[3], double t[3]) {
  const int lo = off[b], hi = off[b + 1];
  double pf[3] = {0, 0, 0}, pt[3] = {0, 0, 0};
  for (int m = lo + threadIdx.x; m < hi; m += blockDim.x) {
    double r[3], l[3] = {0, 0, 0};
    rel_pos(dim, R, X, m, b, L, r);
    for (int a = 0; a < dim; ++a) {
      l[a] = lam[m * dim + a];
      pf[a] += l[a];
    }
    if (dim == 2) {
      pt[0] += r[0] * l[1] - r[1] * l[0];
    } else {
      pt[0] += r[1] * l[2] - r[2] * l[1];
      pt[1] += r[2] * l[0] - r[0] * l[2];
      pt[2] += r[0] * l[1] - r[1] * l[0];
    }
  }
  for (int a = 0; a < 3; ++a) {
    f[a] = a < dim ? block_sum(pf[a], red) : 0.0;
    t[a] = (a < (dim == 3 ? 3 : 1)) ? block_sum(pt[a], red) : 0.0;
  }
}

template <typename TI>
__global__ void __launch_bounds__(256) k_free_body_rows(int dim, int nb, const int* __restrict__ off,
                                                        const double* __restrict__ R, const double* __restrict__ X,
                                                        double L, const int* __restrict__ free_b,
                                                        const double* __restrict__ lam, const TI* __restrict__ xu,
                                                        const TI* __restrict__ xo, double* __restrict__ yu,
                                                        double* __restrict__ yo) {
  __shared__ double red[256 / kWave];
  const int b = blockIdx.x;
  const int nr = dim == 3 ? 3 : 1;
  if (!free_b[b]) {
    if ((int)threadIdx.x < dim) yu[b * dim + threadIdx.x] = (double)xu[b * dim + threadIdx.x];
    if ((int)threadIdx.x < nr) yo[b * nr + threadIdx.x] = (double)xo[b * nr + threadIdx.x];
    return;
  }
  double f[3], t[3];
  body_sums(dim, off, R, X, L, lam, b, red, f, t);
  if ((int)threadIdx.x < dim) yu[b * dim + threadIdx.x] = f[threadIdx.x];
  if ((int)threadIdx.x < nr) yo[b * nr + threadIdx.x] = t[threadIdx.x];
}

// Per free body: Y = M~^-1 K (rows dim N_p, q = dim + rotations columns,
// row-major q wide at yoff[b]) and N~ = (K* Y)^-1 (q x q at b q^2).  M~^-1
// is the explicit symmetric inverse (row-major, leading dimension pad16).
// fail[b] = 1 when K* Y is not numerically positive definite.
template <int DIM>
__global__ void __launch_bounds__(256) k_free_setup(const int* __restrict__ off,
                                                    const int64_t* __restrict__ moff,
                                                    const double* __restrict__ Minv, const double* __restrict__ R,
                                                    const double* __restrict__ X, double L,
                                                    const int* __restrict__ free_b,
                                                    const int64_t* __restrict__ yoff, double* __restrict__ Y,
                                                    double* __restrict__ Nm, int* __restrict__ fail) {
  constexpr int dim = DIM;
  constexpr int q = DIM == 3 ? 6 : 3;
  __shared__ double red[256 / kWave];
  __shared__ double G[q * q];
  const int b = blockIdx.x;
  if (!free_b[b]) return;
  const int lo = off[b];
  const int n = dim * (off[b + 1] - lo);
  const int ld = pad16f(n);
  const double* Mi = Minv + moff[b];
  double* Yb = Y + yoff[b];
  double g[q * q];
#pragma unroll
  for (int e = 0; e < q * q; ++e) g[e] = 0.0;
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    double acc[q];
#pragma unroll
    for (int col = 0; col < q; ++col) acc[col] = 0.0;
    for (int i = 0; i < n / dim; ++i) {
      double r[3];
      rel_pos(dim, R, X, lo + i, b, L, r);
#pragma unroll
      for (int a = 0; a < dim; ++a) {
        // symmetric: column `row` read along c = i dim + a, coalesced over rows
        const double mv = Mi[(int64_t)(i * dim + a) * ld + row];
#pragma unroll
        for (int col = 0; col < q; ++col) acc[col] += mv * rigid_entry(dim, a, col, r);
      }
    }
#pragma unroll
    for (int col = 0; col < q; ++col) Yb[(int64_t)row * q + col] = acc[col];
    // this row's share of K* Y
    const int i = row / dim, a = row - i * dim;
    double r[3];
    rel_pos(dim, R, X, lo + i, b, L, r);
#pragma unroll
    for (int qa = 0; qa < q; ++qa) {
      const double k = rigid_entry(dim, a, qa, r);
#pragma unroll
      for (int qb = 0; qb < q; ++qb) g[qa * q + qb] += k * acc[qb];
    }
  }
#pragma unroll
  for (int e = 0; e < q * q; ++e) {
    const double s = block_sum(g[e], red);
    if (threadIdx.x == 0) G[e] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  // symmetrise, Cholesky G = C C^T, then N~ = G^-1 column by column
  double A[q * q], Cf[q * q];
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) A[i * q + j] = 0.5 * (G[i * q + j] + G[j * q + i]);
  bool ok = true;
  for (int j = 0; j < q && ok; ++j) {
    double s = A[j * q + j];
    for (int k = 0; k < j; ++k) s -= Cf[j * q + k] * Cf[j * q + k];
    if (!(s > 1e-14 * fabs(A[j * q + j])) || !(s > 0.0)) {
      ok = false;
      break;
    }
    const double dj = sqrt(s);
    Cf[j * q + j] = dj;
    for (int i = j + 1; i < q; ++i) {
      double t = A[i * q + j];
      for (int k = 0; k < j; ++k) t -= Cf[i * q + k] * Cf[j * q + k];
      Cf[i * q + j] = t / dj;
    }
  }
  fail[b] = ok ? 0 : 1;
  if (!ok) return;
  double* Nb = Nm + (int64_t)b * q * q;
  for (int col = 0; col < q; ++col) {
    double z[q];
    for (int i = 0; i < q; ++i) {  // C z = e_col
      double t = i == col ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= Cf[i * q + k] * z[k];
      z[i] = t / Cf[i * q + i];
    }
    for (int i = q - 1; i >= 0; --i) {  // C^T x = z
      double t = z[i];
      for (int k = i + 1; k < q; ++k) t -= Cf[k * q + i] * z[k];
      z[i] = t / Cf[i * q + i];
    }
    for (int i = 0; i < q; ++i) Nb[i * q + col] = z[i];
  }
}

// Per body: free -> U = N~ (r_U - K* lam), lam += Y U, z_U = U (lam holds
// M~^-1 dU on entry); prescribed -> z_U = r_U.
template <typename TZ>
__global__ void __launch_bounds__(256) k_free_precond(int dim, int nb, const int* __restrict__ off,
                                                      const double* __restrict__ R, const double* __restrict__ X,
                                                      double L, const int* __restrict__ free_b,
                                                      const int64_t* __restrict__ yoff, const double* __restrict__ Y,
                                                      const double* __restrict__ Nm, const double* __restrict__ ru,
                                                      const double* __restrict__ ro, double* __restrict__ lam,
                                                      TZ* __restrict__ zu, TZ* __restrict__ zo) {
  __shared__ double red[256 / kWave];
  __shared__ double Us[6];
  const int b = blockIdx.x;
  const int nr = dim == 3 ? 3 : 1;
  const int q = dim + nr;
  if (!free_b[b]) {
    if ((int)threadIdx.x < dim) zu[b * dim + threadIdx.x] = (TZ)ru[b * dim + threadIdx.x];
    if ((int)threadIdx.x < nr) zo[b * nr + threadIdx.x] = (TZ)ro[b * nr + threadIdx.x];
    return;
  }
  double f[3], t[3];
  body_sums(dim, off, R, X, L, lam, b, red, f, t);
  if (threadIdx.x == 0) {
    double rhs[6];
    for (int a = 0; a < dim; ++a) rhs[a] = ru[b * dim + a] - f[a];
    for (int a = 0; a < nr; ++a) rhs[dim + a] = ro[b * nr + a] - t[a];
    const double* Nb = Nm + (int64_t)b * q * q;
    for (int i = 0; i < q; ++i) {
      double s = 0.0;
      for (int k = 0; k < q; ++k) s += Nb[i * q + k] * rhs[k];
      Us[i] = s;
    }
  }
  __syncthreads();
  const int lo = off[b];
  const int n = dim * (off[b + 1] - lo);
  const double* Yb = Y + yoff[b];
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    double s = 0.0;
    for (int col = 0; col < q; ++col) s += Yb[(int64_t)row * q + col] * Us[col];
    lam[(int64_t)lo * dim + row] += s;
  }
  if ((int)threadIdx.x < dim) zu[b * dim + threadIdx.x] = (TZ)Us[threadIdx.x];
  if ((int)threadIdx.x < nr) zo[b * nr + threadIdx.x] = (TZ)Us[dim + threadIdx.x];
}

// Marker right-hand side W = 0 on the markers of free bodies.
__global__ void k_free_zero_markers(int dim, int N, const int* __restrict__ body, const int* __restrict__ free_b,
                                    double* __restrict__ W) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N || !free_b[body[m]]) return;
  for (int a = 0; a < dim; ++a) W[m * dim + a] = 0.0;
}

inline unsigned nblk_free(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename TI>
void launch_free_apply(int dim, int N, int nb, const int* off, const int* body, const double* R, const double* X,
                       double L, const int* free_b, const double* lam, const TI* xu, const TI* xo, double* yl,
                       double* yu, double* yo, hipStream_t s) {
  hipLaunchKernelGGL(k_free_rigid_add<TI>, dim3(nblk_free(N)), dim3(256), 0, s, dim, N, R, body, X, L, free_b, xu,
                     xo, yl);
  hipLaunchKernelGGL(k_free_body_rows<TI>, dim3(nb), dim3(256), 0, s, dim, nb, off, R, X, L, free_b, lam, xu, xo, yu,
                     yo);
}
template void launch_free_apply<double>(int, int, int, const int*, const int*, const double*, const double*, double,
                                        const int*, const double*, const double*, const double*, double*, double*,
                                        double*, hipStream_t);
template void launch_free_apply<float>(int, int, int, const int*, const int*, const double*, const double*, double,
                                       const int*, const double*, const float*, const float*, double*, double*,
                                       double*, hipStream_t);

void launch_free_setup(int dim, int nb, const int* off, const int64_t* moff, const double* Minv, const double* R,
                       const double* X, double L, const int* free_b, const int64_t* yoff, double* Y, double* Nm,
                       int* fail, hipStream_t s) {
  if (dim == 3)
    hipLaunchKernelGGL(k_free_setup<3>, dim3(nb), dim3(256), 0, s, off, moff, Minv, R, X, L, free_b, yoff, Y, Nm, fail);
  else
    hipLaunchKernelGGL(k_free_setup<2>, dim3(nb), dim3(256), 0, s, off, moff, Minv, R, X, L, free_b, yoff, Y, Nm, fail);
}

template <typename TZ>
void launch_free_precond(int dim, int nb, const int* off, const double* R, const double* X, double L,
                         const int* free_b, const int64_t* yoff, const double* Y, const double* Nm, const double* ru,
                         const double* ro, double* lam, TZ* zu, TZ* zo, hipStream_t s) {
  hipLaunchKernelGGL(k_free_precond<TZ>, dim3(nb), dim3(256), 0, s, dim, nb, off, R, X, L, free_b, yoff, Y, Nm, ru,
                     ro, lam, zu, zo);
}
template void launch_free_precond<double>(int, int, const int*, const double*, const double*, double, const int*,
                                          const int64_t*, const double*, const double*, const double*, const double*,
                                          double*, double*, double*, hipStream_t);
template void launch_free_precond<float>(int, int, const int*, const double*, const double*, double, const int*,
                                         const int64_t*, const double*, const double*, const double*, const double*,
                                         double*, float*, float*, hipStream_t);

void launch_free_zero_markers(int dim, int N, const int* body, const int* free_b, double* W, hipStream_t s) {
  hipLaunchKernelGGL(k_free_zero_markers, dim3(nblk_free(N)), dim3(256), 0, s, dim, N, body, free_b, W);
}

}  // namespace ibr
