// Krylov building blocks (Sec. 5): block Gram-Schmidt passes, norms, basis
// combination and the Givens-rotation Hessenberg least squares of GMRES.
// All reductions are two-pass with a fixed partition, so results are
// bitwise reproducible run to run.
#include "kernels.h"

namespace ibr {

namespace {

constexpr int kDotCols = 8;  // basis vectors per multi-dot block

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

// part[j * nblocks + block] = partial <w, V_j> for j in this block's column chunk.
template <typename TV, typename TW>
__global__ void __launch_bounds__(256) k_multi_dot(const TV* __restrict__ V, int64_t ld, int k,
                                                   const TW* __restrict__ w, int64_t len, double* __restrict__ part) {
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
  if (threadIdx.x < nj) {
    double s = 0;
    for (int u = 0; u < (int)(blockDim.x / kWave); ++u) s += red[threadIdx.x][u];
    part[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_dot_finish(const double* __restrict__ part, int nblocks, double* __restrict__ h, int accumulate) {
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
                                                    double* __restrict__ norm_part) {
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
                                                 const double* __restrict__ y, TX* __restrict__ x, int64_t len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    double acc = (double)x[i];
    for (int j = 0; j < k; ++j) acc += y[j] * (double)Z[(int64_t)j * ld + i];
    x[i] = (TX)acc;
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
                      double* h, bool accumulate, hipStream_t s) {
  if (k <= 0) return;
  const int nchunk = (k + kDotCols - 1) / kDotCols;
  hipLaunchKernelGGL((k_multi_dot<TV, TW>), dim3(nblocks, nchunk), dim3(256), 0, s, V, ld, k, w, len, part);
  hipLaunchKernelGGL(k_dot_finish, dim3(k), dim3(256), 0, s, part, nblocks, h, accumulate ? 1 : 0);
}
template void launch_multi_dot<double, double>(const double*, int64_t, int, const double*, int64_t, double*, int,
                                               double*, bool, hipStream_t);
template void launch_multi_dot<float, float>(const float*, int64_t, int, const float*, int64_t, double*, int,
                                             double*, bool, hipStream_t);

template <typename TV, typename TW>
void launch_multi_axpy(const TV* V, int64_t ld, int k, const double* h, TW* w, int64_t len, double* norm_part,
                       int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_multi_axpy<TV, TW>), dim3(nblocks), dim3(256), 0, s, V, ld, k, h, w, len, norm_part);
}
template void launch_multi_axpy<double, double>(const double*, int64_t, int, const double*, double*, int64_t,
                                                double*, int, hipStream_t);
template void launch_multi_axpy<float, float>(const float*, int64_t, int, const double*, float*, int64_t, double*,
                                              int, hipStream_t);

template <typename TZ, typename TX>
void launch_combine(const TZ* Z, int64_t ld, int k, const double* y, TX* x, int64_t len, hipStream_t s) {
  if (k <= 0) return;
  unsigned g = nblk(len);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL((k_combine<TZ, TX>), dim3(g), dim3(256), 0, s, Z, ld, k, y, x, len);
}
template void launch_combine<double, double>(const double*, int64_t, int, const double*, double*, int64_t,
                                             hipStream_t);
template void launch_combine<float, double>(const float*, int64_t, int, const double*, double*, int64_t,
                                            hipStream_t);
template void launch_combine<float, float>(const float*, int64_t, int, const double*, float*, int64_t,
                                           hipStream_t);

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
