// Multigrid V-cycle with no-slip walls at both ends of the last axis (z in
// 3D, y in 2D), periodic along the others: the slit channel of Sec. 7 with
// the boundary rules of the appendix on physical boundary conditions.
//
// Same cycle as the periodic one (red-black Gauss-Seidel, nu_pre sweeps from
// zero, residual restriction, rediscretised coarse operator c0 - (c1/4) L,
// prolongation, nu_post sweeps, nu_coarse sweeps on the 4^dim grid), with
// the walls' rules per field kind along the wall axis:
//   tangential velocity (cell-centred, mirror with the sign reversed) and the
//   pressure (cell-centred, mirror with the sign kept): a boundary cell's
//   ghost neighbour is the cell itself, so it moves into the diagonal
//   (c0 + (2 dim +- 1) c1); restriction averages the 2^dim children;
//   prolongation is multilinear (3/4, 1/4) with the ghost coarse value;
//   normal velocity (faces, the wall faces pinned to 0): vertex-centred along
//   the wall axis, so coarse face K sits on fine face 2K; restriction weights
//   the fine faces 2K-1, 2K, 2K+1 by 1/4, 1/2, 1/4 (and averages across the
//   periodic axes); prolongation copies coarse faces onto the even fine faces
//   and averages neighbours onto the odd ones (the wall faces get nothing).
// The singular Neumann problem (pressure, c0 = 0) loses the mean of its
// coarsest right-hand side; its finest right-hand side has zero mean when it
// is a divergence, as in P_S^-1.
//
// Fields are in split (red half, black half) storage like the periodic
// hierarchy; these kernels take one cell per thread and address neighbours
// through split_index: the walls change the stencil only in the two boundary
// layers, and the slit path is not the bandwidth-tuned periodic one.  From
// 4096 cells (16^3, 64^2) down, the cycle runs in one workgroup per field
// with the levels in LDS (k_wvcycle_lds), on the same per-cell steps.
#include "kernels.h"

namespace ibr {

namespace {

enum WallKind : int { kCellDir = 1, kFaceDir = 2, kCellNeu = 3 };

// mode 1: a velocity cycle (fields 0..dim-2 tangential, field dim-1 normal);
// mode 2: the pressure cycle (one Neumann field).
template <int DIM>
__device__ inline int wall_kind(int mode, int f) {
  return mode == 2 ? kCellNeu : (f == DIM - 1 ? kFaceDir : kCellDir);
}

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

// Cell of colour `color` with half-index t: natural coordinates.
template <int DIM>
__device__ inline void colour_cell(int t, int color, int logn, int& i, int& j, int& k) {
  const int hl = logn - 1;
  const int mask = (1 << logn) - 1;
  const int m = t & ((1 << hl) - 1);
  const int row = t >> hl;
  j = row & mask;
  k = DIM == 3 ? (row >> logn) : 0;
  i = 2 * m + ((color + j + k) & 1);
}

template <typename T, int DIM>
__device__ inline T at(const T* x, int i, int j, int k, int logn) {
  return x[split_index<DIM>(i, j, k, logn)];
}

// Sum of the neighbours that are other unknowns, and the diagonal of
// (c0 - c1 L) at cell (i, j, k); w is the wall-axis coordinate.
template <typename T, int DIM>
__device__ inline T nbr_sum(const T* x, int i, int j, int k, int logn, int kind, T c0, T c1, T& diag) {
  const int n = 1 << logn;
  const int w = DIM == 3 ? k : j;
  diag = c0 + T(2 * DIM) * c1;
  const T s = kind == kCellDir ? T(1) : T(-1);
  T up = T(0), dn = T(0);
  if (DIM == 3) {
    if (kind == kFaceDir) {
      up = w + 1 < n ? at<T, DIM>(x, i, j, k + 1, logn) : T(0);
      dn = at<T, DIM>(x, i, j, k - 1, logn);
    } else {
      if (w + 1 < n) up = at<T, DIM>(x, i, j, k + 1, logn); else diag += s * c1;
      if (w > 0) dn = at<T, DIM>(x, i, j, k - 1, logn); else diag += s * c1;
    }
  } else {
    if (kind == kFaceDir) {
      up = w + 1 < n ? at<T, DIM>(x, i, j + 1, k, logn) : T(0);
      dn = at<T, DIM>(x, i, j - 1, k, logn);
    } else {
      if (w + 1 < n) up = at<T, DIM>(x, i, j + 1, k, logn); else diag += s * c1;
      if (w > 0) dn = at<T, DIM>(x, i, j - 1, k, logn); else diag += s * c1;
    }
  }
  T sum = up + dn;
  if (DIM == 3) sum += at<T, DIM>(x, i, j + 1, k, logn) + at<T, DIM>(x, i, j - 1, k, logn);
  sum += at<T, DIM>(x, i + 1, j, k, logn) + at<T, DIM>(x, i - 1, j, k, logn);
  return sum;
}

template <typename T, int DIM>
__device__ inline T resid_at(const T* x, const T* b, int i, int j, int k, int logn, int kind, T c0, T c1) {
  const int w = DIM == 3 ? k : j;
  if (kind == kFaceDir && w == 0) return T(0);
  T diag;
  const T sum = nbr_sum<T, DIM>(x, i, j, k, logn, kind, c0, c1, diag);
  return at<T, DIM>(b, i, j, k, logn) - (diag * at<T, DIM>(x, i, j, k, logn) - c1 * sum);
}

// ---- per-cell steps (global kernels: one cell per thread; the tail: loops)
// Half sweep at cell t of colour `color`.
template <typename T, int DIM>
__device__ inline void wrb_cell(T* x, const T* b, int logn, T c0, T c1, int color, int t, int kind) {
  const int C = 1 << (DIM * logn);
  int i, j, k;
  colour_cell<DIM>(t, color, logn, i, j, k);
  const int own = color * (C >> 1) + t;
  const int w = DIM == 3 ? k : j;
  if (kind == kFaceDir && w == 0) {
    x[own] = T(0);
    return;
  }
  T diag;
  const T sum = nbr_sum<T, DIM>(x, i, j, k, logn, kind, c0, c1, diag);
  x[own] = (b[own] + c1 * sum) / diag;
}

// Coarse right-hand side of coarse cell t (natural index) from the fine
// residual: its split index on the coarse level is returned in *at_c.
template <typename T, int DIM>
__device__ inline T wrestrict_cell(const T* x, const T* b, int logn, T c0, T c1, int t, int kind, int* at_c) {
  const int lognc = logn - 1;
  const int maskc = (1 << lognc) - 1;
  const int I = t & maskc, J = (t >> lognc) & maskc, K = DIM == 3 ? (t >> (2 * lognc)) : 0;
  const int W = DIM == 3 ? K : J;
  *at_c = split_index<DIM>(I, J, K, lognc);
  T out = T(0);
  if (kind == kFaceDir) {
    if (W > 0) {
      // full weighting along the wall axis over fine faces 2W-1, 2W, 2W+1; average across
      const T wz[3] = {T(0.25), T(0.5), T(0.25)};
      for (int q = 0; q < 3; ++q) {
        const int wf = 2 * W - 1 + q;
        T acc = T(0);
        if (DIM == 3) {
          for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
              acc += resid_at<T, DIM>(x, b, 2 * I + dx, 2 * J + dy, wf, logn, kind, c0, c1);
          acc *= T(0.25);
        } else {
          for (int dx = 0; dx < 2; ++dx) acc += resid_at<T, DIM>(x, b, 2 * I + dx, wf, 0, logn, kind, c0, c1);
          acc *= T(0.5);
        }
        out += wz[q] * acc;
      }
    }
  } else {
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          out += resid_at<T, DIM>(x, b, 2 * I + dx, 2 * J + dy, 2 * K + dz, logn, kind, c0, c1);
    out *= DIM == 3 ? T(0.125) : T(0.25);
  }
  return out;
}

// Coarse value used by the prolongation at coarse wall-axis index Wn (may be
// one beyond the lattice: the ghost), periodic axes already chosen.
template <typename T, int DIM>
__device__ inline T coarse_at(const T* e, int I, int J, int Wn, int Wp, int lognc, int kind) {
  const int nc = 1 << lognc;
  int Wu = Wn;
  T s = T(1);
  if (Wn < 0 || Wn >= nc) {
    if (kind == kFaceDir) return T(0);  // the wall face (only Wn == nc arises)
    Wu = Wp;
    s = kind == kCellDir ? T(-1) : T(1);
  }
  return DIM == 3 ? s * at<T, DIM>(e, I, J, Wu, lognc) : s * at<T, DIM>(e, I, Wu, 0, lognc);
}

// x += P e at fine cell t (natural index).
template <typename T, int DIM>
__device__ inline void wprolong_cell(T* x, const T* e, int logn, int t, int kind) {
  const int lognc = logn - 1;
  const int mask = (1 << logn) - 1;
  const int i = t & mask, j = (t >> logn) & mask, k = DIM == 3 ? (t >> (2 * logn)) : 0;
  const int w = DIM == 3 ? k : j;
  if (kind == kFaceDir && w == 0) return;
  // periodic axes: cell-centred 3/4, 1/4
  const int I = i >> 1, In = (i & 1) ? I + 1 : I - 1;
  int J = 0, Jn = 0;
  if (DIM == 3) {
    J = j >> 1;
    Jn = (j & 1) ? J + 1 : J - 1;
  }
  // wall axis: two coarse indices and their weights
  int W0, W1;
  T a0, a1;
  const int Wp = w >> 1;
  if (kind == kFaceDir) {
    W0 = Wp;
    W1 = Wp + 1;
    a0 = (w & 1) ? T(0.5) : T(1);
    a1 = (w & 1) ? T(0.5) : T(0);
  } else {
    W0 = Wp;
    W1 = (w & 1) ? Wp + 1 : Wp - 1;
    a0 = T(0.75);
    a1 = T(0.25);
  }
  T val = T(0);
  for (int q = 0; q < 2; ++q) {
    const int Wq = q == 0 ? W0 : W1;
    const T aq = q == 0 ? a0 : a1;
    if (aq == T(0)) continue;
    T plane;
    if (DIM == 3) {
      const T r0 = T(0.75) * coarse_at<T, DIM>(e, I, J, Wq, Wp, lognc, kind) +
                   T(0.25) * coarse_at<T, DIM>(e, In, J, Wq, Wp, lognc, kind);
      const T r1 = T(0.75) * coarse_at<T, DIM>(e, I, Jn, Wq, Wp, lognc, kind) +
                   T(0.25) * coarse_at<T, DIM>(e, In, Jn, Wq, Wp, lognc, kind);
      plane = T(0.75) * r0 + T(0.25) * r1;
    } else {
      plane = T(0.75) * coarse_at<T, DIM>(e, I, 0, Wq, Wp, lognc, kind) +
              T(0.25) * coarse_at<T, DIM>(e, In, 0, Wq, Wp, lognc, kind);
    }
    val += aq * plane;
  }
  x[split_index<DIM>(i, j, k, logn)] += val;
}

// ---- global kernels: fields in blockIdx.y
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wrb(T* __restrict__ x, const T* __restrict__ b, int logn, T c0, T c1,
                                             int color, int mode) {
  const int C = 1 << (DIM * logn);
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= (C >> 1)) return;
  const int f = blockIdx.y;
  wrb_cell<T, DIM>(x + (int64_t)f * C, b + (int64_t)f * C, logn, c0, c1, color, t, wall_kind<DIM>(mode, f));
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wresid_restrict(const T* __restrict__ x, const T* __restrict__ b,
                                                         T* __restrict__ bc, int logn, T c0, T c1, int mode) {
  const int C = 1 << (DIM * logn), Cc = C >> DIM;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= Cc) return;
  const int f = blockIdx.y;
  int at_c;
  const T r = wrestrict_cell<T, DIM>(x + (int64_t)f * C, b + (int64_t)f * C, logn, c0, c1, t,
                                     wall_kind<DIM>(mode, f), &at_c);
  bc[(int64_t)f * Cc + at_c] = r;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wprolong(T* __restrict__ x, const T* __restrict__ e, int logn, int mode) {
  const int C = 1 << (DIM * logn), Cc = C >> DIM;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= C) return;
  const int f = blockIdx.y;
  wprolong_cell<T, DIM>(x + (int64_t)f * C, e + (int64_t)f * Cc, logn, t, wall_kind<DIM>(mode, f));
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

template <typename T, int DIM>
__global__ void __launch_bounds__(kWallTailThreads) k_wvcycle_lds(const T* __restrict__ bg, T* __restrict__ xg,
                                                                  int logn, T c0, T c1, int nu_pre, int nu_post,
                                                                  int nu_coarse, int mode) {
  constexpr int kX = wall_pyramid<DIM>(kWallTailCells);
  constexpr int kB = wall_pyramid<DIM>(kWallTailCells >> DIM) + 1;
  __shared__ T xs[kX];
  __shared__ T bs[kB];
  __shared__ T red[kWallTailThreads / kWave];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int f = blockIdx.x;
  const int kind = wall_kind<DIM>(mode, f);
  const int C0 = 1 << (DIM * logn);
  const T* b0 = bg + (int64_t)f * C0;
  T* x0 = xg + (int64_t)f * C0;
  const int nlev = logn - 1;  // entry level down to n = 4
  int off[12], boff[12];
  {
    int xo = 0, bo = 0;
    for (int l = 0; l < nlev; ++l) {
      const int Cl = 1 << (DIM * (logn - l));
      off[l] = xo;
      xo += Cl;
      boff[l] = bo;
      if (l > 0) bo += Cl;
    }
  }
  auto bl = [&](int l) -> const T* { return l == 0 ? b0 : bs + boff[l]; };
  T cl = c1;
  auto sweeps = [&](int l, T cc, int nsw) {
    const int lg = logn - l;
    const int H = 1 << (DIM * lg - 1);
    for (int sw = 0; sw < nsw; ++sw)
      for (int color = 0; color < 2; ++color) {
        for (int t = tid; t < H; t += nt) wrb_cell<T, DIM>(xs + off[l], bl(l), lg, c0, cc, color, t, kind);
        __syncthreads();
      }
  };
  for (int l = 0; l < nlev - 1; ++l) {
    const int lg = logn - l;
    const int Cl = 1 << (DIM * lg);
    for (int c = tid; c < Cl; c += nt) xs[off[l] + c] = T(0);
    __syncthreads();
    sweeps(l, cl, nu_pre);
    for (int t = tid; t < (Cl >> DIM); t += nt) {
      int at_c;
      const T r = wrestrict_cell<T, DIM>(xs + off[l], bl(l), lg, c0, cl, t, kind, &at_c);
      bs[boff[l + 1] + at_c] = r;
    }
    __syncthreads();
    cl = cl * T(0.25);
  }
  {
    const int l = nlev - 1;
    const int Cl = 1 << (DIM * (logn - l));
    if (mode == 2 && c0 == T(0)) {
      // the singular Neumann problem: the coarsest right-hand side loses its mean
      T* b = bs + boff[l];
      T sm = T(0);
      for (int c = tid; c < Cl; c += nt) sm += b[c];
      sm = block_sum(sm, red);
      const T mean = sm / T(Cl);
      __syncthreads();
      for (int c = tid; c < Cl; c += nt) b[c] -= mean;
    }
    for (int c = tid; c < Cl; c += nt) xs[off[l] + c] = T(0);
    __syncthreads();
    sweeps(l, cl, nu_coarse);
  }
  for (int l = nlev - 2; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const int Cl = 1 << (DIM * lg);
    for (int t = tid; t < Cl; t += nt) wprolong_cell<T, DIM>(xs + off[l], xs + off[l + 1], lg, t, kind);
    __syncthreads();
    sweeps(l, cl, nu_post);
  }
  for (int c = tid; c < C0; c += nt) x0[c] = xs[c];
}

}  // namespace

template <typename T>
void launch_wall_vcycle(int dim, int logn, int nf, const T* b, T* x, const std::vector<T*>& wx,
                        const std::vector<T*>& wb, double c0, double c1, int nu_pre, int nu_post, int nu_coarse,
                        int mode, hipStream_t s) {
  if (logn < 3) throw DeviceError("walls: grids need n >= 8");
  // levels above the tail run the global kernels; the tail starts at <= kWallTailCells cells
  int lt = 0;
  while (((int64_t)1 << (dim * (logn - lt))) > kWallTailCells) ++lt;
  if ((int)wx.size() <= lt || (int)wb.size() <= lt) throw DeviceError("walls: multigrid buffers missing");
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
                            mode);
    else
      hipExtLaunchKernelGGL(k_wrb<T, 2>, g, dim3(256), 0, s, ev.start, ev.stop, 0, xl(l), bl(l), lg, tc0, cl, color,
                            mode);
  };
  for (int l = 0; l < lt; ++l) {
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    launch_fill<T>(xl(l), Cl * nf, T(0), s);
    for (int sw = 0; sw < nu_pre; ++sw)
      for (int color = 0; color < 2; ++color) half(l, color);
    const dim3 g(nblk(Cl >> dim), nf);
    if (three)
      hipLaunchKernelGGL((k_wresid_restrict<T, 3>), g, dim3(256), 0, s, xl(l), bl(l), wb[l + 1], lg, tc0, cl, mode);
    else
      hipLaunchKernelGGL((k_wresid_restrict<T, 2>), g, dim3(256), 0, s, xl(l), bl(l), wb[l + 1], lg, tc0, cl, mode);
    cl = cl * T(0.25);
  }
  if (three)
    hipLaunchKernelGGL((k_wvcycle_lds<T, 3>), dim3(nf), dim3(kWallTailThreads), 0, s, bl(lt), xl(lt), logn - lt,
                       tc0, cl, nu_pre, nu_post, nu_coarse, mode);
  else
    hipLaunchKernelGGL((k_wvcycle_lds<T, 2>), dim3(nf), dim3(kWallTailThreads), 0, s, bl(lt), xl(lt), logn - lt,
                       tc0, cl, nu_pre, nu_post, nu_coarse, mode);
  for (int l = lt - 1; l >= 0; --l) {
    cl = cl * T(4);
    const int lg = logn - l;
    const int64_t Cl = (int64_t)1 << (dim * lg);
    const dim3 g(nblk(Cl), nf);
    if (three)
      hipLaunchKernelGGL((k_wprolong<T, 3>), g, dim3(256), 0, s, xl(l), (const T*)xl(l + 1), lg, mode);
    else
      hipLaunchKernelGGL((k_wprolong<T, 2>), g, dim3(256), 0, s, xl(l), (const T*)xl(l + 1), lg, mode);
    for (int sw = 0; sw < nu_post; ++sw)
      for (int color = 0; color < 2; ++color) half(l, color);
  }
}

template void launch_wall_vcycle<double>(int, int, int, const double*, double*, const std::vector<double*>&,
                                         const std::vector<double*>&, double, double, int, int, int, int,
                                         hipStream_t);
template void launch_wall_vcycle<float>(int, int, int, const float*, float*, const std::vector<float*>&,
                                        const std::vector<float*>&, double, double, int, int, int, int,
                                        hipStream_t);

}  // namespace ibr
