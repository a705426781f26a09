// Fluid-marker coupling (Sec. 3.1): interpolation J, spreading S, marker
// binning, rigid-body kinematics and body force / torque sums (Sec. 2).
//
// Spreading is a deterministic, atomic-free GATHER: markers are binned by the
// 8^3 (2D: 16^2) tile that holds their cell; one workgroup owns one active
// tile and component, walks the markers of the neighbouring tiles in a fixed
// order and accumulates their taps into its own faces.  Interpolation gives one
// wavefront to each marker: 64 lanes = the 4^3 taps, reduced with shuffles.
#include "kernels.h"

namespace ibr {

namespace {

inline unsigned nblk(int64_t len, int bs = 256) { return (unsigned)((len + bs - 1) / bs); }

__device__ inline int tap_base_index(int m, int s, int beta) { return (m * 2 + s) * 3 + beta; }

// ---------------------------------------------------------------- marker set-up
// walls (bit beta = no-slip walls at both ends of axis beta): along a walled
// axis the taps beyond a wall fold back onto
// their mirror images with the sign reversed and taps on the wall faces of
// the normal component are dropped (J = J0 E, S = E^T S0 with the extension
// E of the appendix on physical boundary conditions); the folded taps are
// kept as 4 consecutive points inside the lattice, so interpolation and
// spreading use them unchanged.
__device__ inline void fold_wall_taps(int& b0, double* w, int n, bool face) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int nb0 = b0 < 0 ? 0 : (b0 > n - 4 ? n - 4 : b0);
  for (int t = 0; t < 4; ++t) {
    int j = b0 + t;
    double wt = w[t];
    if (face) {
      if (j == 0 || j == n) continue;
      if (j < 0) {
        j = -j;
        wt = -wt;
      } else if (j > n) {
        j = 2 * n - j;
        wt = -wt;
      }
    } else {
      if (j < 0) {
        j = -1 - j;
        wt = -wt;
      } else if (j >= n) {
        j = 2 * n - 1 - j;
        wt = -wt;
      }
    }
    acc[j - nb0] += wt;
  }
  b0 = nb0;
  for (int t = 0; t < 4; ++t) w[t] = acc[t];
}

__global__ void k_marker_setup(int dim, int logn, int N, double h, double L, const double* __restrict__ R,
                               int* __restrict__ base, double* __restrict__ w64, float* __restrict__ w32,
                               int* __restrict__ tile_of, int tile_log, int walls) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int n = 1 << logn;
  const int nt_log = logn - tile_log;
  int tile = 0;
  for (int beta = dim - 1; beta >= 0; --beta) {
    double x = R[m * dim + beta];
    x = x - L * floor(x / L);
    for (int s = 0; s < 2; ++s) {
      const double sc = x / h - (s == 0 ? 0.5 : 0.0);
      const double fl = floor(sc);
      int b0 = (int)fl - 1;
      const int bi = tap_base_index(m, s, beta);
      double w[4];
      for (int t = 0; t < 4; ++t) w[t] = phi4<double>(sc - (double)(b0 + t));
      if ((walls >> beta) & 1) fold_wall_taps(b0, w, n, s == 1);
      base[bi] = b0;
      for (int t = 0; t < 4; ++t) {
        w64[bi * 4 + t] = w[t];
        w32[bi * 4 + t] = (float)w[t];
      }
    }
    const int cell = ((int)floor(x / h)) & (n - 1);
    tile = (tile << nt_log) | (cell >> tile_log);
  }
  tile_of[m] = tile;
}

__global__ void k_marker_velocity(int dim, int N, const double* __restrict__ R, const int* __restrict__ body,
                                  const double* __restrict__ X, const double* __restrict__ U,
                                  const double* __restrict__ Om, double L, double* __restrict__ V) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int b = body[m];
  double r[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) {
    double d = R[m * dim + a] - X[b * dim + a];
    d -= L * rint(d / L);
    r[a] = d;
  }
  if (dim == 2) {
    const double w = Om[b];
    V[m * 2 + 0] = U[b * 2 + 0] - w * r[1];
    V[m * 2 + 1] = U[b * 2 + 1] + w * r[0];
  } else {
    const double* w = Om + 3 * b;
    V[m * 3 + 0] = U[b * 3 + 0] + (w[1] * r[2] - w[2] * r[1]);
    V[m * 3 + 1] = U[b * 3 + 1] + (w[2] * r[0] - w[0] * r[2]);
    V[m * 3 + 2] = U[b * 3 + 2] + (w[0] * r[1] - w[1] * r[0]);
  }
}

__global__ void k_move_markers(int dim, int N, int nb, double* __restrict__ R, double* __restrict__ X,
                               const int* __restrict__ body, const double* __restrict__ U, double dt, double L) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) {
    const int b = body[t];
    for (int a = 0; a < dim; ++a) {
      double x = R[t * dim + a] + dt * U[b * dim + a];
      R[t * dim + a] = x - L * floor(x / L);
    }
  } else if (t < N + nb) {
    const int b = t - N;
    for (int a = 0; a < dim; ++a) {
      double x = X[b * dim + a] + dt * U[b * dim + a];
      X[b * dim + a] = x - L * floor(x / L);
    }
  }
}

// ---------------------------------------------------------------- binning
__global__ void k_bin_count(int N, const int* __restrict__ tile_of, int* __restrict__ counts) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) atomicAdd(&counts[tile_of[m]], 1);
}

// Exclusive scan of counts[0..n) into off[0..n], single workgroup of 1024.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ counts, int n, int* __restrict__ off) {
  __shared__ int sums[1024];
  const int tid = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = tid * chunk;
  const int hi = min(n, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  sums[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int v = tid >= d ? sums[tid - d] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int run = sums[tid] - s;
  for (int i = lo; i < hi; ++i) {
    off[i] = run;
    run += counts[i];
  }
  if (tid == 1023) off[n] = sums[1023];
}

__global__ void k_bin_scatter(int N, const int* __restrict__ tile_of, const int* __restrict__ off,
                              int* __restrict__ cursor, int* __restrict__ perm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int t = tile_of[m];
  const int pos = off[t] + atomicAdd(&cursor[t], 1);
  perm[pos] = m;
}

// Sort each tile's segment by marker index (fixed order => deterministic
// sums).  One workgroup per tile: the segment is copied into LDS and each
// entry goes to its rank (the count of smaller indices; marker indices are
// distinct).  A segment longer than the LDS copy (only markers packed far
// more densely than a kernel width apart make one) is sorted by insertion
// in place by one thread.
constexpr int kSortThreads = 128;
constexpr int kSortLds = 2048;
__global__ void __launch_bounds__(kSortThreads) k_bin_sort(const int* __restrict__ off, int* __restrict__ perm) {
  __shared__ int seg[kSortLds];
  const int t = blockIdx.x;
  const int lo = off[t], n = off[t + 1] - lo;
  if (n <= 1) return;
  if (n > kSortLds) {
    if (threadIdx.x == 0)
      for (int i = lo + 1; i < lo + n; ++i) {
        const int v = perm[i];
        int j = i - 1;
        while (j >= lo && perm[j] > v) {
          perm[j + 1] = perm[j];
          --j;
        }
        perm[j + 1] = v;
      }
    return;
  }
  for (int i = threadIdx.x; i < n; i += kSortThreads) seg[i] = perm[lo + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kSortThreads) {
    const int v = seg[i];
    int r = 0;
    for (int j = 0; j < n; ++j) r += seg[j] < v ? 1 : 0;
    perm[lo + r] = v;
  }
}

// Distinct neighbour tile coordinates along one axis (1, 2 or 3 of them).
__device__ inline int nbr_coords(int t, int nt, int* out) {
  if (nt == 1) {
    out[0] = 0;
    return 1;
  }
  if (nt == 2) {
    out[0] = t;
    out[1] = t ^ 1;
    return 2;
  }
  out[0] = (t - 1 + nt) % nt;
  out[1] = t;
  out[2] = (t + 1) % nt;
  return 3;
}

__global__ void k_active_tiles(int dim, int tiles_log, const int* __restrict__ off, int* __restrict__ flags,
                               int* __restrict__ list, int* __restrict__ count) {
  const int nt = 1 << tiles_log;
  const int ntiles = 1 << (dim * tiles_log);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int tc[3] = {t & (nt - 1), (t >> tiles_log) & (nt - 1), dim == 3 ? (t >> (2 * tiles_log)) : 0};
  int cx[3], cy[3], cz[3];
  const int nx = nbr_coords(tc[0], nt, cx);
  const int ny = nbr_coords(tc[1], nt, cy);
  const int nz = dim == 3 ? nbr_coords(tc[2], nt, cz) : 1;
  if (dim == 2) cz[0] = 0;
  int any = 0;
  for (int a = 0; a < nz; ++a)
    for (int b = 0; b < ny; ++b)
      for (int c = 0; c < nx; ++c) {
        const int tt = cx[c] | (cy[b] << tiles_log) | (cz[a] << (2 * tiles_log));
        if (off[tt + 1] > off[tt]) any = 1;
      }
  flags[t] = any;
  if (any) {
    const int pos = atomicAdd(count, 1);
    list[pos] = t;
  }
}

// ---------------------------------------------------------------- spreading (gather)
// One workgroup of four wavefronts per (active tile, component a).  The
// candidate markers (those binned in the neighbouring tiles, tiles in a fixed
// order, markers sorted inside each tile) are taken kChunk at a time: each
// thread tests one candidate against the tile and the hits are compacted, in
// order, into LDS with their first taps and weights (lam folded into the x
// weights).  A chunk of 192 covers the neighbourhood of a tile of spheres at
// a marker spacing of about 2h in one pass and keeps the workgroup's LDS
// under 40 KB, so four workgroups share a compute unit; the tile's own
// values of y are loaded at the start, while the candidates are gathered.
// Wavefront w then takes hits w, w+4, ...; for one marker its 64 lanes are the
// 4^3 taps (distinct faces) and add into that wavefront's own accumulator.  The
// four accumulators are summed in a fixed order at the end: no atomics, and
// the result is bitwise reproducible.  2D uses 16 lanes per marker.
template <typename TL, typename TY, int DIM, bool SPLIT>
__global__ void __launch_bounds__(256) k_spread(int logn, int tile_log, const int* __restrict__ active,
                                                const int* __restrict__ nactive, const int* __restrict__ off,
                                                const int* __restrict__ perm, const int* __restrict__ tbase,
                                                const double* __restrict__ tw, const TL* __restrict__ lam,
                                                TY* __restrict__ y, double scale) {
  if ((int)blockIdx.x >= nactive[0]) return;  // grid sized to a capacity, count read on the device
  constexpr int kCells = DIM == 3 ? 512 : 256;  // 8^3 or 16^2
  constexpr int kWaves = 4;
  constexpr int kChunk = 192;
  constexpr int kPer = kCells / 256;  // cells of the tile per thread
  __shared__ double acc[kWaves][kCells];
  __shared__ double sw[kChunk][DIM][4];
  __shared__ int sd[kChunk][DIM];
  __shared__ int rlo[27], rpre[28];  // first candidate of neighbour tile r; prefix sums of their counts
  __shared__ int wcnt[kWaves];

  const int n = 1 << logn;
  const int mask = n - 1;
  const int64_t C = (int64_t)1 << (DIM * logn);
  const int tiles_log = logn - tile_log;
  const int nt = 1 << tiles_log;
  const int tile = active[blockIdx.x];
  const int a = blockIdx.y;
  const int tsz = 1 << tile_log;
  const int tc[3] = {tile & (nt - 1), (tile >> tiles_log) & (nt - 1), DIM == 3 ? (tile >> (2 * tiles_log)) : 0};
  const int lo[3] = {tc[0] * tsz, tc[1] * tsz, tc[2] * tsz};
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int cells = 1 << (DIM * tile_log);
  // this thread's cells of the tile: their indices in y and their old values
  int64_t yidx[kPer];
  TY yold[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int q = tid + 256 * u;
    const int l0 = q & (tsz - 1), l1 = (q >> tile_log) & (tsz - 1), l2 = DIM == 3 ? (q >> (2 * tile_log)) : 0;
    const int64_t c = SPLIT ? (int64_t)split_index<DIM>(lo[0] + l0, lo[1] + l1, lo[2] + l2, logn)
                            : (int64_t)natural_index<DIM>(lo[0] + l0, lo[1] + l1, lo[2] + l2, logn);
    yidx[u] = q < cells ? (int64_t)a * C + c : -1;
    yold[u] = q < cells ? y[yidx[u]] : TY(0);
  }
  for (int q = tid; q < kWaves * kCells; q += 256) (&acc[0][0])[q] = 0.0;
  {
    // neighbour tile r (in a fixed order) fetched by thread r
    int cx[3], cy[3], cz[3];
    const int nx = nbr_coords(tc[0], nt, cx);
    const int ny = nbr_coords(tc[1], nt, cy);
    int nz = 1;
    cz[0] = 0;
    if (DIM == 3) nz = nbr_coords(tc[2], nt, cz);
    if (wave == 0) {
      int lo_r = 0, len = 0;
      if (lane < nx * ny * nz) {
        const int c3 = lane % nx, b3 = (lane / nx) % ny, a3 = lane / (nx * ny);
        const int tt = cx[c3] | (cy[b3] << tiles_log) | (cz[a3] << (2 * tiles_log));
        lo_r = off[tt];
        len = off[tt + 1] - lo_r;
      }
      // inclusive scan of the lengths over the wavefront's first 32 lanes
      int incl = len;
#pragma unroll
      for (int o = 1; o < 32; o <<= 1) {
        const int t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
      }
      if (lane < 27) {
        rlo[lane] = lo_r;
        rpre[lane + 1] = incl;
      }
      if (lane == 0) rpre[0] = 0;
    }
  }
  __syncthreads();
  const int total = rpre[27];
  // lane -> tap offsets (x fastest)
  const int tx = lane & 3, ty = (lane >> 2) & 3, tz = lane >> 4;
  const bool live = DIM == 3 || lane < 16;

  for (int c0 = 0; c0 < total; c0 += kChunk) {
    const int q = c0 + tid;
    bool hit = false;
    int m = 0, d[3] = {0, 0, 0};
    double lm = 0.0, wv[DIM][4];
    if (tid < kChunk && q < total) {
      // neighbour tile of candidate q: rpre[r] <= q < rpre[r + 1] (rpre[27] = total > q)
      int r = 0, rh = 27;
      while (rh - r > 1) {
        const int mid = (r + rh) >> 1;
        if (rpre[mid] <= q)
          r = mid;
        else
          rh = mid;
      }
      m = perm[rlo[r] + (q - rpre[r])];
      hit = true;
      // the candidate's weights and force are loaded with its taps, whether it hits or not
      lm = (double)lam[m * DIM + a];
      for (int beta = 0; beta < DIM; ++beta) {
        const int s = beta == a ? 1 : 0;
        d[beta] = (tbase[(m * 2 + s) * 3 + beta] - lo[beta]) & mask;
        const double* wp = tw + ((m * 2 + s) * 3 + beta) * 4;
        for (int t = 0; t < 4; ++t) wv[beta][t] = wp[t];
        // the 4 taps along beta meet the tile when the first one is within [-3, tsz)
        hit = hit && (d[beta] < tsz || d[beta] >= n - 3);
      }
    }
    const unsigned long long bal = __ballot(hit);
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int base = 0, nhit = 0;
    for (int w = 0; w < kWaves; ++w) {
      base += w < wave ? wcnt[w] : 0;
      nhit += wcnt[w];
    }
    if (hit) {
      const int slot = base + rank;
      for (int beta = 0; beta < DIM; ++beta) {
        sd[slot][beta] = d[beta];
        for (int t = 0; t < 4; ++t) sw[slot][beta][t] = beta == 0 ? lm * wv[beta][t] : wv[beta][t];
      }
    }
    __syncthreads();
    if (live) {
      for (int j = wave; j < nhit; j += kWaves) {
        const int f0 = (sd[j][0] + tx) & mask;
        const int f1 = (sd[j][1] + ty) & mask;
        int f2 = 0;
        if constexpr (DIM == 3) f2 = (sd[j][2] + tz) & mask;
        if (f0 < tsz && f1 < tsz && f2 < tsz) {
          double w = sw[j][0][tx] * sw[j][1][ty];
          if constexpr (DIM == 3) w *= sw[j][2][tz];
          acc[wave][f0 + (f1 << tile_log) + (f2 << (2 * tile_log))] += w;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int q = tid + 256 * u;
    if (yidx[u] < 0) continue;
    const double v = ((acc[0][q] + acc[1][q]) + acc[2][q]) + acc[3][q];
    y[yidx[u]] = (TY)((double)yold[u] + scale * v);
  }
}

// ---------------------------------------------------------------- interpolation
template <typename TV>
__global__ void __launch_bounds__(256) k_interp(int dim, int logn, int N, const int* __restrict__ tbase,
                                                const double* __restrict__ tw, const TV* __restrict__ v,
                                                double alpha, const double* __restrict__ add, double beta,
                                                double* __restrict__ out, const double* __restrict__ vshift) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (wave >= N) return;
  const int m = wave;
  const int n = 1 << logn;
  const int64_t C = (int64_t)1 << (dim * logn);
  const int tx = lane & 3, ty = (lane >> 2) & 3, tz = lane >> 4;
  const bool live = dim == 3 || lane < 16;
  for (int a = 0; a < dim; ++a) {
    double val = 0.0;
    if (live) {
      const int sx = a == 0, sy = a == 1, sz = a == 2;
      const int bx = tbase[m * 6 + sx * 3 + 0], by = tbase[m * 6 + sy * 3 + 1];
      const int ix = (bx + tx) & (n - 1), iy = (by + ty) & (n - 1);
      double w = tw[(m * 6 + sx * 3 + 0) * 4 + tx] * tw[(m * 6 + sy * 3 + 1) * 4 + ty];
      int64_t c = ix + ((int64_t)iy << logn);
      if (dim == 3) {
        const int bz = tbase[m * 6 + sz * 3 + 2];
        const int iz = (bz + tz) & (n - 1);
        w *= tw[(m * 6 + sz * 3 + 2) * 4 + tz];
        c += (int64_t)iz << (2 * logn);
      }
      val = w * (double)v[a * C + c];
    }
    val = wave_sum(val);
    if (lane == 0) {
      if (vshift) val -= vshift[a];
      double o = alpha * val;
      if (add) o += beta * add[m * dim + a];
      out[m * dim + a] = o;
    }
  }
}

// ---------------------------------------------------------------- reductions
__global__ void __launch_bounds__(256) k_lambda_partial(int dim, int N, const double* __restrict__ lam,
                                                        double* __restrict__ part) {
  __shared__ double red[256 / kWave];
  for (int a = 0; a < dim; ++a) {
    double s = 0;
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) s += lam[m * dim + a];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[a * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_lambda_finish(int dim, int nblocks, const double* __restrict__ part, double scale,
                                double* __restrict__ out) {
  __shared__ double red[256 / kWave];
  for (int a = 0; a < dim; ++a) {
    double s = 0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += part[a * nblocks + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[a] = s * scale;
  }
}

__global__ void __launch_bounds__(256) k_body_ft(int dim, const int* __restrict__ off, const double* __restrict__ R,
                                                 const double* __restrict__ X, double L,
                                                 const double* __restrict__ lam, double* __restrict__ F,
                                                 double* __restrict__ T) {
  __shared__ double red[256 / kWave];
  const int b = blockIdx.x;
  const int lo = off[b], hi = off[b + 1];
  double f[3] = {0, 0, 0}, t[3] = {0, 0, 0};
  for (int m = lo + threadIdx.x; m < hi; m += blockDim.x) {
    double r[3] = {0, 0, 0}, l[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      double d = R[m * dim + a] - X[b * dim + a];
      d -= L * rint(d / L);
      r[a] = d;
      l[a] = lam[m * dim + a];
      f[a] += l[a];
    }
    if (dim == 2) {
      t[0] += r[0] * l[1] - r[1] * l[0];
    } else {
      t[0] += r[1] * l[2] - r[2] * l[1];
      t[1] += r[2] * l[0] - r[0] * l[2];
      t[2] += r[0] * l[1] - r[1] * l[0];
    }
  }
  const int nt = dim == 3 ? 3 : 1;
  for (int a = 0; a < dim; ++a) {
    double s = block_sum(f[a], red);
    if (threadIdx.x == 0) F[b * dim + a] = s;
  }
  for (int a = 0; a < nt; ++a) {
    double s = block_sum(t[a], red);
    if (threadIdx.x == 0) T[b * nt + a] = s;
  }
}

}  // namespace

void launch_marker_setup(int dim, int logn, int N, double h, double L, const double* R, MarkerTaps taps,
                         int* tile_of, int tile_log, hipStream_t s, int walls) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_marker_setup, dim3(nblk(N)), dim3(256), 0, s, dim, logn, N, h, L, R, taps.base, taps.w64,
                     taps.w32, tile_of, tile_log, walls);
}

void launch_marker_velocity(int dim, int N, const double* R, const int* body, const double* centres,
                            const double* U, const double* Om, double L, double* V, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_marker_velocity, dim3(nblk(N)), dim3(256), 0, s, dim, N, R, body, centres, U, Om, L, V);
}

void launch_move_markers(int dim, int N, int nb, double* R, double* centres, const int* body, const double* U,
                         double dt, double L, hipStream_t s) {
  hipLaunchKernelGGL(k_move_markers, dim3(nblk(N + nb)), dim3(256), 0, s, dim, N, nb, R, centres, body, U, dt, L);
}

void launch_bin_markers(int N, int ntiles, const int* tile_of, int* counts, int* offsets, int* cursor, int* perm,
                        hipStream_t s) {
  launch_fill<int>(counts, ntiles, 0, s);
  launch_fill<int>(cursor, ntiles, 0, s);
  if (N > 0) hipLaunchKernelGGL(k_bin_count, dim3(nblk(N)), dim3(256), 0, s, N, tile_of, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, ntiles, offsets);
  if (N > 0) {
    hipLaunchKernelGGL(k_bin_scatter, dim3(nblk(N)), dim3(256), 0, s, N, tile_of, offsets, cursor, perm);
    hipLaunchKernelGGL(k_bin_sort, dim3(ntiles), dim3(kSortThreads), 0, s, offsets, perm);
  }
}

void launch_active_tiles(int dim, int tiles_log, const int* offsets, int* flags, int* active_list,
                         int* active_count, hipStream_t s) {
  const int ntiles = 1 << (dim * tiles_log);
  launch_fill<int>(active_count, 1, 0, s);
  hipLaunchKernelGGL(k_active_tiles, dim3(nblk(ntiles)), dim3(256), 0, s, dim, tiles_log, offsets, flags,
                     active_list, active_count);
}

template <typename TL, typename TY>
void launch_spread(int dim, int logn, int tile_log, int grid_cap, const int* active_list, const int* nactive,
                   const int* offsets, const int* perm, MarkerTaps taps, const TL* lam, TY* y, double scale,
                   hipStream_t s, bool split) {
  if (grid_cap <= 0) return;
#define IBR_SPREAD(D, S)                                                                                        \
  hipLaunchKernelGGL((k_spread<TL, TY, D, S>), dim3(grid_cap, D), dim3(256), 0, s, logn, tile_log, active_list, \
                     nactive, offsets, perm, taps.base, taps.w64, lam, y, scale)
  if (dim == 3) {
    if (split) IBR_SPREAD(3, true); else IBR_SPREAD(3, false);
  } else {
    if (split) IBR_SPREAD(2, true); else IBR_SPREAD(2, false);
  }
#undef IBR_SPREAD
}
template void launch_spread<double, double>(int, int, int, int, const int*, const int*, const int*, const int*,
                                            MarkerTaps, const double*, double*, double, hipStream_t, bool);
template void launch_spread<float, double>(int, int, int, int, const int*, const int*, const int*, const int*,
                                           MarkerTaps, const float*, double*, double, hipStream_t, bool);
template void launch_spread<double, float>(int, int, int, int, const int*, const int*, const int*, const int*,
                                           MarkerTaps, const double*, float*, double, hipStream_t, bool);

template <typename TV>
void launch_interp(int dim, int logn, int N, MarkerTaps taps, const TV* v, double alpha, const double* add,
                   double beta, double* out, hipStream_t s, const double* vshift) {
  if (N <= 0) return;
  const int64_t threads = (int64_t)N * kWave;
  hipLaunchKernelGGL((k_interp<TV>), dim3(nblk(threads)), dim3(256), 0, s, dim, logn, N, taps.base, taps.w64, v,
                     alpha, add, beta, out, vshift);
}
template void launch_interp<double>(int, int, int, MarkerTaps, const double*, double, const double*, double,
                                    double*, hipStream_t, const double*);
template void launch_interp<float>(int, int, int, MarkerTaps, const float*, double, const double*, double,
                                   double*, hipStream_t, const double*);

void launch_lambda_sums(int dim, int N, const double* lam, double* part, double* out, double scale,
                        hipStream_t s) {
  const int nb = 64;
  hipLaunchKernelGGL(k_lambda_partial, dim3(nb), dim3(256), 0, s, dim, N, lam, part);
  hipLaunchKernelGGL(k_lambda_finish, dim3(1), dim3(256), 0, s, dim, nb, part, scale, out);
}

void launch_body_force_torque(int dim, int nb, const int* offsets, const double* R, const double* centres,
                              double L, const double* lam, double* F, double* T, hipStream_t s) {
  hipLaunchKernelGGL(k_body_ft, dim3(nb), dim3(256), 0, s, dim, offsets, R, centres, L, lam, F, T);
}

}  // namespace ibr
