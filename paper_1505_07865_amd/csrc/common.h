// Shared device-side definitions for the constrained immersed-boundary solver.
// gfx950 only: wave64, 8 XCDs, fp64 MFMA for the dense mobility blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace ibr {

constexpr int kWave = 64;
constexpr int kXcds = 8;

// Grid geometry of one multigrid level or of the fine grid.
struct Geom {
  int n;       // cells per direction (power of two)
  int logn;    // log2(n)
  int dim;     // 2 or 3
  int64_t C;   // n^dim
};

__host__ __device__ inline int wrapi(int i, int n) { return i & (n - 1); }

// XCD-aware remap of a flat 1D block index: the hardware hands consecutive
// workgroups to different XCDs round-robin; remapping gives each XCD one
// contiguous slab of the grid so stencil neighbours share that XCD's L2.
__device__ inline int64_t xcd_block(int64_t nblocks) {
  int64_t b = blockIdx.x;
  if (nblocks % kXcds != 0) return b;
  int64_t per = nblocks / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

// Orders one wavefront's LDS accesses across its lanes: every access before
// it is complete and visible to the wavefront's other lanes before any after it.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum (blockDim.x a multiple of 64, <= 1024); result valid in all threads.
template <typename T>
__device__ inline T block_sum(T v, T* smem) {
  v = wave_sum(v);
  int lane = threadIdx.x & (kWave - 1);
  int w = threadIdx.x / kWave;
  int nw = blockDim.x / kWave;
  __syncthreads();
  if (lane == 0) smem[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += smem[i];
  return s;
}

// Cell lattices of the preconditioner and the multigrid hierarchy use split
// storage: the red cells (i+j+k even) first, then the black cells, each half
// row-major over (row = j + k n, i >> 1).  Storage index of cell (i, j, k),
// wrapped into the periodic lattice:
template <int DIM>
__device__ inline int split_index(int i, int j, int k, int logn) {
  const int mask = (1 << logn) - 1;
  i &= mask;
  j &= mask;
  k &= mask;
  const int row = DIM == 3 ? (j | (k << logn)) : j;
  return (((i + j + k) & 1) << (DIM * logn - 1)) | (row << (logn - 1)) | (i >> 1);
}
// Natural (x-fastest) index of cell (i, j, k), wrapped.
template <int DIM>
__device__ inline int natural_index(int i, int j, int k, int logn) {
  const int mask = (1 << logn) - 1;
  int c = (i & mask) | ((j & mask) << logn);
  if (DIM == 3) c |= (k & mask) << (2 * logn);
  return c;
}

// Peskin's four-point kernel, r in units of h (|r| < 2 support).
template <typename T>
__device__ inline T phi4(T r) {
  T a = r < T(0) ? -r : r;
  if (a <= T(1)) return (T(3) - T(2) * a + sqrt(T(1) + T(4) * a - T(4) * a * a)) * T(0.125);
  if (a < T(2)) {
    T q = T(-7) + T(12) * a - T(4) * a * a;
    q = q > T(0) ? q : T(0);
    return (T(5) - T(2) * a - sqrt(q)) * T(0.125);
  }
  return T(0);
}

}  // namespace ibr
