// Spreading S (Sec. 3.1) with no context and no device allocation.
//
// ibr_spread_noalloc runs the same kernels as a context's ibr_spread (marker
// taps, tile binning, the atomic-free gather), but every temporary array lives
// in one file-scope device array of fixed size, so the call never allocates:
// it can run under HIP graph capture or in a serving loop that must not call
// hipMalloc.  Each GPU holds its own copy of the array for the life of the
// process; its device address is looked up once per device and kept.  All
// calls on one GPU share it, so calls that overlap on one GPU (two streams,
// two host threads) race; the call itself is asynchronous on the stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "ibr.h"
#include "kernels.h"

using namespace ibr;

namespace {

constexpr size_t kScratchBytes = IBR_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// The scratch array of every device (see the file comment).  Host code never
// uses this name as an address: it takes the per-device address from
// hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

struct NoallocError {
  ibr_status code;
  std::string msg;
};

// Address of the device's scratch array, looked up once per device with that
// device current (each GPU holds its own copy at its own address).
void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw NoallocError{IBR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte layout of the temporaries inside the scratch array.
struct Layout {
  size_t base, w64, w32, tile_of, perm, counts, toff, cursor, flags, active, nactive, end;
};

Layout layout(int64_t N, int64_t ntiles) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.base = take((size_t)N * 6 * sizeof(int));
  L.w64 = take((size_t)N * 24 * sizeof(double));
  L.w32 = take((size_t)N * 24 * sizeof(float));
  L.tile_of = take((size_t)N * sizeof(int));
  L.perm = take((size_t)N * sizeof(int));
  L.counts = take((size_t)ntiles * sizeof(int));
  L.toff = take((size_t)(ntiles + 1) * sizeof(int));
  L.cursor = take((size_t)ntiles * sizeof(int));
  L.flags = take((size_t)ntiles * sizeof(int));
  L.active = take((size_t)ntiles * sizeof(int));
  L.nactive = take(sizeof(int));
  L.end = o;
  return L;
}

void require_device(const void* p, int device, const char* what) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    throw NoallocError{IBR_EINVAL, std::string(what) + " is not device memory"};
  }
  if (a.type != hipMemoryTypeDevice || a.device != device)
    throw NoallocError{IBR_EINVAL, std::string(what) + " is not device memory of params->device"};
}

void set_msg(char* msg, size_t len, const std::string& s) {
  if (!msg || len == 0) return;
  const size_t k = std::min(len - 1, s.size());
  std::memcpy(msg, s.data(), k);
  msg[k] = '\0';
}

}  // namespace

extern "C" ibr_status ibr_spread_noalloc(const ibr_params* p, int nmarkers, const void* R, const void* lambda,
                                         void* f, char* msg, size_t msg_len) {
  set_msg(msg, msg_len, "");
  try {
    if (!p) throw NoallocError{IBR_EINVAL, "params is NULL"};
    const int d = p->dim;
    if (d != 2 && d != 3) throw NoallocError{IBR_EINVAL, "dim must be 2 or 3"};
    const int lo = d == 3 ? 8 : 16, hi = d == 3 ? 512 : 4096;
    if (p->n < lo || p->n > hi || (p->n & (p->n - 1)))
      throw NoallocError{IBR_EINVAL, "n must be a power of two in [" + std::to_string(lo) + ", " +
                                         std::to_string(hi) + "]"};
    if (!(p->h > 0) || !std::isfinite(p->h)) throw NoallocError{IBR_EINVAL, "h must be > 0"};
    if (p->walls != IBR_WALLS_NONE && p->walls != IBR_WALLS_NOSLIP && p->walls != IBR_WALLS_BOX)
      throw NoallocError{IBR_EINVAL, "bad walls"};
    if (p->device < 0 || p->device >= kMaxDevices) throw NoallocError{IBR_EINVAL, "bad device"};
    if (nmarkers < 0) throw NoallocError{IBR_EINVAL, "nmarkers must be >= 0"};
    if (!f) throw NoallocError{IBR_EINVAL, "f is required"};
    if (nmarkers > 0 && (!R || !lambda)) throw NoallocError{IBR_EINVAL, "R and lambda are required"};
    const int logn = ilog2(p->n);
    int tile_log = d == 3 ? 3 : 4;
    if (tile_log > logn) tile_log = logn;
    const int tiles_log = logn - tile_log;
    const int64_t ntiles = (int64_t)1 << (d * tiles_log);
    const Layout L = layout(nmarkers, ntiles);
    if (L.end > kScratchBytes) {
      // largest marker count whose temporaries fit beside this grid's tile arrays
      int64_t lo_n = 0, hi_n = nmarkers;
      while (lo_n < hi_n) {
        const int64_t mid = (lo_n + hi_n + 1) / 2;
        if (layout(mid, ntiles).end <= kScratchBytes) lo_n = mid; else hi_n = mid - 1;
      }
      throw NoallocError{IBR_EINVAL, std::to_string(nmarkers) + " markers on a " + std::to_string(p->n) +
                                         "^" + std::to_string(d) + " grid exceed the " +
                                         std::to_string(kScratchBytes >> 20) + " MiB scratch (at most " +
                                         std::to_string(lo_n) + " markers fit)"};
    }
    IBR_HIP(hipSetDevice(p->device));
    if (nmarkers > 0) {
      require_device(R, p->device, "R");
      require_device(lambda, p->device, "lambda");
    }
    require_device(f, p->device, "f");
    unsigned char* sc = (unsigned char*)scratch_of(p->device);
    hipStream_t s = (hipStream_t)p->stream;
    const int64_t C = (int64_t)1 << (d * logn);
    double* fd = (double*)f;
    launch_fill<double>(fd, (int64_t)d * C, 0.0, s);
    if (nmarkers == 0) return IBR_OK;
    MarkerTaps taps{(int*)(sc + L.base), (double*)(sc + L.w64), (float*)(sc + L.w32)};
    int* tile_of = (int*)(sc + L.tile_of);
    int* perm = (int*)(sc + L.perm);
    int* counts = (int*)(sc + L.counts);
    int* toff = (int*)(sc + L.toff);
    int* cursor = (int*)(sc + L.cursor);
    int* flags = (int*)(sc + L.flags);
    int* active = (int*)(sc + L.active);
    int* nactive = (int*)(sc + L.nactive);
    const double len = p->n * p->h;
    // walls along the last axis (slit) or every axis (box): one bit per axis
    const int wm = p->walls == IBR_WALLS_NOSLIP ? 1 << (d - 1) : (p->walls == IBR_WALLS_BOX ? (1 << d) - 1 : 0);
    launch_marker_setup(d, logn, nmarkers, p->h, len, (const double*)R, taps, tile_of, tile_log, s, wm);
    launch_bin_markers(nmarkers, (int)ntiles, tile_of, counts, toff, cursor, perm, s);
    launch_active_tiles(d, tiles_log, toff, flags, active, nactive, s);
    // a tile is active when one of its 3^d neighbours holds a marker: at most
    // 3^d N tiles, so the grid needs no host read of the count
    const int64_t cap = std::min<int64_t>(ntiles, (int64_t)nmarkers * (d == 3 ? 27 : 9));
    launch_spread<double, double>(d, logn, tile_log, (int)cap, active, nactive, toff, perm, taps,
                                  (const double*)lambda, fd, std::pow(p->h, -d), s);
    IBR_HIP(hipGetLastError());
    return IBR_OK;
  } catch (const NoallocError& e) {
    set_msg(msg, msg_len, e.msg);
    return e.code;
  } catch (const DeviceError& e) {
    set_msg(msg, msg_len, e.what());
    return IBR_EDEVICE;
  } catch (const std::exception& e) {
    set_msg(msg, msg_len, e.what());
    return IBR_EDEVICE;
  }
}
