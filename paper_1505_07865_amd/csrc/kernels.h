// Internal launchers shared by the kernel files and the solver.  Not part of
// the public C ABI (include/ibr.h).
#pragma once

#include <stdexcept>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "common.h"

namespace ibr {

struct DeviceError : std::runtime_error {
  explicit DeviceError(const std::string& m) : std::runtime_error(m) {}
};

#define IBR_HIP(call)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess)                                                                           \
      throw ::ibr::DeviceError(std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

template <typename T>
T* dev_alloc(int64_t count) {
  if (count <= 0) return nullptr;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, (size_t)count * sizeof(T));
  if (e != hipSuccess) throw DeviceError(std::string("hipMalloc: ") + hipGetErrorString(e));
  return (T*)p;
}
inline void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

// ---------------------------------------------------------------- live kernel timers
enum TimerId {
  kTimerRbFine = 0,
  kTimerOrthoDot = 1,
  kTimerOrthoAxpy = 2,
  kTimerStokes = 3,
  kTimerVcycle = 4,  // whole V-cycles (events recorded around all of their kernels)
  kTimerWallRbFine = 5,  // finest-level half sweeps of the slit channel's V-cycle
  kTimerRbRedProlong = 6,  // finest-level red half sweeps with the prolongation folded in
  kTimerCount = 7
};
// A launch of a timed class is sampled (every stride-th one): the sampled launch
// gets a start and a stop event to pass to hipExtLaunchKernelGGL, which stamps
// them with the kernel's own start and end; unsampled launches get null events
// (a plain launch).  bytes: the launch's algorithmic bytes.
struct TimerEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
TimerEvents timer_sample(int id, double bytes);
bool timers_any();  // some timer is enabled

// ---------------------------------------------------------------- grid stencils
// Cell lattices are in natural storage (x fastest, the public layout) or, with
// split, in split storage (red half, black half; see split_index in common.h).
template <typename TI, typename TO>
void launch_stokes_apply(int dim, int logn, const TI* v, const TI* p, TO* yv, TO* yp, double c0, double ch2,
                         double inv_h, const double* addc, hipStream_t s, bool split = false,
                         TimerEvents ev = TimerEvents(), int walls = 0);
// Partial sums of the normal equations of min_y || r - [W_0 .. W_{ns-2}, w] y ||
// with w = K (v, p) (split storage, ns in 1..3) formed without storing w:
// stokes_gram_blocks(dim, logn) workgroups, part needs (ns(ns+1)/2 + ns) times
// that many doubles; launch_gram_finish solves for y from them.
int stokes_gram_blocks(int dim, int logn);
template <typename T>
void launch_stokes_gram(int dim, int logn, const T* v, const T* p, const T* W, int64_t ld, int ns, const T* r,
                        double c0, double ch2, double inv_h, int walls, double* part, hipStream_t s);
template <typename T>
void launch_div_q(int dim, int logn, const T* v, const T* hp, T* q, double inv_h, hipStream_t s,
                  bool split = false);
template <typename T>
void launch_ps_finish(int dim, int logn, T* v, const T* phi, const T* q, T* pi, double h, double c0h2, double eta,
                      const double* vmean, hipStream_t s, bool split = false, int walls = 0);
// nf fields: natural -> split storage (with conversion TS -> TD), and back
template <typename TS, typename TD>
void launch_to_split(int dim, int logn, const TS* src, TD* dst, int nf, hipStream_t s);
template <typename TS, typename TD>
void launch_from_split(int dim, int logn, const TS* src, TD* dst, int nf, hipStream_t s);
// x (natural, nf fields) = [x +] sum_j y[j] Z_j (split, stride ld)
template <typename TZ, typename TX>
void launch_combine_from_split(int dim, int logn, const TZ* Z, int64_t ld, int k, const double* y, TX* x, int nf,
                               bool assign, hipStream_t s);
// walls: bit a = no-slip walls at both ends of axis a (0: periodic box)
void launch_zero_wall_faces(int dim, int logn, double* v, int walls, hipStream_t s);
// Moving walls: the velocities of the walls at the low and high end of the
// walled axis; their background flow is linear along that axis.
struct WallVel {
  double lo[3], hi[3];
};
// skip: wall mask whose wall faces are left untouched (0: every face)
void launch_add_background(int dim, int logn, double* v, double h, double len, int axis, WallVel wv, double scale,
                           int skip, hipStream_t s);
void launch_sub_background_markers(double* Vm, const double* R, int N, int dim, int axis, double len, WallVel wv,
                                   hipStream_t s);
void launch_advect(int dim, int logn, const double* v, double* N, double inv_2h, hipStream_t s, int walls = 0);
void launch_advect_sl(int dim, int logn, const double* v, double* N, double dtoh, double inv_dt, hipStream_t s,
                      int walls = 0);
void launch_ns_rhs(const double* v, const double* N1, const double* N0, double* g, int64_t len, double rdt,
                   double rho, double w1, double w0, hipStream_t s);

// ---------------------------------------------------------------- multigrid
template <typename T>
void launch_fill(T* x, int64_t len, T v, hipStream_t s);
template <typename T>
void launch_field_means(const T* x, int nf, int64_t C, double* part, int part_blocks, double* out, hipStream_t s);
template <typename T>
void launch_sub_field_mean(T* x, int nf, int64_t C, const double* mean, hipStream_t s);

// Fused 3D level kernels (one workgroup per 8^3 tile and field, LDS temporal
// blocking): pre = first sweep from zero + nu - 1 sweeps + residual
// restriction into bc; post = black-cell prolongation of e + nu sweeps, from
// xi into xo (neighbouring tiles read xi around their own tile, so it cannot
// be updated in place).
bool fused_level_ok(int dim, int logn, int nu);
template <typename V>
void launch_mg_pre_fused(const V* b, V* x, V* bc, int logn, int nf, V c0, V c1, int nu, hipStream_t s,
                         TimerEvents ev = TimerEvents());
template <typename V>
void launch_mg_post_fused(const V* b, const V* xi, V* xo, const V* e, int logn, int nf, V c0, V c1, int nu,
                          hipStream_t s, TimerEvents ev = TimerEvents());

template <typename T>
struct MGHier {
  int dim = 3, logn = 0, nfmax = 0, lds_logn = 0;
  std::vector<int> levels;          // log2 n of the multi-kernel levels (finest first)
  std::vector<T*> bufs_x, bufs_b;   // per level >= 1, nfmax fields each
  // fused 3D levels: the post kernel reads the pre-smoothed x around its
  // tile and so writes the result to a second buffer (bufs_xo, level >= 1;
  // x0_tmp holds the pre-smoothed finest level when that level is fused)
  std::vector<T*> bufs_xo;
  T* x0_tmp = nullptr;
  // no-slip walls (wall_mask bit b: walls at both ends of axis b): every
  // level below the finest down to 4^dim in global memory (index 1 .. logn-2)
  int wall_mask = 0;
  std::vector<T*> wall_x, wall_b;
  bool fused(int lg, int nu, int nf) const;
  void init(int dim, int logn, int nfmax, int wall_mask = 0);
  void release();
  static size_t bytes(int dim, int logn, int nf, bool walls = false);
  // One V-cycle for nf fields: x = V(b).  x and b hold nf fields of n^dim in
  // split (red half, black half) storage; see launch_to_split.  wall_mode 0:
  // periodic; with walls 1: the velocity cycle (nf = dim: field f is
  // component f), 2: the pressure cycle (nf = 1).
  void vcycle(int nf, const T* b, T* x, double c0, double c1, int nu_pre, int nu_post, int nu_coarse,
              hipStream_t s, int wall_mode = 0);
  void rb_half(T* x, const T* b, int lg, int nf, T c0, T c1, int color, bool fine, hipStream_t s);
  // first sweep (red then black) from a zero guess, in one pass
  void rb_first(T* x, const T* b, int lg, int nf, T c0, T c1, bool fine, hipStream_t s);
  void rb_red_prolong(T* x, const T* b, const T* e, int lg, int nf, T c0, T c1, bool fine, hipStream_t s);
};

// V-cycle with no-slip walls at both ends of the axes in wm (bit b: axis b;
// mode as in MGHier::vcycle); wx, wb: per-level buffers 1 .. logn-2 (nf
// fields each).
template <typename T>
void launch_wall_vcycle(int dim, int logn, int nf, const T* b, T* x, const std::vector<T*>& wx,
                        const std::vector<T*>& wb, double c0, double c1, int nu_pre, int nu_post, int nu_coarse,
                        int mode, int wm, hipStream_t s);

// ---------------------------------------------------------------- free kinematics
// Body block of the stacked vector: U[nb][dim] then Omega[nb][1 or 3].
// y_L += K U on free bodies' markers; y_U = K* lam (free) or x_U (prescribed).
template <typename TI>
void launch_free_apply(int dim, int N, int nb, const int* off, const int* body, const double* R, const double* X,
                       double L, const int* free_b, const double* lam, const TI* xu, const TI* xo, double* yl,
                       double* yu, double* yo, hipStream_t s);
// Y = M~^-1 K and N~ = (K* Y)^-1 per free body; fail[b] set when K* Y is not SPD.
void launch_free_setup(int dim, int nb, const int* off, const int64_t* moff, const double* Minv, const double* R,
                       const double* X, double L, const int* free_b, const int64_t* yoff, double* Y, double* Nm,
                       int* fail, hipStream_t s);
// Per-body step of the preconditioner (lam = M~^-1 dU on entry).
template <typename TZ>
void launch_free_precond(int dim, int nb, const int* off, const double* R, const double* X, double L,
                         const int* free_b, const int64_t* yoff, const double* Y, const double* Nm, const double* ru,
                         const double* ro, double* lam, TZ* zu, TZ* zo, hipStream_t s);
void launch_free_zero_markers(int dim, int N, const int* body, const int* free_b, double* W, hipStream_t s);

// ---------------------------------------------------------------- markers / IB
// Per-marker interpolation data: for every dimension beta the first tap index
// (not wrapped) and the 4 weights, for the cell-centred (c) and the face (f)
// staggering of that axis.  Component a uses the face staggering on axis a.
struct MarkerTaps {
  int* base;        // [N][2][3]: base[(m*2 + s)*3 + beta], s = 0 cell-centred, 1 face
  double* w64;      // [N][2][3][4]
  float* w32;       // same, fp32
};

void launch_marker_setup(int dim, int logn, int N, double h, double L, const double* R, MarkerTaps taps,
                         int* tile_of, int tile_log, hipStream_t s, int walls = 0);
void launch_marker_velocity(int dim, int N, const double* R, const int* body, const double* centres,
                            const double* U, const double* Om, double L, double* V, hipStream_t s);
void launch_move_markers(int dim, int N, int nb, double* R, double* centres, const int* body, const double* U,
                         double dt, double L, hipStream_t s);

// Tile binning: count/scan/scatter/sort so that tile t owns perm[off[t] .. off[t+1]).
void launch_bin_markers(int N, int ntiles, const int* tile_of, int* counts, int* offsets, int* cursor, int* perm,
                        hipStream_t s);
void launch_active_tiles(int dim, int tiles_log, const int* offsets, int* flags, int* active_list,
                         int* active_count, hipStream_t s);

// y_face[a] += scale * sum_i lam[i][a] * w  over the active tiles (y in natural
// storage, or in split storage with split).  The grid
// holds grid_cap workgroups per component; the number of active tiles is read
// on the device from *nactive (<= grid_cap), so the launch needs no host sync.
template <typename TL, typename TY>
void launch_spread(int dim, int logn, int tile_log, int grid_cap, const int* active_list, const int* nactive,
                   const int* offsets, const int* perm, MarkerTaps taps, const TL* lam, TY* y, double scale,
                   hipStream_t s, bool split = false);
// out[i][a] = alpha * (J (v - vshift))[i][a] + beta * add[i][a]   (add may be
// null; vshift, if not null, is a constant per component a, vshift[a]: the
// kernel weights sum to one, so J of a constant is that constant)
template <typename TV>
void launch_interp(int dim, int logn, int N, MarkerTaps taps, const TV* v, double alpha, const double* add,
                   double beta, double* out, hipStream_t s, const double* vshift = nullptr);
void launch_lambda_sums(int dim, int N, const double* lam, double* part, double* out, double scale,
                        hipStream_t s);
void launch_body_force_torque(int dim, int nb, const int* offsets, const double* R, const double* centres,
                              double L, const double* lam, double* F, double* T, hipStream_t s);

// ---------------------------------------------------------------- Krylov
// h[j] = <w, V_j> for j < k (V_j = V + j*ld); two-pass deterministic reduction.
// cond: optional device flag; when it holds 0 the kernels return at once.
template <typename TV, typename TW>
void launch_multi_dot(const TV* V, int64_t ld, int k, const TW* w, int64_t len, double* part, int nblocks,
                      double* h, bool accumulate, hipStream_t s, const int* cond = nullptr);
// w -= sum_j h[j] V_j ; if norm_part != null also writes partial sums of w^2.
template <typename TV, typename TW>
void launch_multi_axpy(const TV* V, int64_t ld, int k, const double* h, TW* w, int64_t len, double* norm_part,
                       int nblocks, hipStream_t s, const int* cond = nullptr);
// Arnoldi orthogonalisation of w = V_{k+1} against V_0..V_k (basis stride ld):
// classical Gram-Schmidt; with reorth, a second pass when the DGKS criterion
// asks for it.  Writes hcol[0..k+1] (hcol[k+1] = ||w||); w is left unnormalised.
template <typename T>
void arnoldi_step(const T* V, int64_t ld, int k, double* hcol, double* h2, double* part1, double* part2,
                  int nblocks, int* flag, hipStream_t s, bool timed = false, bool reorth = true);
// One delayed-CGS2 Arnoldi step of the outer FGMRES (see ops_krylov.hip);
// basis vectors of length len at stride ld:
// V_k pending on entry, w = V_{k+1}; afterwards V_k is final, V_{k+1} pending,
// H column k-1 final and rotated, column k provisional, *resid the estimate.
// G needs 2(k+2) doubles, coef 2k+2, part 2(k+2)*nblocks.
// With split non-null, the new pending V_{k+1}'s first nsplit = (dim+1) C
// entries (velocity and pressure) are also written to split, in split storage
// and type TS, as the conversion of the next preconditioner input would.
template <typename T, typename TS>
void dcgs2_step(T* V, int64_t ld, int64_t len, int k, double* H, int ldh, double* G, double* coef, double* part,
                int nblocks, double* cs, double* sn, double* g, double* resid, hipStream_t s, bool timed,
                TS* split, int dim, int logn, int64_t nsplit);
// x += sum_j y[j] Z_j  (Z in TZ, x in TX); with assign, x = sum_j y[j] Z_j.
// With zmean (stride 4 per column), the first dim blocks of C entries of
// column j are taken as Z_j - zmean[4j + a]: the velocity components of the
// stored directions with their fp64 means removed.
template <typename TZ, typename TX>
void launch_combine(const TZ* Z, int64_t ld, int k, const double* y, TX* x, int64_t len, hipStream_t s,
                    bool assign = false, const double* zmean = nullptr, int64_t C = 0, int dim = 0);
// y[0..ns) = argmin || r - sum_j y_j W_j ||  (ns in 1..3) from the partial
// sums of the normal equations (launch_stokes_gram), nblocks per product.
template <typename T>
void launch_gram_finish(const double* part, int nblocks, int ns, double* y, hipStream_t s);
void launch_norm_finish(const double* part, int nblocks, double* out, hipStream_t s);
template <typename T>
void launch_sumsq_partial(const T* w, int64_t len, double* part, int nblocks, hipStream_t s);
// dst = src * (1/ *nrm) (0 if nrm == 0); types may differ (conversion)
template <typename TS, typename TD>
void launch_scale_copy(const TS* src, TD* dst, int64_t len, const double* nrm, hipStream_t s);
template <typename TS, typename TD>
void launch_copy(const TS* src, TD* dst, int64_t len, hipStream_t s);
// y = a*x + b*y (a, b host scalars)
void launch_axpby(const double* x, double* y, int64_t len, double a, double b, hipStream_t s);

// Givens / Hessenberg least squares (a single wavefront).
//   H: column-major (m+1) x m, leading dimension m+1.
void launch_givens_step(double* H, int ldh, int k, double* cs, double* sn, double* g, double* resid,
                        hipStream_t s);
void launch_lsq_solve(const double* H, int ldh, int k, const double* g, double* y, hipStream_t s);
// g = (beta, 0, ..., 0) with beta read from device memory.
void launch_init_g(double* g, int len, const double* beta, hipStream_t s);
// Number of blocks for the two-pass reductions over a vector of length len.
int krylov_dot_blocks(int64_t len);

// ---------------------------------------------------------------- mobility blocks
struct MobParams {
  int dim;
  int steady;
  double a, eta, L, finf0, f00, alpha, dt_rho, periodic_shift;
  // fitted forms (3D): 0 = the analytic readings; 1 = the steady fit (ah =
  // a/h, fs = b0..b6); 2 = the finite-beta fit at viscous CFL number beta:
  // phi0(beta), and the two table rows around beta (fa = a0..a9, fb =
  // b0..b5), whose forms, both evaluated at beta, are blended with weights
  // 1 - tw, tw (tw linear in log beta).
  // 2D (Appendix B): 3 = the steady fit (self0 = f(0), f2s = a0..a4,
  // b0..b3); 4 = the finite-beta fit (phi0, rows f2r = a0..a3, p1, b1, b2,
  // c0..c3, p2, p3, blended like the 3D rows).
  // mean_mode: dt / (rho l^d), the uniform velocity a unit force gives the
  // fluid of an unsteady periodic box, added to f by the fitted forms
  int fit;
  double h, beta, phi0, ah, mean_mode, tw, self0, fs[7], fa[2][10], fb[2][6], f2s[9], f2r[2][13];
};
void launch_mob_assemble(int dim, int nb, const int* offsets, const int64_t* moff, const double* R, MobParams p,
                         double* M, int max_np, hipStream_t s);
// Xf receives the inverses of the 64 x 64 diagonal blocks of each factor
// (the diagonal blocks of L^-1), which launch_chol_inverse completes.
void launch_chol(int nb, const int* offsets, int dim, const int64_t* moff, const double* M, double* Lf, double* Xf,
                 const int* active, const double* shift, double f0, double pivot_tol, int* fail, int max_rows,
                 hipStream_t s);
void launch_chol_inverse(int nb, const int* offsets, int dim, const int64_t* moff, double* Lf, double* Minv,
                         double* X, int max_n, hipStream_t s);
void launch_mob_apply(int nb, const int* offsets, int dim, const int64_t* moff, const double* Minv,
                      const double* dU, double* lam, int max_rows, hipStream_t s);

}  // namespace ibr
