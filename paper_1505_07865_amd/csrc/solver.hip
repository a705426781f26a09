// Host orchestration and C ABI (include/ibr.h).
//
// Outer solver: right-preconditioned flexible GMRES (Sec. 5) on the stacked
// fp64 vector x = [v (dim C), pi (C), Lambda (dim N)] with restart m; the
// Arnoldi step is delayed classical Gram-Schmidt with re-orthogonalisation
// (one reduction and one update pass per iteration), the Hessenberg least
// squares uses Givens rotations on the device, and the host reads one
// residual estimate per iteration.  Each iteration can be replayed as a
// captured HIP graph.
//
// Preconditioner (Sec. 5.1): inner GMRES(N_s) on the Stokes block with
// P_S^-1 (eq. P1_practical) in the working precision T (fp64, or fp32 in the
// mixed mode) on split (red/black) storage, slip dU = -(J v + r_L), per-body
// Lambda = M~^-1 dU in fp64, and for the full variant a second inner solve
// with r_v + S'Lambda.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "ibr.h"
#include "kernels.h"

using namespace ibr;

namespace {

#include "mobility_fit_4pt.inc"
#include "mobility_fit_4pt_2d.inc"

constexpr double kPi = 3.14159265358979323846;
constexpr double kA3D = 1.25;      // four-point marker hydrodynamic radius, units of h (3D)
constexpr double kA2D = 1.04;      // four-point marker radius in the 2D periodic self-mobility
constexpr double kPeriodic3D = 2.84;
constexpr double kPivotTol = 1e-8;
constexpr double kShifts[] = {0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.3, 0.4, 0.5,
                               0.7, 1.0, 1.5, 2.0, 3.0, 5.0, 10.0, 20.0, 50.0};
constexpr int kNumShifts = sizeof(kShifts) / sizeof(kShifts[0]);
constexpr int kMaxBlockRows = 8192;

// Axes with no-slip walls at both ends, one bit per axis.
int wall_mask(int walls, int dim) {
  if (walls == IBR_WALLS_NOSLIP) return 1 << (dim - 1);
  if (walls == IBR_WALLS_BOX) return (1 << dim) - 1;
  return 0;
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

struct Status : std::runtime_error {
  ibr_status code;
  Status(ibr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

}  // namespace

struct ibr_ctx {
  ibr_params p{};
  int dim = 3, n = 0, logn = 0;
  int64_t C = 0;
  double h = 0, L = 0, c0 = 0, ch2 = 0, inv_h = 0, vol = 0;
  bool steady = true;
  // no-slip walls: wm bit a = walls at both ends of axis a (the slit channel
  // has the last axis, the box every axis); the velocity then has no null
  // space, so only periodic steady Stokes (vnull) carries the mean-velocity
  // condition and S'
  bool walls = false;
  int wm = 0;
  bool vnull = true;
  // per body and axis (host, [nb][dim]): centre, marker extent below and
  // above it, prescribed velocity; ibr_step checks the next position along
  // every walled axis
  std::vector<double> wall_z, wall_lo, wall_hi, wall_uz;
  bool mixed = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  // markers
  int nb = 0, N = 0, Ncap = 0;
  std::vector<int> off_h;
  int* off_d = nullptr;
  int* body_d = nullptr;
  double *R = nullptr, *X = nullptr, *U = nullptr, *Om = nullptr, *Vm = nullptr;
  MarkerTaps taps{nullptr, nullptr, nullptr};
  int *tile_of = nullptr, *counts = nullptr, *toff = nullptr, *cursor = nullptr, *perm = nullptr, *flags = nullptr,
      *active = nullptr, *nactive_d = nullptr;
  int tile_log = 3, tiles_log = 0, ntiles = 0, nactive = 0;
  int act_cap = 0;  // spread grid capacity (>= nactive), baked into captured graphs

  // mobility blocks
  std::vector<int64_t> moff_h;
  int64_t* moff_d = nullptr;
  double *Mb = nullptr, *Lb = nullptr, *Xb = nullptr, *Minv = nullptr;
  double *shift_d = nullptr;
  int *act_d = nullptr, *fail_d = nullptr;
  std::vector<double> shift_h;
  int max_np = 0, max_rows = 0;
  int nbcap = 0;      // bodies the body-sized buffers hold
  int64_t mcap = 0;   // doubles each mobility-block buffer holds
  double f0 = 1.0;
  MobParams mp{};

  // stacked vectors (fp64)
  int64_t NF = 0, NV = 0;
  int64_t ldv = 0;  // stride of the Krylov basis vectors: NV rounded up to 64 entries
  double *Xs = nullptr, *Bs = nullptr, *T1 = nullptr, *T2 = nullptr;
  double *lamd = nullptr, *dU = nullptr, *addc = nullptr, *lsum_part = nullptr;
  double *Nprev = nullptr, *Ncur = nullptr;
  bool have_prev = false;
  bool have_solution = false;
  bool rotating = false;  // some body has Omega != 0

  // free kinematics: bodies moving under applied loads (body block after Lambda)
  std::vector<int> free_h;
  int nfree = 0;
  // moving walls: the background flow u_b (linear along the last axis) of
  // ibr_set_wall_velocity; the solver's state holds u - u_b
  bool wallvel = false;
  WallVel wvel{};
  int64_t nq = 0;  // length of the body block: nb (dim + rotations) once some body is free, else 0
  int* free_d = nullptr;
  int64_t* yoff_d = nullptr;
  double *Yf = nullptr, *Nf = nullptr;
  std::vector<double> load_h;  // applied loads in the body-block layout (0 for prescribed bodies)

  // outer Krylov
  int m = 0;
  double* Vb = nullptr;
  void* Zb = nullptr;  // double or float
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *resid = nullptr, *beta = nullptr,
         *hc2 = nullptr, *part = nullptr, *part2 = nullptr, *G = nullptr, *coef = nullptr;
  // steady periodic: fp64 mean of each stored direction's velocity components
  // (column k at zmean + 4k); the directions enter K and the solution with
  // these means removed, so <v> = 0 holds in fp64 whatever Z's precision
  double* zmean = nullptr;
  int* flag = nullptr;
  int part_blocks = 0;  // blocks of the vector reductions' partial sums
  // partial sums of the inner solve's normal equations, one row of
  // stokes_gram_blocks per product (n_s <= 3)
  double* gpart = nullptr;
  int gpart_blocks = 0;
  int mean_blocks = 0;  // blocks of the per-field means' partial sums
  double* hres = nullptr;  // pinned

  // inner (precision T)
  int ns = 2;
  void *Qi = nullptr, *Zi = nullptr, *rhsT = nullptr, *qT = nullptr, *phiT = nullptr;
  double *Hi = nullptr, *csi = nullptr, *sni = nullptr, *gi = nullptr, *yi = nullptr, *residi = nullptr,
         *betai = nullptr, *hc2i = nullptr, *vmean = nullptr, *mpart = nullptr;
  MGHier<double> mg64;
  MGHier<float> mg32;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int64_t bytes = 0;

  // one captured graph per outer iteration index k (preconditioner, operator, Arnoldi)
  struct IterGraph {
    hipGraphExec_t exec = nullptr;
    int version = -1, ps = 0, vc = 0;
  };
  std::vector<IterGraph> graphs;
  int graph_version = 0;
  bool use_graphs = true;
  void drop_graphs();

  // counters of the current solve
  int cnt_ps = 0, cnt_vc = 0;

  ~ibr_ctx();
  void alloc_grid();
  void alloc_markers(int Nnew);
  void free_markers();
  void clear_free();
  template <typename T>
  T* track(int64_t count) {
    bytes += count * (int64_t)sizeof(T);
    return dev_alloc<T>(count);
  }
};

namespace {

void sync(ibr_ctx* c) { IBR_HIP(hipStreamSynchronize(c->stream)); }

template <typename T>
MGHier<T>& mg_of(ibr_ctx* c);
template <>
MGHier<double>& mg_of<double>(ibr_ctx* c) {
  return c->mg64;
}
template <>
MGHier<float>& mg_of<float>(ibr_ctx* c) {
  return c->mg32;
}

// ---------------------------------------------------------------- operator K
// y = K x,  x stored in TI (fp64, or fp32 for mixed Z vectors), y in fp64.
// xmean (steady periodic, may be null): per-component constants taken off x's
// velocity, which only J sees (the stencils and S' ignore constants).
template <typename TI>
void apply_K(ibr_ctx* c, const TI* x, double* y, const double* xmean = nullptr) {
  hipStream_t s = c->stream;
  const int d = c->dim;
  const TI* xv = x;
  const TI* xp = x + (int64_t)d * c->C;
  const TI* xl = x + c->NF;
  launch_copy<TI, double>(xl, c->lamd, (int64_t)c->N * d, s);
  const double* addc = nullptr;
  if (c->vnull) {
    // -S' Lambda = -S Lambda + vol^-1 sum Lambda
    launch_lambda_sums(d, c->N, c->lamd, c->lsum_part, c->addc, 1.0 / c->vol, s);
    addc = c->addc;
  }
  const TimerEvents ev = timer_sample(kTimerStokes, (double)(d + 1) * c->C * (sizeof(TI) + sizeof(double)));
  launch_stokes_apply<TI, double>(d, c->logn, xv, xp, y, y + (int64_t)d * c->C, c->c0, c->ch2, c->inv_h, addc, s,
                                  false, ev, c->wm);
  launch_spread<double, double>(d, c->logn, c->tile_log, c->act_cap, c->active, c->nactive_d, c->toff, c->perm,
                                c->taps, c->lamd, y, -std::pow(c->h, -d), s);
  launch_interp<TI>(d, c->logn, c->N, c->taps, xv, -1.0, nullptr, 0.0, y + c->NF, s, xmean);
  if (c->nq) {
    const int64_t ub = c->NF + (int64_t)d * c->N;
    launch_free_apply<TI>(d, c->N, c->nb, c->off_d, c->body_d, c->R, c->X, c->L, c->free_d, c->lamd, x + ub,
                          x + ub + (int64_t)c->nb * d, y + c->NF, y + ub, y + ub + (int64_t)c->nb * d, s);
  }
}

// ---------------------------------------------------------------- P_S^-1
template <typename T>
void ps_inv(ibr_ctx* c, const T* in, T* out) {
  hipStream_t s = c->stream;
  const int d = c->dim;
  const int64_t C = c->C;
  MGHier<T>& mg = mg_of<T>(c);
  const T* g = in;
  const T* hp = in + (int64_t)d * C;
  T* v = out;
  T* pi = out + (int64_t)d * C;
  T* q = (T*)c->qT;
  T* phi = (T*)c->phiT;
  const int wv = c->walls ? 1 : 0, wp = c->walls ? 2 : 0;
  mg.vcycle(d, g, v, c->c0, c->ch2, c->p.mg_pre, c->p.mg_post, c->p.mg_coarse, s, wv);
  const double* vmean = nullptr;
  if (c->vnull) {
    launch_field_means<T>(v, d, C, c->mpart, c->mean_blocks, c->vmean, s);
    vmean = c->vmean;
  }
  launch_div_q<T>(d, c->logn, v, hp, q, c->inv_h, s, true);
  // L_p phi = q  <=>  (0 - (-1) L) phi = q
  mg.vcycle(1, q, phi, 0.0, -1.0, c->p.mg_pre, c->p.mg_post, c->p.mg_coarse, s, wp);
  launch_ps_finish<T>(d, c->logn, v, phi, q, pi, c->h, c->c0 * c->h * c->h, c->p.eta, vmean, s, true, c->wm);
  c->cnt_ps += 1;
  c->cnt_vc += d + 1;
}

// Inner right-preconditioned GMRES(N_s) on the Stokes block, zero initial
// guess: out (fluid part, T) = approx [[A, G], [-D, 0]]^-1 rhs.
//
// For N_s <= 3 the Krylov space span{r, K P r, ...} is taken in its power
// basis: z_j = P p_j, w_j = K z_j, p_{j+1} = w_j, and the minimiser of
// ||r - W y|| comes from the normal equations (one reduction over W and r,
// one tiny Cholesky).  That is the GMRES(N_s) iterate in exact arithmetic
// (same space, same minimised norm) at a third of the vector passes; with
// K P close to I the few columns stay well separated.  Larger N_s use the
// Arnoldi process, whose orthonormal basis keeps the problem conditioned.
template <typename T>
void inner_gmres(ibr_ctx* c, const T* rhs, T* out) {
  hipStream_t s = c->stream;
  const int64_t NF = c->NF;
  const int ns = c->ns;
  const int d = c->dim;
  T* Q = (T*)c->Qi;
  T* Z = (T*)c->Zi;
  if (ns <= 3) {
    for (int j = 0; j < ns; ++j) {
      const T* pj = j == 0 ? rhs : Q + (int64_t)(j - 1) * NF;
      T* Zj = Z + (int64_t)j * NF;
      T* Wj = Q + (int64_t)j * NF;
      ps_inv<T>(c, pj, Zj);
      if (j + 1 < ns) {
        launch_stokes_apply<T, T>(d, c->logn, Zj, Zj + (int64_t)d * c->C, Wj, Wj + (int64_t)d * c->C, c->c0,
                                  c->ch2, c->inv_h, nullptr, s, true, TimerEvents(), c->wm);
      } else {
        // the last column serves only the normal equations: formed there, not stored
        launch_stokes_gram<T>(d, c->logn, Zj, Zj + (int64_t)d * c->C, Q, NF, ns, rhs, c->c0, c->ch2, c->inv_h,
                              c->wm, c->gpart, s);
      }
    }
    launch_gram_finish<T>(c->gpart, c->gpart_blocks, ns, c->yi, s);
    launch_combine_from_split<T, T>(d, c->logn, Z, NF, ns, c->yi, out, d + 1, true, s);
    return;
  }
  const int ldh = ns + 1;
  launch_sumsq_partial<T>(rhs, NF, c->part, c->part_blocks, s);
  launch_norm_finish(c->part, c->part_blocks, c->betai, s);
  launch_scale_copy<T, T>(rhs, Q, NF, c->betai, s);
  launch_init_g(c->gi, ns + 1, c->betai, s);
  launch_fill<double>(c->Hi, (int64_t)ldh * ns, 0.0, s);
  for (int j = 0; j < ns; ++j) {
    T* Qj = Q + (int64_t)j * NF;
    T* Zj = Z + (int64_t)j * NF;
    T* w = Q + (int64_t)(j + 1) * NF;
    ps_inv<T>(c, Qj, Zj);
    launch_stokes_apply<T, T>(d, c->logn, Zj, Zj + (int64_t)d * c->C, w, w + (int64_t)d * c->C, c->c0, c->ch2,
                              c->inv_h, nullptr, s, true, TimerEvents(), c->wm);
    double* hcol = c->Hi + (int64_t)j * ldh;
    // one Gram-Schmidt pass: the inner solve is only a preconditioner (FGMRES is flexible)
    arnoldi_step<T>(Q, NF, j, hcol, c->hc2i, c->part, c->part2, c->part_blocks, c->flag, s, false, false);
    launch_scale_copy<T, T>(w, w, NF, hcol + j + 1, s);
    launch_givens_step(c->Hi, ldh, j, c->csi, c->sni, c->gi, c->residi, s);
  }
  launch_lsq_solve(c->Hi, ldh, ns, c->gi, c->yi, s);
  launch_combine_from_split<T, T>(d, c->logn, Z, NF, ns, c->yi, out, d + 1, true, s);
}

// z = P r (Sec. 5.1).  r fp64 stacked; z stacked in T.  rhs_ready: the
// fluid fields of r are already in rhsT, in split storage (the previous outer
// iteration's Arnoldi update wrote them there).
template <typename T>
void precondition(ibr_ctx* c, const double* r, T* z, bool rhs_ready = false) {
  hipStream_t s = c->stream;
  const int d = c->dim;
  const int64_t NF = c->NF;
  T* rhs = (T*)c->rhsT;
  if (!rhs_ready) launch_to_split<double, T>(d, c->logn, r, rhs, d + 1, s);
  inner_gmres<T>(c, rhs, z);
  // slip dU = -(J v + r_L)
  launch_interp<T>(d, c->logn, c->N, c->taps, z, -1.0, r + NF, -1.0, c->dU, s);
  launch_mob_apply(c->nb, c->off_d, d, c->moff_d, c->Minv, c->dU, c->lamd, c->max_rows, s);
  if (c->nq) {
    // free bodies: U = N~ (r_U - K* Lambda), Lambda += Y U; the body block of z
    const int64_t ub = NF + (int64_t)d * c->N;
    launch_free_precond<T>(d, c->nb, c->off_d, c->R, c->X, c->L, c->free_d, c->yoff_d, c->Yf, c->Nf, r + ub,
                           r + ub + (int64_t)c->nb * d, c->lamd, z + ub, z + ub + (int64_t)c->nb * d, s);
  }
  if (c->p.pc == IBR_PC_FULL) {
    // second fluid solve with r_v + S' Lambda
    launch_spread<double, T>(d, c->logn, c->tile_log, c->act_cap, c->active, c->nactive_d, c->toff, c->perm,
                             c->taps, c->lamd, rhs, std::pow(c->h, -d), s, true);
    if (c->vnull) {
      launch_lambda_sums(d, c->N, c->lamd, c->lsum_part, c->addc, 1.0 / c->vol, s);
      launch_sub_field_mean<T>(rhs, d, c->C, c->addc, s);
    }
    inner_gmres<T>(c, rhs, z);
  }
  launch_copy<double, T>(c->lamd, z + NF, (int64_t)c->N * d, s);
}

// ---------------------------------------------------------------- FGMRES
// One outer iteration k: z_k = P v_k, w = K z_k, delayed-CGS2 Arnoldi step.
template <typename TZ>
void iteration_body(ibr_ctx* c, int k) {
  const int64_t NV = c->NV, ld = c->ldv;
  double* V = c->Vb;
  TZ* Z = (TZ*)c->Zb;
  double* vk = V + (int64_t)k * ld;
  double* w = V + (int64_t)(k + 1) * ld;
  TZ* zk = Z + (int64_t)k * ld;
  // V_k for k > 0 is the vector the previous iteration's update left pending,
  // and that update also wrote its split copy
  precondition<TZ>(c, vk, zk, k > 0);
  // Steady periodic Stokes (eq. constrained_periodic): K has d null vectors
  // that carry a mean velocity (and a net force), invisible to the residual,
  // so the gauge <v> = 0 is kept exactly: z_k counts as z_k - <z_k>, the
  // means taken in fp64 from the stored (fp32 in mixed precision) values.
  const double* zm = nullptr;
  if (c->vnull) {
    launch_field_means<TZ>(zk, c->dim, c->C, c->mpart, c->mean_blocks, c->zmean + 4 * k, c->stream);
    zm = c->zmean + 4 * k;
  }
  apply_K<TZ>(c, zk, w, zm);
  dcgs2_step<double, TZ>(V, ld, NV, k, c->H, c->m + 1, c->G, c->coef, c->part, c->part_blocks, c->cs, c->sn, c->g,
                         c->resid, c->stream, true, (TZ*)c->rhsT, c->dim, c->logn, c->NF);
}

// The graph of iteration k, captured on first use (and again when buffers or
// the spread capacity changed).  All its kernels use fixed device addresses,
// so one capture serves every restart cycle and every later solve of the
// context.  Returns null if capture is unavailable.  Live kernel timers bracket
// single launches on the stream, so while one is enabled no graph is used.
template <typename TZ>
ibr_ctx::IterGraph* iter_graph(ibr_ctx* c, int k) {
  if ((int)c->graphs.size() < c->m) c->graphs.resize(c->m);
  ibr_ctx::IterGraph& G = c->graphs[k];
  if (G.exec && G.version == c->graph_version) return &G;
  if (G.exec) {
    (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
  }
  hipStream_t s = c->stream;
  const int ps0 = c->cnt_ps, vc0 = c->cnt_vc;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
    c->use_graphs = false;
    return nullptr;
  }
  try {
    iteration_body<TZ>(c, k);
  } catch (...) {
    (void)hipStreamEndCapture(s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    c->cnt_ps = ps0;
    c->cnt_vc = vc0;
    throw;
  }
  const hipError_t e1 = hipStreamEndCapture(s, &graph);
  G.ps = c->cnt_ps - ps0;
  G.vc = c->cnt_vc - vc0;
  c->cnt_ps = ps0;
  c->cnt_vc = vc0;
  if (e1 != hipSuccess || !graph || hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    G.exec = nullptr;
    c->use_graphs = false;  // stay on plain stream launches
    return nullptr;
  }
  (void)hipGraphDestroy(graph);
  G.version = c->graph_version;
  return &G;
}

template <typename TZ>
ibr_status fgmres(ibr_ctx* c, ibr_info* info) {
  hipStream_t s = c->stream;
  const int64_t NV = c->NV;
  const int m = c->m;
  const int ldh = m + 1;
  TZ* Z = (TZ*)c->Zb;
  double* V = c->Vb;
  c->cnt_ps = 0;
  c->cnt_vc = 0;
  IBR_HIP(hipEventRecord(c->ev0, s));

  launch_sumsq_partial<double>(c->Bs, NV, c->part, c->part_blocks, s);
  launch_norm_finish(c->part, c->part_blocks, c->beta, s);
  IBR_HIP(hipMemcpyAsync(c->hres, c->beta, sizeof(double), hipMemcpyDeviceToHost, s));
  sync(c);
  const double bnorm = c->hres[0];
  const double target = c->p.rtol * bnorm;
  int total = 0, restarts = 0;
  ibr_status st = IBR_OK;
  double relres = 0.0;
  if (!(bnorm > 0.0)) {
    launch_fill<double>(c->Xs, NV, 0.0, s);
    if (!std::isfinite(bnorm)) st = IBR_ENUMERIC;
  } else {
    while (true) {
      // r = b - K x
      apply_K<double>(c, c->Xs, V);
      launch_axpby(c->Bs, V, NV, 1.0, -1.0, s);
      launch_sumsq_partial<double>(V, NV, c->part, c->part_blocks, s);
      launch_norm_finish(c->part, c->part_blocks, c->beta, s);
      IBR_HIP(hipMemcpyAsync(c->hres, c->beta, sizeof(double), hipMemcpyDeviceToHost, s));
      sync(c);
      const double rn = c->hres[0];
      relres = rn / bnorm;
      if (!std::isfinite(rn)) {
        st = IBR_ENUMERIC;
        break;
      }
      if (rn <= target) break;
      if (total >= c->p.max_iters) {
        st = IBR_ENOCONV;
        break;
      }
      ++restarts;
      launch_scale_copy<double, double>(V, V, NV, c->beta, s);
      launch_init_g(c->g, m + 1, c->beta, s);
      int kused = 0;
      bool stop = false;
      for (int k = 0; k < m; ++k) {
        ibr_ctx::IterGraph* G = c->use_graphs && !timers_any() ? iter_graph<TZ>(c, k) : nullptr;
        if (G) {
          IBR_HIP(hipGraphLaunch(G->exec, s));
          c->cnt_ps += G->ps;
          c->cnt_vc += G->vc;
        } else {
          iteration_body<TZ>(c, k);
        }
        IBR_HIP(hipMemcpyAsync(c->hres, c->resid, sizeof(double), hipMemcpyDeviceToHost, s));
        sync(c);
        ++total;
        kused = k + 1;
        const double est = c->hres[0];
        if (!std::isfinite(est)) {
          st = IBR_ENUMERIC;
          stop = true;
          break;
        }
        if (est <= target || total >= c->p.max_iters) break;
      }
      // the last column is still provisional: rotate it as it stands
      launch_givens_step(c->H, ldh, kused - 1, c->cs, c->sn, c->g, c->resid, s);
      launch_lsq_solve(c->H, ldh, kused, c->g, c->y, s);
      launch_combine<TZ, double>(Z, c->ldv, kused, c->y, c->Xs, NV, s, false, c->vnull ? c->zmean : nullptr, c->C,
                                 c->dim);
      if (stop) break;
    }
  }
  IBR_HIP(hipEventRecord(c->ev1, s));
  sync(c);
  float ms = 0;
  IBR_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  c->have_solution = true;
  if (info) {
    info->iters = total;
    info->restarts = restarts;
    info->ps_applications = c->cnt_ps;
    info->vcycles = c->cnt_vc;
    info->status = st;
    info->rel_residual = relres;
    info->ms = ms;
    double mx = 0;
    for (double v : c->shift_h) mx = std::max(mx, v);
    info->max_mobility_shift = mx;
  }
  return st;
}

// ---------------------------------------------------------------- set-up helpers
void validate(const ibr_params* p) {
  if (!p) throw Status(IBR_EINVAL, "params is NULL");
  if (p->dim != 2 && p->dim != 3) throw Status(IBR_EINVAL, "dim must be 2 or 3");
  const int lo = p->dim == 3 ? 8 : 16;
  const int hi = p->dim == 3 ? 512 : 4096;
  if (p->n < lo || p->n > hi || (p->n & (p->n - 1)))
    throw Status(IBR_EINVAL, "n must be a power of two in [" + std::to_string(lo) + ", " + std::to_string(hi) + "]");
  if (!(p->h > 0) || !std::isfinite(p->h)) throw Status(IBR_EINVAL, "h must be > 0");
  if (!(p->eta > 0) || !std::isfinite(p->eta)) throw Status(IBR_EINVAL, "eta must be > 0");
  if (p->rho < 0 || !std::isfinite(p->rho)) throw Status(IBR_EINVAL, "rho must be >= 0");
  if (p->rho > 0 && !(p->dt > 0)) throw Status(IBR_EINVAL, "dt must be > 0 when rho > 0");
  if (p->precision != IBR_FP64 && p->precision != IBR_MIXED) throw Status(IBR_EINVAL, "bad precision");
  if (p->pc != IBR_PC_LOWER && p->pc != IBR_PC_FULL) throw Status(IBR_EINVAL, "bad pc");
  if (p->n_s < 1 || p->n_s > 16) throw Status(IBR_EINVAL, "n_s must be in [1, 16]");
  if (p->restart < 1 || p->restart > 400) throw Status(IBR_EINVAL, "restart must be in [1, 400]");
  if (p->max_iters < 1) throw Status(IBR_EINVAL, "max_iters must be >= 1");
  if (!(p->rtol > 0) || p->rtol >= 1) throw Status(IBR_EINVAL, "rtol must be in (0, 1)");
  if (p->mg_pre < 0 || p->mg_post < 0 || p->mg_coarse < 1 || p->mg_pre > 16 || p->mg_post > 16 ||
      p->mg_coarse > 256)
    throw Status(IBR_EINVAL, "bad multigrid sweep counts");
  if (p->walls != IBR_WALLS_NONE && p->walls != IBR_WALLS_NOSLIP && p->walls != IBR_WALLS_BOX)
    throw Status(IBR_EINVAL, "bad walls");
  if (p->advection != IBR_ADVECT_CENTRED && p->advection != IBR_ADVECT_SL)
    throw Status(IBR_EINVAL, "bad advection");
  if (p->mobility != IBR_MOB_ANALYTIC && p->mobility != IBR_MOB_FITTED && p->mobility != IBR_MOB_AUTO)
    throw Status(IBR_EINVAL, "bad mobility");
  if (p->mobility == IBR_MOB_FITTED && (p->dim == 3 ? kFitRows : kFit2Rows) == 0)
    throw Status(IBR_EINVAL, "no fitted mobility table for this dimension");
}

MobParams mob_params(const ibr_ctx* c) {
  MobParams mp{};
  mp.dim = c->dim;
  mp.steady = c->steady ? 1 : 0;
  mp.eta = c->p.eta;
  mp.L = c->L;
  mp.a = (c->dim == 3 ? kA3D : kA2D) * c->h;
  if (c->dim == 3)
    mp.finf0 = 1.0 / (6.0 * kPi * mp.eta * mp.a);
  else
    mp.finf0 = std::log(c->L / (3.708 * mp.a)) / (4.0 * kPi * mp.eta);
  mp.periodic_shift = c->dim == 3 ? kPeriodic3D / (6.0 * kPi * mp.eta * c->L) : 0.0;
  if (!c->steady) {
    const double vm = std::pow(8.0 / 3.0, c->dim) * std::pow(c->h, c->dim);
    const double f0inv = (c->dim - 1.0) / c->dim * (c->p.dt / c->p.rho) / vm;
    mp.f00 = 1.0 / (1.0 / f0inv + 1.0 / mp.finf0);
    mp.alpha = std::sqrt(c->p.rho / (mp.eta * c->p.dt));
    mp.dt_rho = c->p.dt / c->p.rho;
  }
  mp.h = c->h;
  const bool fitted = c->p.mobility == IBR_MOB_FITTED || c->p.mobility == IBR_MOB_AUTO;
  if (fitted && c->dim == 2 && kFit2Rows > 0) {
    // Appendix B's forms
    mp.ah = kFit2Ah;
    for (int i = 0; i < 9; ++i) mp.f2s[i] = kFit2Steady[i];
    const double beta = c->steady ? 0.0 : c->p.eta * c->p.dt / (c->p.rho * c->h * c->h);
    if (!c->steady && !c->walls) mp.mean_mode = c->p.dt / (c->p.rho * c->vol);
    if (c->steady || beta > kFit2Beta[kFit2Rows - 1]) {
      mp.fit = 3;
      // the periodic square's self mobility ln(l / (3.708 a)) / (4 pi eta)
      mp.self0 = std::log(c->L / (3.708 * kFit2Ah * c->h)) / (4.0 * kPi * mp.eta);
    } else {
      mp.fit = 4;
      mp.beta = beta;
      const double z0 = 1.0 / (2.0 * (8.0 / 3.0) * (8.0 / 3.0));  // h^2 / (2 V_m), the inviscid self mobility
      mp.phi0 = (z0 + kFit2Z[0] * beta * beta * beta * std::log(beta)) /
                (1.0 + kFit2Z[1] * beta + kFit2Z[2] * beta * beta + kFit2Z[3] * beta * beta * beta * beta);
      int i = 0;
      while (i + 1 < kFit2Rows && kFit2Beta[i + 1] < beta) ++i;
      double t = 0.0;
      int k = i;
      if (beta > kFit2Beta[i] && i + 1 < kFit2Rows) {
        k = i + 1;
        t = std::log(beta / kFit2Beta[i]) / std::log(kFit2Beta[k] / kFit2Beta[i]);
      }
      mp.tw = t;
      const int row[2] = {i, k};
      for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 13; ++q) mp.f2r[r][q] = kFit2Row[row[r]][q];
    }
  } else if (fitted && c->dim == 3 && kFitRows > 0) {
    mp.ah = kFitAh;
    for (int i = 0; i < 7; ++i) mp.fs[i] = kFitSteady[i];
    const double beta = c->steady ? 0.0 : c->p.eta * c->p.dt / (c->p.rho * c->h * c->h);
    // the fitted forms describe the kernel's pair mobility without the box;
    // an unsteady periodic box adds its mean mode (walls block it)
    if (!c->steady && !c->walls) mp.mean_mode = c->p.dt / (c->p.rho * c->vol);
    if (c->steady || beta > kFitBeta[kFitRows - 1]) {
      mp.fit = 1;
      if (!c->steady) mp.periodic_shift = 0.0;  // an unsteady box keeps S: no mean-flow shift
    } else {
      mp.fit = 2;
      mp.beta = beta;
      const double z1 = kFitZ[0], z2 = kFitZ[1], z3 = kFitZ[2];
      const double z0 = 1.5 * std::pow(8.0 / 3.0, 3);  // 3 V_m / (2 h^3), the inviscid self mobility
      mp.phi0 = (1.0 + z1 * std::sqrt(beta) + z2 * beta) / (z0 + z3 * beta + 6.0 * kPi * kFitAh * z2 * beta * beta);
      // the rows around beta: their forms at beta are blended with weights
      // linear in log beta (below the first row, that row alone)
      int i = 0;
      while (i + 1 < kFitRows && kFitBeta[i + 1] < beta) ++i;
      double t = 0.0;
      int k = i;
      if (beta > kFitBeta[i] && i + 1 < kFitRows) {
        k = i + 1;
        t = std::log(beta / kFitBeta[i]) / std::log(kFitBeta[k] / kFitBeta[i]);
      }
      mp.tw = t;
      const int row[2] = {i, k};
      for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < 10; ++q) mp.fa[r][q] = kFitA[row[r]][q];
        for (int q = 0; q < 6; ++q) mp.fb[r][q] = kFitB[row[r]][q];
      }
    }
  }
  return mp;
}

double self_term(const MobParams& mp) {
  if (mp.fit == 1) return 1.0 / (6.0 * kPi * mp.eta * mp.ah * mp.h) - mp.periodic_shift + mp.mean_mode;
  if (mp.fit == 2) return mp.phi0 * mp.beta / (mp.eta * mp.h) + mp.mean_mode;
  if (mp.fit == 3) return mp.self0 + mp.mean_mode;
  if (mp.fit == 4) return mp.phi0 * mp.beta / mp.eta + mp.mean_mode;
  if (!mp.steady) return mp.f00;
  if (mp.dim == 3) return mp.finf0 - mp.periodic_shift;
  return mp.finf0;
}

void setup_markers(ibr_ctx* c) {
  hipStream_t s = c->stream;
  launch_marker_setup(c->dim, c->logn, c->N, c->h, c->L, c->R, c->taps, c->tile_of, c->tile_log, s, c->wm);
  launch_bin_markers(c->N, c->ntiles, c->tile_of, c->counts, c->toff, c->cursor, c->perm, s);
  launch_active_tiles(c->dim, c->tiles_log, c->toff, c->flags, c->active, c->nactive_d, s);
  int na = 0;
  IBR_HIP(hipMemcpyAsync(c->hres, c->nactive_d, sizeof(int), hipMemcpyDeviceToHost, s));
  sync(c);
  std::memcpy(&na, c->hres, sizeof(int));
  c->nactive = na;
  if (na > c->act_cap) {
    // grow the spread grid capacity; graphs captured with the old size are stale
    c->act_cap = std::min(c->ntiles, na + na / 4 + 8);
    ++c->graph_version;
  }
}

void factor_blocks(ibr_ctx* c) {
  hipStream_t s = c->stream;
  const int nb = c->nb;
  c->mp = mob_params(c);
  c->f0 = self_term(c->mp);
  launch_mob_assemble(c->dim, nb, c->off_d, c->moff_d, c->R, c->mp, c->Mb, c->max_np, s);
  std::vector<int> idx(nb, 0), act(nb, 1), fail(nb, 0);
  c->shift_h.assign(nb, 0.0);
  for (int round = 0; round < kNumShifts; ++round) {
    for (int b = 0; b < nb; ++b) c->shift_h[b] = kShifts[idx[b]];
    IBR_HIP(hipMemcpyAsync(c->shift_d, c->shift_h.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
    IBR_HIP(hipMemcpyAsync(c->act_d, act.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    launch_chol(nb, c->off_d, c->dim, c->moff_d, c->Mb, c->Lb, c->Xb, c->act_d, c->shift_d, c->f0, kPivotTol, c->fail_d,
                c->max_rows, s);
    IBR_HIP(hipMemcpyAsync(fail.data(), c->fail_d, nb * sizeof(int), hipMemcpyDeviceToHost, s));
    sync(c);
    bool any = false;
    for (int b = 0; b < nb; ++b) {
      if (act[b] && fail[b]) {
        any = true;
        if (idx[b] + 1 >= kNumShifts) throw Status(IBR_EFACTOR, "mobility block " + std::to_string(b) + " could not be factored");
        ++idx[b];
      } else {
        act[b] = 0;
      }
    }
    if (!any) break;
  }
  launch_chol_inverse(nb, c->off_d, c->dim, c->moff_d, c->Lb, c->Minv, c->Xb, (c->max_rows + 15) & ~15, s);
  sync(c);
}

void build_rhs_markers(ibr_ctx* c) {
  // W = -V in the constraint block of b (with moving walls -(V - u_b))
  launch_marker_velocity(c->dim, c->N, c->R, c->body_d, c->X, c->U, c->Om, c->L, c->Vm, c->stream);
  if (c->wallvel) launch_sub_background_markers(c->Vm, c->R, c->N, c->dim, c->dim - 1, c->L, c->wvel, c->stream);
  launch_copy<double, double>(c->Vm, c->Bs + c->NF, (int64_t)c->N * c->dim, c->stream);
  launch_axpby(c->Vm, c->Bs + c->NF, (int64_t)c->N * c->dim, -1.0, 0.0, c->stream);
  if (c->nq) {
    // free bodies: no prescribed marker velocity; their rows of the body block carry the applied load
    launch_free_zero_markers(c->dim, c->N, c->body_d, c->free_d, c->Bs + c->NF, c->stream);
    IBR_HIP(hipMemcpyAsync(c->Bs + c->NF + (int64_t)c->dim * c->N, c->load_h.data(), c->nq * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  }
}

// Bodies overlap (Sec. 2 takes them disjoint; Sec. 5.3: markers closer than
// about h/2 make the mobility too ill-conditioned to solve) when a marker of
// one body lies closer than h to a marker of another: the two kernels then
// nearly coincide.  Only pairs of bodies whose bounding spheres (about the
// given centres, minimum image along periodic axes) come within h of each
// other are compared marker by marker.  Throws IBR_EINVAL naming the bodies.
void check_overlap(int d, double h, double L, int wm, int nb, const int* off, const double* R,
                   const double* X) {
  if (nb < 2) return;
  auto delta = [&](const double* a, const double* b, int ax) {
    double dx = a[ax] - b[ax];
    if (!((wm >> ax) & 1)) dx -= L * std::nearbyint(dx / L);
    return dx;
  };
  std::vector<double> rad(nb, 0.0);
  for (int p = 0; p < nb; ++p)
    for (int i = off[p]; i < off[p + 1]; ++i) {
      double r2 = 0;
      for (int a = 0; a < d; ++a) {
        const double dx = delta(R + (int64_t)i * d, X + (int64_t)p * d, a);
        r2 += dx * dx;
      }
      rad[p] = std::max(rad[p], std::sqrt(r2));
    }
  const double h2 = h * h;
  for (int p = 0; p < nb; ++p)
    for (int q = p + 1; q < nb; ++q) {
      double c2 = 0;
      for (int a = 0; a < d; ++a) {
        const double dx = delta(X + (int64_t)p * d, X + (int64_t)q * d, a);
        c2 += dx * dx;
      }
      if (std::sqrt(c2) > rad[p] + rad[q] + h) continue;
      for (int i = off[p]; i < off[p + 1]; ++i)
        for (int j = off[q]; j < off[q + 1]; ++j) {
          double r2 = 0;
          for (int a = 0; a < d; ++a) {
            const double dx = delta(R + (int64_t)i * d, R + (int64_t)j * d, a);
            r2 += dx * dx;
          }
          if (r2 < h2)
            throw Status(IBR_EINVAL, "bodies " + std::to_string(p) + " and " + std::to_string(q) +
                                         " overlap: markers " + std::to_string(i) + " and " + std::to_string(j) +
                                         " are closer than h");
        }
    }
}

template <typename F>
ibr_status guard(ibr_ctx* c, F&& f) {
  try {
    f();
    if (c) c->err.clear();
    return IBR_OK;
  } catch (const Status& e) {
    if (c) c->err = e.what();
    return e.code;
  } catch (const DeviceError& e) {
    if (c) c->err = e.what();
    return IBR_EDEVICE;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return IBR_ENOMEM;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return IBR_EDEVICE;
  }
}

void require_bodies(const ibr_ctx* c) {
  if (c->N <= 0) throw Status(IBR_ESTATE, "ibr_set_bodies has not been called");
}

}  // namespace

// ---------------------------------------------------------------- ctx members
void ibr_ctx::drop_graphs() {
  for (IterGraph& G : graphs) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
  }
  graphs.clear();
}

ibr_ctx::~ibr_ctx() {
  drop_graphs();
  free_markers();
  for (void* q : {(void*)Xs, (void*)Bs, (void*)T1, (void*)T2, (void*)Nprev, (void*)Ncur, (void*)H, (void*)cs,
                  (void*)sn, (void*)g, (void*)y, (void*)resid, (void*)beta, (void*)hc2, (void*)part, (void*)Qi,
                  (void*)Zi, (void*)rhsT, (void*)qT, (void*)phiT, (void*)Hi, (void*)csi, (void*)sni, (void*)gi,
                  (void*)yi, (void*)residi, (void*)betai, (void*)hc2i, (void*)vmean, (void*)mpart, (void*)addc,
                  (void*)lsum_part, (void*)part2, (void*)G, (void*)coef, (void*)flag, (void*)zmean})
    dev_free(q);
  mg64.release();
  mg32.release();
  if (hres) (void)hipHostFree(hres);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void ibr_ctx::clear_free() {
  dev_free(free_d);
  dev_free(yoff_d);
  dev_free(Yf);
  dev_free(Nf);
  free_d = nullptr;
  yoff_d = nullptr;
  Yf = Nf = nullptr;
  free_h.clear();
  load_h.clear();
  nfree = 0;
  nq = 0;
}

void ibr_ctx::free_markers() {
  clear_free();
  for (void* q : {(void*)off_d, (void*)body_d, (void*)R, (void*)X, (void*)U, (void*)Om, (void*)Vm, (void*)taps.base,
                  (void*)taps.w64, (void*)taps.w32, (void*)tile_of, (void*)counts, (void*)toff, (void*)cursor,
                  (void*)perm, (void*)flags, (void*)active, (void*)nactive_d, (void*)moff_d, (void*)Mb, (void*)Lb,
                  (void*)Xb, (void*)Minv, (void*)shift_d, (void*)act_d, (void*)fail_d, (void*)Vb, Zb, (void*)lamd,
                  (void*)dU})
    dev_free(q);
  off_d = body_d = nullptr;
  R = X = U = Om = Vm = nullptr;
  taps = MarkerTaps{nullptr, nullptr, nullptr};
  tile_of = counts = toff = cursor = perm = flags = active = nactive_d = nullptr;
  moff_d = nullptr;
  Mb = Lb = Xb = Minv = shift_d = nullptr;
  act_d = fail_d = nullptr;
  Vb = nullptr;
  Zb = nullptr;
  lamd = dU = nullptr;
  nbcap = 0;
  mcap = 0;
}

void ibr_ctx::alloc_grid() {
  const int d = dim;
  NF = (int64_t)(d + 1) * C;
  Nprev = track<double>((int64_t)d * C);
  Ncur = track<double>((int64_t)d * C);
  m = p.restart;
  ns = p.n_s;
  H = track<double>((int64_t)(m + 1) * m);
  cs = track<double>(m + 1);
  sn = track<double>(m + 1);
  g = track<double>(m + 2);
  y = track<double>(m + 1);
  resid = track<double>(1);
  beta = track<double>(1);
  hc2 = track<double>(m + 2);
  // partial-sum blocks of the reductions, from the vector length: one
  // element per thread at least, up to the 1024 blocks that stream a large
  // state at full bandwidth (the update pass shares this grid, so fewer
  // blocks on mid-size grids slowed it); small grids' finishing kernels
  // then sum few partials (all reductions are grid-stride)
  part_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(8, (NF + 255) / 256));
  mean_blocks = (int)std::min<int64_t>(256, std::max<int64_t>(1, (C + 1023) / 1024));
  part = track<double>((int64_t)(2 * m + 8) * part_blocks);
  if (ns <= 3) {
    gpart_blocks = stokes_gram_blocks(d, logn);
    gpart = track<double>((int64_t)(ns * (ns + 1) / 2 + ns) * gpart_blocks);
  }
  part2 = track<double>((int64_t)(m + 3) * part_blocks);
  G = track<double>(2 * m + 8);
  coef = track<double>(2 * m + 8);
  zmean = track<double>(4 * (int64_t)m);
  flag = track<int>(4);
  Hi = track<double>((int64_t)(ns + 1) * ns);
  csi = track<double>(ns + 1);
  sni = track<double>(ns + 1);
  gi = track<double>(ns + 2);
  yi = track<double>(ns + 1);
  residi = track<double>(1);
  betai = track<double>(1);
  hc2i = track<double>(ns + 2);
  vmean = track<double>(4);
  mpart = track<double>(4 * 256);
  addc = track<double>(4);
  lsum_part = track<double>(4 * 64);
  const int64_t tsz = mixed ? 4 : 8;
  auto talloc = [&](int64_t count) -> void* {
    bytes += count * tsz;
    return mixed ? (void*)dev_alloc<float>(count) : (void*)dev_alloc<double>(count);
  };
  Qi = talloc((int64_t)(ns + 1) * NF);
  Zi = talloc((int64_t)ns * NF);
  rhsT = talloc(NF);
  qT = talloc(C);
  phiT = talloc(C);
  if (mixed) {
    mg32.init(d, logn, d, wm);
    bytes += MGHier<float>::bytes(d, logn, d, walls);
  } else {
    mg64.init(d, logn, d, wm);
    bytes += MGHier<double>::bytes(d, logn, d, walls);
  }
  IBR_HIP(hipHostMalloc((void**)&hres, 64, hipHostMallocDefault));
  IBR_HIP(hipEventCreate(&ev0));
  IBR_HIP(hipEventCreate(&ev1));
  tile_log = d == 3 ? 3 : 4;
  if (tile_log > logn) tile_log = logn;
  tiles_log = logn - tile_log;
  ntiles = 1 << (d * tiles_log);
}

void ibr_ctx::alloc_markers(int Nnew) {
  // Grid-sized stacked vectors depend on N through the Lambda tail.
  const int d = dim;
  if (Nnew <= Ncap && Vb) return;
  const int cap = std::max(Nnew, 16);
  for (void* q : {(void*)R, (void*)Vm, (void*)body_d, (void*)taps.base, (void*)taps.w64, (void*)taps.w32,
                  (void*)tile_of, (void*)perm, (void*)Vb, Zb, (void*)lamd, (void*)dU, (void*)Xs, (void*)Bs, (void*)T1,
                  (void*)T2})
    dev_free(q);
  R = Vm = lamd = dU = Xs = Bs = T1 = T2 = Vb = nullptr;
  body_d = tile_of = perm = nullptr;
  taps = MarkerTaps{nullptr, nullptr, nullptr};
  Zb = nullptr;
  Ncap = 0;
  Ncap = cap;
  // Lambda (dim per marker) and room for the body block of free kinematics
  // (dim + rotations per body, at most one body per marker)
  const int64_t NVc = NF + (int64_t)(d + d + (d == 3 ? 3 : 1)) * cap;
  R = track<double>((int64_t)cap * d);
  Vm = track<double>((int64_t)cap * d);
  body_d = track<int>(cap);
  taps.base = track<int>((int64_t)cap * 6);
  taps.w64 = track<double>((int64_t)cap * 24);
  taps.w32 = track<float>((int64_t)cap * 24);
  tile_of = track<int>(cap);
  perm = track<int>(cap);
  lamd = track<double>((int64_t)cap * d);
  dU = track<double>((int64_t)cap * d);
  Xs = track<double>(NVc);
  Bs = track<double>(NVc);
  T1 = track<double>(NVc);
  T2 = track<double>(NVc);
  const int64_t ldc = (NVc + 63) & ~(int64_t)63;  // basis stride at capacity
  Vb = track<double>((int64_t)(m + 1) * ldc);
  if (mixed) {
    Zb = dev_alloc<float>((int64_t)m * ldc);
    bytes += (int64_t)m * ldc * 4;
  } else {
    Zb = dev_alloc<double>((int64_t)m * ldc);
    bytes += (int64_t)m * ldc * 8;
  }
  launch_fill<double>(Xs, NVc, 0.0, stream);
  launch_fill<double>(Bs, NVc, 0.0, stream);
}

// ---------------------------------------------------------------- C ABI
extern "C" {

void ibr_default_params(ibr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dim = 3;
  p->n = 32;
  p->h = 1.0 / 32.0;
  p->rho = 0.0;
  p->eta = 1.0;
  p->dt = 0.0;
  p->precision = IBR_FP64;
  p->pc = IBR_PC_LOWER;
  p->n_s = 2;
  p->restart = 100;
  p->max_iters = 1000;
  p->rtol = 1e-8;
  p->mg_pre = 2;
  p->mg_post = 2;
  p->mg_coarse = 4;
  p->device = 0;
  p->stream = nullptr;
  p->graphs = 1;
  p->walls = IBR_WALLS_NONE;
  p->advection = IBR_ADVECT_CENTRED;
  p->mobility = IBR_MOB_AUTO;
}

const char* ibr_status_string(int st) {
  switch (st) {
    case IBR_OK: return "ok";
    case IBR_EINVAL: return "invalid argument";
    case IBR_ENOMEM: return "out of device memory";
    case IBR_ENOCONV: return "not converged";
    case IBR_EBREAKDOWN: return "Krylov breakdown";
    case IBR_EFACTOR: return "mobility block factorisation failed";
    case IBR_ENUMERIC: return "NaN or Inf in the residual";
    case IBR_EDEVICE: return "device error";
    case IBR_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

ibr_status ibr_create(const ibr_params* params, ibr_ctx** out) {
  if (!out) return IBR_EINVAL;
  *out = nullptr;
  std::unique_ptr<ibr_ctx> c(new ibr_ctx());
  ibr_status st = guard(c.get(), [&] {
    validate(params);
    c->p = *params;
    IBR_HIP(hipSetDevice(params->device));
    c->dim = params->dim;
    c->n = params->n;
    c->logn = ilog2(params->n);
    c->C = (int64_t)1 << (c->dim * c->logn);
    c->h = params->h;
    c->L = params->n * params->h;
    c->vol = std::pow(c->L, c->dim);
    c->steady = params->rho == 0.0;
    c->wm = wall_mask(params->walls, params->dim);
    c->walls = c->wm != 0;
    c->vnull = c->steady && !c->walls;
    c->c0 = c->steady ? 0.0 : params->rho / params->dt;
    c->ch2 = params->eta / (c->h * c->h);
    c->inv_h = 1.0 / c->h;
    c->mixed = params->precision == IBR_MIXED;
    c->use_graphs = params->graphs != 0;
    if (params->stream) {
      c->stream = (hipStream_t)params->stream;
    } else {
      IBR_HIP(hipStreamCreate(&c->stream));
      c->own_stream = true;
    }
    c->alloc_grid();
    sync(c.get());
  });
  if (st != IBR_OK) return st;
  *out = c.release();
  return IBR_OK;
}

void ibr_destroy(ibr_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->p.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* ibr_last_error(const ibr_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t ibr_footprint_bytes(const ibr_params* p, int nbodies, const int* markers_per_body) {
  if (!p || p->dim < 2 || p->dim > 3 || p->n < 4 || nbodies < 0 || (nbodies > 0 && !markers_per_body)) return 0;
  const int d = p->dim;
  int64_t nmarkers = 0, mtot = 0;
  for (int b = 0; b < nbodies; ++b) {
    const int np = markers_per_body[b];
    if (np < 0) return 0;
    nmarkers += np;
    const int64_t ld = ((int64_t)d * np + 15) & ~(int64_t)15;  // as ibr_set_bodies lays the blocks out
    mtot += ld * ld;
  }
  const int64_t C = (int64_t)1 << (d * ilog2(p->n));
  const int64_t NF = (int64_t)(d + 1) * C;
  const int64_t NV = NF + (int64_t)(d + d + (d == 3 ? 3 : 1)) * std::max<int64_t>(nmarkers, 16);
  const int m = p->restart > 0 ? p->restart : 100;
  const int ns = p->n_s > 0 ? p->n_s : 2;
  const int64_t ts = p->precision == IBR_MIXED ? 4 : 8;
  size_t b = 0;
  const int64_t ldv = (NV + 63) & ~(int64_t)63;
  b += (size_t)(m + 1) * ldv * 8;      // V basis
  b += (size_t)m * ldv * ts;           // Z basis
  b += (size_t)4 * NV * 8;             // x, b, two temporaries
  b += (size_t)2 * d * C * 8;          // advection history
  b += (size_t)((2 * ns + 2) * NF + 2 * C) * ts;  // inner bases and P_S^-1 scratch
  if (ns <= 3) b += (size_t)(ns * (ns + 1) / 2 + ns) * (size_t)stokes_gram_blocks(d, ilog2(p->n)) * 8;  // Gram partials
  const bool w = p->walls == IBR_WALLS_NOSLIP || p->walls == IBR_WALLS_BOX;
  b += ts == 4 ? MGHier<float>::bytes(d, ilog2(p->n), d, w) : MGHier<double>::bytes(d, ilog2(p->n), d, w);
  b += (size_t)4 * mtot * 8;           // mobility blocks: M~, its factor, the inverse factor, M~^-1
  b += (size_t)nmarkers * 420;         // per-marker positions, taps, weights, binning, forces
  b += (size_t)16 << 20;               // the allocator's rounding of the context's ~80 buffers
  return b;
}

ibr_status ibr_set_bodies(ibr_ctx* c, int nbodies, const int* offsets, const double* R, const double* centres) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    if (nbodies < 1 || !offsets || !R || !centres) throw Status(IBR_EINVAL, "need nbodies >= 1, offsets, R, centres");
    if (offsets[0] != 0) throw Status(IBR_EINVAL, "offsets[0] must be 0");
    int maxnp = 0;
    for (int b = 0; b < nbodies; ++b) {
      const int np = offsets[b + 1] - offsets[b];
      if (np < 1) throw Status(IBR_EINVAL, "every body needs at least one marker");
      maxnp = std::max(maxnp, np);
    }
    const int d = c->dim;
    if (maxnp * d > kMaxBlockRows)
      throw Status(IBR_EINVAL, "a body has more than " + std::to_string(kMaxBlockRows / d) + " markers");
    const int N = offsets[nbodies];
    for (int64_t i = 0; i < (int64_t)N * d; ++i)
      if (!std::isfinite(R[i])) throw Status(IBR_EINVAL, "marker positions must be finite");
    for (int64_t i = 0; i < (int64_t)nbodies * d; ++i)
      if (!std::isfinite(centres[i])) throw Status(IBR_EINVAL, "centres must be finite");
    check_overlap(d, c->h, c->L, c->wm, nbodies, offsets, R, centres);
    if (c->walls) {
      for (int64_t m = 0; m < N; ++m)
        for (int a = 0; a < d; ++a) {
          if (!((c->wm >> a) & 1)) continue;
          const double z = R[m * d + a];
          if (!(z > 0.0 && z < c->L)) throw Status(IBR_EINVAL, "markers must lie strictly between the walls");
        }
      c->wall_z.assign((size_t)nbodies * d, 0.0);
      c->wall_lo.assign((size_t)nbodies * d, 0.0);
      c->wall_hi.assign((size_t)nbodies * d, 0.0);
      c->wall_uz.assign((size_t)nbodies * d, 0.0);
      for (int b = 0; b < nbodies; ++b)
        for (int a = 0; a < d; ++a) {
          const double zc = centres[b * d + a];
          double lo = 0.0, hi = 0.0;
          for (int m = offsets[b]; m < offsets[b + 1]; ++m) {
            lo = std::min(lo, R[(int64_t)m * d + a] - zc);
            hi = std::max(hi, R[(int64_t)m * d + a] - zc);
          }
          c->wall_z[b * d + a] = zc;
          c->wall_lo[b * d + a] = lo;
          c->wall_hi[b * d + a] = hi;
        }
    }
    IBR_HIP(hipSetDevice(c->p.device));
    sync(c);
    // body-sized buffers grow with the body count and the blocks' size and are
    // reused otherwise (a served request brings new bodies: no allocation
    // unless they need more room than any before); tile buffers depend on
    // the grid only
    auto drop = [](auto*& q) {
      dev_free((void*)q);
      q = nullptr;
    };
    int64_t mtot = 0;
    for (int b = 0; b < nbodies; ++b) {
      const int64_t ld = ((int64_t)d * (offsets[b + 1] - offsets[b]) + 15) & ~(int64_t)15;
      mtot += ld * ld;
    }
    if (nbodies > c->nbcap) {
      drop(c->off_d);
      drop(c->X);
      drop(c->U);
      drop(c->Om);
      drop(c->moff_d);
      drop(c->shift_d);
      drop(c->act_d);
      drop(c->fail_d);
      c->nbcap = 0;
    }
    if (mtot > c->mcap) {
      drop(c->Mb);
      drop(c->Lb);
      drop(c->Xb);
      drop(c->Minv);
      c->mcap = 0;
    }
    c->N = 0;
    c->clear_free();
    c->drop_graphs();
    ++c->graph_version;
    c->act_cap = 0;
    const bool grow = N > c->Ncap || !c->Vb;
    c->alloc_markers(N);
    c->nb = nbodies;
    c->N = N;
    c->NV = c->NF + (int64_t)d * N;
    c->ldv = (c->NV + 63) & ~(int64_t)63;
    c->off_h.assign(offsets, offsets + nbodies + 1);
    if (c->nbcap == 0) {
      c->off_d = dev_alloc<int>(nbodies + 1);
      c->X = dev_alloc<double>((int64_t)nbodies * d);
      c->U = dev_alloc<double>((int64_t)nbodies * d);
      c->Om = dev_alloc<double>((int64_t)nbodies * 3);
      c->moff_d = dev_alloc<int64_t>(nbodies + 1);
      c->shift_d = dev_alloc<double>(nbodies);
      c->act_d = dev_alloc<int>(nbodies);
      c->fail_d = dev_alloc<int>(nbodies);
      c->nbcap = nbodies;
    }
    if (!c->counts) {
      c->counts = dev_alloc<int>(c->ntiles);
      c->toff = dev_alloc<int>(c->ntiles + 1);
      c->cursor = dev_alloc<int>(c->ntiles);
      c->flags = dev_alloc<int>(c->ntiles);
      c->active = dev_alloc<int>(c->ntiles);
      c->nactive_d = dev_alloc<int>(1);
    }
    std::vector<int> body(N);
    for (int b = 0; b < nbodies; ++b)
      for (int i = offsets[b]; i < offsets[b + 1]; ++i) body[i] = b;
    c->moff_h.assign(nbodies + 1, 0);
    c->max_np = maxnp;
    c->max_rows = maxnp * d;
    for (int b = 0; b < nbodies; ++b) {
      const int64_t ld = ((int64_t)d * (offsets[b + 1] - offsets[b]) + 15) & ~(int64_t)15;
      c->moff_h[b + 1] = c->moff_h[b] + ld * ld;
    }
    if (c->mcap == 0) {
      c->Mb = dev_alloc<double>(mtot);
      c->Lb = dev_alloc<double>(mtot);
      c->Xb = dev_alloc<double>(mtot);
      c->Minv = dev_alloc<double>(mtot);
      c->mcap = mtot;
    }
    hipStream_t s = c->stream;
    IBR_HIP(hipMemcpyAsync(c->off_d, offsets, (nbodies + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    IBR_HIP(hipMemcpyAsync(c->R, R, (size_t)N * d * sizeof(double), hipMemcpyHostToDevice, s));
    IBR_HIP(hipMemcpyAsync(c->X, centres, (size_t)nbodies * d * sizeof(double), hipMemcpyHostToDevice, s));
    IBR_HIP(hipMemcpyAsync(c->body_d, body.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
    IBR_HIP(hipMemcpyAsync(c->moff_d, c->moff_h.data(), (nbodies + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    // (the blocks' padding rows and columns are never read: no fill)
    launch_fill<double>(c->U, (int64_t)nbodies * d, 0.0, s);
    launch_fill<double>(c->Om, (int64_t)nbodies * 3, 0.0, s);
    // positions are wrapped into the box by the marker set-up kernel's taps; keep R itself wrapped too
    launch_move_markers(d, N, nbodies, c->R, c->X, c->body_d, c->U, 0.0, c->L, s);
    setup_markers(c);
    factor_blocks(c);
    if (grow) launch_fill<double>(c->Xs, c->NV, 0.0, s);
    build_rhs_markers(c);
    c->have_prev = false;
    sync(c);
  });
}

ibr_status ibr_set_velocities(ibr_ctx* c, const double* U, const double* Omega) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (!U || !Omega) throw Status(IBR_EINVAL, "U and Omega are required");
    const int d = c->dim;
    const int no = d == 3 ? 3 : 1;
    for (int64_t i = 0; i < (int64_t)c->nb * d; ++i)
      if (!std::isfinite(U[i])) throw Status(IBR_EINVAL, "U must be finite");
    bool rot = false;
    for (int64_t i = 0; i < (int64_t)c->nb * no; ++i) {
      if (!std::isfinite(Omega[i])) throw Status(IBR_EINVAL, "Omega must be finite");
      rot = rot || Omega[i] != 0.0;
    }
    c->rotating = rot;
    if (c->walls)
      for (int64_t i = 0; i < (int64_t)c->nb * d; ++i) c->wall_uz[i] = U[i];
    IBR_HIP(hipSetDevice(c->p.device));
    IBR_HIP(hipMemcpyAsync(c->U, U, (size_t)c->nb * d * sizeof(double), hipMemcpyHostToDevice, c->stream));
    IBR_HIP(hipMemcpyAsync(c->Om, Omega, (size_t)c->nb * no * sizeof(double), hipMemcpyHostToDevice, c->stream));
    build_rhs_markers(c);
    sync(c);
  });
}

}  // extern "C"

namespace {

// A caller pointer passed to a device-pointer entry point must be device
// memory of the context's GPU (hipMalloc'd, e.g. a torch tensor's data).
void require_device_ptr(const ibr_ctx* c, const void* ptr, const char* what) {
  if (!ptr) return;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    throw Status(IBR_EINVAL, std::string(what) + " is not device memory");
  }
  if (a.type != hipMemoryTypeDevice || a.device != c->p.device)
    throw Status(IBR_EINVAL, std::string(what) + " is not device memory of the context's GPU");
}

void set_rhs_impl(ibr_ctx* c, const double* gh, const double* hp, hipMemcpyKind kind) {
  require_bodies(c);
  const int d = c->dim;
  hipStream_t s = c->stream;
  IBR_HIP(hipSetDevice(c->p.device));
  if (gh)
    IBR_HIP(hipMemcpyAsync(c->Bs, gh, (size_t)d * c->C * sizeof(double), kind, s));
  else
    launch_fill<double>(c->Bs, (int64_t)d * c->C, 0.0, s);
  if (hp)
    IBR_HIP(hipMemcpyAsync(c->Bs + (int64_t)d * c->C, hp, (size_t)c->C * sizeof(double), kind, s));
  else
    launch_fill<double>(c->Bs + (int64_t)d * c->C, c->C, 0.0, s);
  // consistency: <h> = 0 always, <g> = 0 for periodic steady Stokes (Sec. 3.4)
  launch_field_means<double>(c->Bs + (int64_t)d * c->C, 1, c->C, c->mpart, c->mean_blocks, c->vmean, s);
  launch_sub_field_mean<double>(c->Bs + (int64_t)d * c->C, 1, c->C, c->vmean, s);
  // with walls the normal components' wall faces are not unknowns: no momentum there
  if (c->walls) launch_zero_wall_faces(d, c->logn, c->Bs, c->wm, s);
  if (c->vnull) {
    launch_field_means<double>(c->Bs, d, c->C, c->mpart, c->mean_blocks, c->vmean, s);
    launch_sub_field_mean<double>(c->Bs, d, c->C, c->vmean, s);
  }
  sync(c);
}

void get_solution_impl(ibr_ctx* c, double* u, double* pr, double* lambda, double* F, double* T,
                       hipMemcpyKind kind) {
  require_bodies(c);
  IBR_HIP(hipSetDevice(c->p.device));
  hipStream_t s = c->stream;
  const int d = c->dim;
  double* pdev = c->Xs + (int64_t)d * c->C;
  launch_field_means<double>(pdev, 1, c->C, c->mpart, c->mean_blocks, c->vmean, s);
  launch_sub_field_mean<double>(pdev, 1, c->C, c->vmean, s);
  if (u) {
    IBR_HIP(hipMemcpyAsync(u, c->Xs, (size_t)d * c->C * sizeof(double), kind, s));
    // the state holds u - u_b: add the walls' background flow to the copy
    if (c->wallvel && kind == hipMemcpyDeviceToDevice)
      launch_add_background(d, c->logn, u, c->h, c->L, d - 1, c->wvel, 1.0, 0, s);
  }
  if (pr) IBR_HIP(hipMemcpyAsync(pr, pdev, (size_t)c->C * sizeof(double), kind, s));
  if (lambda) IBR_HIP(hipMemcpyAsync(lambda, c->Xs + c->NF, (size_t)c->N * d * sizeof(double), kind, s));
  if (F || T) {
    const int nt = d == 3 ? 3 : 1;
    launch_body_force_torque(d, c->nb, c->off_d, c->R, c->X, c->L, c->Xs + c->NF, c->T1, c->T1 + c->nb * 3, s);
    if (F) IBR_HIP(hipMemcpyAsync(F, c->T1, (size_t)c->nb * d * sizeof(double), kind, s));
    if (T) IBR_HIP(hipMemcpyAsync(T, c->T1 + c->nb * 3, (size_t)c->nb * nt * sizeof(double), kind, s));
  }
  sync(c);
  if (u && c->wallvel && kind == hipMemcpyDeviceToHost) {
    // host copy: the same background flow, added on the host
    const int n = c->n;
    const int64_t C = c->C;
    for (int a = 0; a < d; ++a)
      for (int64_t i = 0; i < C; ++i) {
        const int k = (int)(i >> ((d - 1) * c->logn));  // coordinate along the last axis
        const double z = (k + (a == d - 1 ? 0.0 : 0.5)) * c->h;
        u[a * C + i] += c->wvel.lo[a] + (c->wvel.hi[a] - c->wvel.lo[a]) * z / c->L;
      }
    (void)n;
  }
}

}  // namespace

extern "C" {

ibr_status ibr_set_rhs(ibr_ctx* c, const double* gh, const double* hp) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] { set_rhs_impl(c, gh, hp, hipMemcpyHostToDevice); });
}

ibr_status ibr_set_rhs_dev(ibr_ctx* c, const void* g, const void* hp) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_device_ptr(c, g, "g");
    require_device_ptr(c, hp, "h");
    set_rhs_impl(c, (const double*)g, (const double*)hp, hipMemcpyDeviceToDevice);
  });
}

ibr_status ibr_solve(ibr_ctx* c, int warm_start, ibr_info* info) {
  if (!c) return IBR_EINVAL;
  ibr_status st = IBR_OK;
  ibr_status g = guard(c, [&] {
    require_bodies(c);
    if (c->wallvel && c->nfree) throw Status(IBR_EINVAL, "moving walls and free bodies together are not supported");
    IBR_HIP(hipSetDevice(c->p.device));
    if (!warm_start || !c->have_solution) launch_fill<double>(c->Xs, c->NV, 0.0, c->stream);
    // with inertia the walls' background flow takes (rho/dt) u_b from the
    // momentum right-hand side (not from the wall faces' identity rows)
    const bool shift = c->wallvel && c->c0 != 0.0;
    if (shift)
      launch_add_background(c->dim, c->logn, c->Bs, c->h, c->L, c->dim - 1, c->wvel, -c->c0, c->wm, c->stream);
    st = c->mixed ? fgmres<float>(c, info) : fgmres<double>(c, info);
    if (shift) {
      launch_add_background(c->dim, c->logn, c->Bs, c->h, c->L, c->dim - 1, c->wvel, c->c0, c->wm, c->stream);
      sync(c);
    }
  });
  if (g != IBR_OK) return g;
  // guard() clears the message of a call that threw nothing: set it afterwards
  if (st == IBR_ENOCONV) c->err = "FGMRES did not reach rtol within max_iters";
  if (st == IBR_ENUMERIC) c->err = "NaN or Inf in the FGMRES residual";
  return st;
}

ibr_status ibr_step(ibr_ctx* c, ibr_info* info) {
  if (!c) return IBR_EINVAL;
  ibr_status st = IBR_OK;
  ibr_status g = guard(c, [&] {
    require_bodies(c);
    // every check before any state changes: a refused step leaves the context as it was
    if (c->steady) throw Status(IBR_ESTATE, "ibr_step needs rho > 0 (unsteady)");
    if (c->rotating) throw Status(IBR_EINVAL, "ibr_step translates the bodies: Omega must be zero");
    if (c->nfree) throw Status(IBR_EINVAL, "ibr_step moves bodies with prescribed velocities only: no free bodies");
    if (c->wallvel) throw Status(IBR_EINVAL, "ibr_step with moving walls is not supported (advection is nonlinear)");
    if (c->walls) {
      // bodies translate with their prescribed velocity: every marker must stay between the walls
      const int d0 = c->dim;
      for (int b = 0; b < c->nb; ++b)
        for (int a = 0; a < d0; ++a) {
          if (!((c->wm >> a) & 1)) continue;
          const int i = b * d0 + a;
          const double zc = c->wall_z[i] + c->p.dt * c->wall_uz[i];
          if (!(zc + c->wall_lo[i] > 0.0 && zc + c->wall_hi[i] < c->L))
            throw Status(IBR_EINVAL, "ibr_step: body " + std::to_string(b) + " would cross a wall");
        }
    }
    IBR_HIP(hipSetDevice(c->p.device));
    hipStream_t s = c->stream;
    const int d = c->dim;
    const int64_t len = (int64_t)d * c->C;
    if (!c->have_solution) launch_fill<double>(c->Xs, c->NV, 0.0, s);
    // explicit advection: semi-Lagrangian transport (g = (rho/dt) v_d), or the
    // centred form with AB2 (forward Euler on the first step)
    const double rho = c->p.rho;
    if (c->p.advection == IBR_ADVECT_SL) {
      launch_advect_sl(d, c->logn, c->Xs, c->Ncur, c->p.dt / c->h, 1.0 / c->p.dt, s, c->wm);
      launch_ns_rhs(c->Xs, c->Ncur, nullptr, c->Bs, len, c->c0, rho, 1.0, 0.0, s);
    } else {
      launch_advect(d, c->logn, c->Xs, c->Ncur, 0.5 / c->h, s, c->wm);
      if (c->have_prev)
        launch_ns_rhs(c->Xs, c->Ncur, c->Nprev, c->Bs, len, c->c0, rho, 1.5, -0.5, s);
      else
        launch_ns_rhs(c->Xs, c->Ncur, nullptr, c->Bs, len, c->c0, rho, 1.0, 0.0, s);
    }
    launch_fill<double>(c->Bs + len, c->C, 0.0, s);
    // move the bodies, re-bin the markers (the mobility blocks are translation invariant)
    launch_move_markers(d, c->N, c->nb, c->R, c->X, c->body_d, c->U, c->p.dt, c->L, s);
    if (c->walls)
      for (size_t i = 0; i < c->wall_z.size(); ++i) c->wall_z[i] += c->p.dt * c->wall_uz[i];
    setup_markers(c);
    build_rhs_markers(c);
    st = c->mixed ? fgmres<float>(c, info) : fgmres<double>(c, info);
    std::swap(c->Nprev, c->Ncur);
    c->have_prev = true;
  });
  if (g != IBR_OK) return g;
  if (st == IBR_ENOCONV) c->err = "FGMRES did not reach rtol within max_iters";
  if (st == IBR_ENUMERIC) c->err = "NaN or Inf in the FGMRES residual";
  return st;
}

ibr_status ibr_set_free_bodies(ibr_ctx* c, const int* free_mask, const double* F, const double* T) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    const int d = c->dim, nb = c->nb;
    const int nr = d == 3 ? 3 : 1;
    int nfree = 0;
    if (free_mask) {
      for (int b = 0; b < nb; ++b) nfree += free_mask[b] != 0;
      if (nfree && (!F || !T)) throw Status(IBR_EINVAL, "F and T are required for free bodies");
      for (int b = 0; b < nb && nfree; ++b) {
        if (!free_mask[b]) continue;
        for (int a = 0; a < d; ++a)
          if (!std::isfinite(F[b * d + a])) throw Status(IBR_EINVAL, "F must be finite");
        for (int a = 0; a < nr; ++a)
          if (!std::isfinite(T[b * nr + a])) throw Status(IBR_EINVAL, "T must be finite");
      }
    }
    IBR_HIP(hipSetDevice(c->p.device));
    hipStream_t s = c->stream;
    sync(c);
    c->clear_free();
    c->drop_graphs();
    ++c->graph_version;
    if (nfree) {
      c->free_h.assign(free_mask, free_mask + nb);
      for (int& f : c->free_h) f = f != 0;
      c->nfree = nfree;
      c->nq = (int64_t)nb * (d + nr);
      c->load_h.assign(c->nq, 0.0);
      std::vector<int64_t> yoff(nb + 1, 0);
      for (int b = 0; b < nb; ++b) {
        const int64_t rows = c->free_h[b] ? (int64_t)d * (c->off_h[b + 1] - c->off_h[b]) : 0;
        yoff[b + 1] = yoff[b] + rows * (d + nr);
        if (c->free_h[b]) {
          for (int a = 0; a < d; ++a) c->load_h[b * d + a] = F[b * d + a];
          for (int a = 0; a < nr; ++a) c->load_h[(int64_t)nb * d + b * nr + a] = T[b * nr + a];
        }
      }
      c->free_d = dev_alloc<int>(nb);
      c->yoff_d = dev_alloc<int64_t>(nb + 1);
      c->Yf = dev_alloc<double>(std::max<int64_t>(yoff[nb], 1));
      c->Nf = dev_alloc<double>((int64_t)nb * (d + nr) * (d + nr));
      IBR_HIP(hipMemcpyAsync(c->free_d, c->free_h.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
      IBR_HIP(hipMemcpyAsync(c->yoff_d, yoff.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
      launch_fill<int>(c->fail_d, nb, 0, s);
      launch_free_setup(d, nb, c->off_d, c->moff_d, c->Minv, c->R, c->X, c->L, c->free_d, c->yoff_d, c->Yf, c->Nf,
                        c->fail_d, s);
      std::vector<int> fail(nb, 0);
      IBR_HIP(hipMemcpyAsync(fail.data(), c->fail_d, nb * sizeof(int), hipMemcpyDeviceToHost, s));
      sync(c);
      for (int b = 0; b < nb; ++b)
        if (c->free_h[b] && fail[b]) {
          c->clear_free();
          c->NV = c->NF + (int64_t)d * c->N;
          build_rhs_markers(c);
          sync(c);
          throw Status(IBR_EFACTOR, "body mobility of free body " + std::to_string(b) + " is not positive definite");
        }
    }
    c->NV = c->NF + (int64_t)d * c->N + c->nq;
    c->ldv = (c->NV + 63) & ~(int64_t)63;
    // a new unknown set: no warm start across it
    launch_fill<double>(c->Xs, c->NV, 0.0, s);
    c->have_solution = false;
    build_rhs_markers(c);
    sync(c);
  });
}

ibr_status ibr_get_velocities(ibr_ctx* c, double* U, double* Omega) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (!U && !Omega) return;
    IBR_HIP(hipSetDevice(c->p.device));
    const int d = c->dim, nb = c->nb;
    const int nr = d == 3 ? 3 : 1;
    hipStream_t s = c->stream;
    std::vector<double> u((size_t)nb * d), w((size_t)nb * nr), q((size_t)c->nq);
    IBR_HIP(hipMemcpyAsync(u.data(), c->U, u.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    IBR_HIP(hipMemcpyAsync(w.data(), c->Om, w.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    if (c->nq)
      IBR_HIP(hipMemcpyAsync(q.data(), c->Xs + c->NF + (int64_t)d * c->N, q.size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    sync(c);
    for (int b = 0; b < nb; ++b) {
      const bool fr = c->nq && c->free_h[b];
      for (int a = 0; a < d; ++a)
        if (U) U[b * d + a] = fr ? q[b * d + a] : u[b * d + a];
      for (int a = 0; a < nr; ++a)
        if (Omega) Omega[b * nr + a] = fr ? q[(size_t)nb * d + b * nr + a] : w[b * nr + a];
    }
  });
}

ibr_status ibr_set_wall_velocity(ibr_ctx* c, const double* lo, const double* hi) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    if (!lo && !hi) {
      c->wallvel = false;
      c->wvel = WallVel{};
    } else {
      if (!lo || !hi) throw Status(IBR_EINVAL, "lo and hi are both required (or both NULL)");
      if (!c->walls) throw Status(IBR_EINVAL, "moving walls need walls");
      const int d = c->dim;
      for (int a = 0; a < d; ++a)
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a])) throw Status(IBR_EINVAL, "wall velocities must be finite");
      if (c->p.walls == IBR_WALLS_NOSLIP && (lo[d - 1] != 0.0 || hi[d - 1] != 0.0))
        throw Status(IBR_EINVAL, "slit channel walls move in their planes: the last components must be 0");
      if (c->p.walls == IBR_WALLS_BOX)
        for (int a = 0; a < d; ++a)
          if (lo[a] != hi[a]) throw Status(IBR_EINVAL, "the box's walls move together: lo must equal hi");
      WallVel w{};
      for (int a = 0; a < d; ++a) {
        w.lo[a] = lo[a];
        w.hi[a] = hi[a];
      }
      c->wvel = w;
      c->wallvel = true;
    }
    if (c->nb > 0) {
      IBR_HIP(hipSetDevice(c->p.device));
      build_rhs_markers(c);
      sync(c);
    }
  });
}

ibr_status ibr_reset(ibr_ctx* c) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    IBR_HIP(hipSetDevice(c->p.device));
    launch_fill<double>(c->Xs, c->NV, 0.0, c->stream);
    c->have_solution = false;
    c->have_prev = false;
    sync(c);
  });
}

ibr_status ibr_get_solution(ibr_ctx* c, double* u, double* pr, double* lambda, double* F, double* T) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] { get_solution_impl(c, u, pr, lambda, F, T, hipMemcpyDeviceToHost); });
}

ibr_status ibr_get_solution_dev(ibr_ctx* c, void* u, void* pr, void* lambda, void* F, void* T) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_device_ptr(c, u, "u");
    require_device_ptr(c, pr, "p");
    require_device_ptr(c, lambda, "lambda");
    require_device_ptr(c, F, "F");
    require_device_ptr(c, T, "T");
    get_solution_impl(c, (double*)u, (double*)pr, (double*)lambda, (double*)F, (double*)T,
                      hipMemcpyDeviceToDevice);
  });
}

ibr_status ibr_get_markers(ibr_ctx* c, double* R, double* centres) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    IBR_HIP(hipSetDevice(c->p.device));
    if (R) IBR_HIP(hipMemcpyAsync(R, c->R, (size_t)c->N * c->dim * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (centres)
      IBR_HIP(hipMemcpyAsync(centres, c->X, (size_t)c->nb * c->dim * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    sync(c);
  });
}

ibr_status ibr_apply_operator(ibr_ctx* c, const double* x, double* yh) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (!x || !yh) throw Status(IBR_EINVAL, "x and y are required");
    IBR_HIP(hipSetDevice(c->p.device));
    IBR_HIP(hipMemcpyAsync(c->T1, x, (size_t)c->NV * sizeof(double), hipMemcpyHostToDevice, c->stream));
    apply_K<double>(c, c->T1, c->T2);
    IBR_HIP(hipMemcpyAsync(yh, c->T2, (size_t)c->NV * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

ibr_status ibr_spread(ibr_ctx* c, const double* lambda, double* f) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (!lambda || !f) throw Status(IBR_EINVAL, "lambda and f are required");
    IBR_HIP(hipSetDevice(c->p.device));
    const int d = c->dim;
    hipStream_t s = c->stream;
    IBR_HIP(hipMemcpyAsync(c->lamd, lambda, (size_t)c->N * d * sizeof(double), hipMemcpyHostToDevice, s));
    launch_fill<double>(c->T2, (int64_t)d * c->C, 0.0, s);
    launch_spread<double, double>(d, c->logn, c->tile_log, c->act_cap, c->active, c->nactive_d, c->toff, c->perm,
                                  c->taps, c->lamd, c->T2, std::pow(c->h, -d), s);
    IBR_HIP(hipMemcpyAsync(f, c->T2, (size_t)d * c->C * sizeof(double), hipMemcpyDeviceToHost, s));
    sync(c);
  });
}

ibr_status ibr_interp(ibr_ctx* c, const double* u, double* V) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (!u || !V) throw Status(IBR_EINVAL, "u and V are required");
    IBR_HIP(hipSetDevice(c->p.device));
    const int d = c->dim;
    hipStream_t s = c->stream;
    IBR_HIP(hipMemcpyAsync(c->T1, u, (size_t)d * c->C * sizeof(double), hipMemcpyHostToDevice, s));
    launch_interp<double>(d, c->logn, c->N, c->taps, c->T1, 1.0, nullptr, 0.0, c->dU, s);
    IBR_HIP(hipMemcpyAsync(V, c->dU, (size_t)c->N * d * sizeof(double), hipMemcpyDeviceToHost, s));
    sync(c);
  });
}

ibr_status ibr_vcycle(ibr_ctx* c, double c0, double c1, int nf, const double* b, double* x) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    if (!b || !x) throw Status(IBR_EINVAL, "b and x are required");
    if (nf < 1 || nf > c->dim) throw Status(IBR_EINVAL, "nfields must be in [1, dim]");
    if (c->walls && nf != 1 && nf != c->dim)
      throw Status(IBR_EINVAL, "with walls nfields is dim (velocity) or 1 (pressure)");
    // with walls: the velocity cycle (field a = component a) or the Neumann pressure cycle
    const int mode = c->walls ? (nf == 1 ? 2 : 1) : 0;
    const bool singular = c0 == 0.0 && mode != 1;
    if (!(c0 >= 0) || !std::isfinite(c1) || c1 == 0.0) throw Status(IBR_EINVAL, "need c0 >= 0 and c1 != 0");
    IBR_HIP(hipSetDevice(c->p.device));
    hipStream_t s = c->stream;
    const int64_t len = (int64_t)nf * c->C;
    // staging in the advection-history buffers (dim C doubles each)
    double* bd = c->Nprev;
    double* xd = c->Ncur;
    IBR_HIP(hipMemcpyAsync(bd, b, (size_t)len * sizeof(double), hipMemcpyHostToDevice, s));
    // the hierarchy works in split storage: convert in and out
    if (c->mixed) {
      float* bf = (float*)c->Qi;
      float* xf = (float*)c->Zi;
      launch_to_split<double, float>(c->dim, c->logn, bd, bf, nf, s);
      c->mg32.vcycle(nf, bf, xf, c0, c1, c->p.mg_pre, c->p.mg_post, c->p.mg_coarse, s, mode);
      if (singular) {
        launch_field_means<float>(xf, nf, c->C, c->mpart, c->mean_blocks, c->vmean, s);
        launch_sub_field_mean<float>(xf, nf, c->C, c->vmean, s);
      }
      launch_from_split<float, double>(c->dim, c->logn, xf, xd, nf, s);
    } else {
      double* bs = (double*)c->Qi;
      double* xs = (double*)c->Zi;
      launch_to_split<double, double>(c->dim, c->logn, bd, bs, nf, s);
      c->mg64.vcycle(nf, bs, xs, c0, c1, c->p.mg_pre, c->p.mg_post, c->p.mg_coarse, s, mode);
      if (singular) {
        launch_field_means<double>(xs, nf, c->C, c->mpart, c->mean_blocks, c->vmean, s);
        launch_sub_field_mean<double>(xs, nf, c->C, c->vmean, s);
      }
      launch_from_split<double, double>(c->dim, c->logn, xs, xd, nf, s);
    }
    IBR_HIP(hipMemcpyAsync(x, xd, (size_t)len * sizeof(double), hipMemcpyDeviceToHost, s));
    c->have_prev = false;
    sync(c);
  });
}

ibr_status ibr_precondition(ibr_ctx* c, const double* r, double* z) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (!r || !z) throw Status(IBR_EINVAL, "r and z are required");
    IBR_HIP(hipSetDevice(c->p.device));
    hipStream_t s = c->stream;
    IBR_HIP(hipMemcpyAsync(c->T1, r, (size_t)c->NV * sizeof(double), hipMemcpyHostToDevice, s));
    if (c->mixed) {
      float* zf = (float*)c->Zb;
      precondition<float>(c, c->T1, zf);
      launch_copy<float, double>(zf, c->T2, c->NV, s);
    } else {
      precondition<double>(c, c->T1, c->T2);
    }
    IBR_HIP(hipMemcpyAsync(z, c->T2, (size_t)c->NV * sizeof(double), hipMemcpyDeviceToHost, s));
    sync(c);
  });
}

ibr_status ibr_mobility_block(ibr_ctx* c, int body, double* M, double* shift) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (body < 0 || body >= c->nb) throw Status(IBR_EINVAL, "body out of range");
    IBR_HIP(hipSetDevice(c->p.device));
    const int64_t n = (int64_t)c->dim * (c->off_h[body + 1] - c->off_h[body]);
    const int64_t ld = (n + 15) & ~(int64_t)15;
    if (M)
      IBR_HIP(hipMemcpy2DAsync(M, n * sizeof(double), c->Mb + c->moff_h[body], ld * sizeof(double),
                               n * sizeof(double), n, hipMemcpyDeviceToHost, c->stream));
    if (shift) *shift = c->shift_h[body];
    sync(c);
  });
}

ibr_status ibr_mobility_inverse(ibr_ctx* c, int body, double* Minv) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    require_bodies(c);
    if (body < 0 || body >= c->nb || !Minv) throw Status(IBR_EINVAL, "body out of range or Minv NULL");
    IBR_HIP(hipSetDevice(c->p.device));
    const int64_t n = (int64_t)c->dim * (c->off_h[body + 1] - c->off_h[body]);
    const int64_t ld = (n + 15) & ~(int64_t)15;
    IBR_HIP(hipMemcpy2DAsync(Minv, n * sizeof(double), c->Minv + c->moff_h[body], ld * sizeof(double),
                             n * sizeof(double), n, hipMemcpyDeviceToHost, c->stream));
    sync(c);
  });
}

ibr_status ibr_advect(ibr_ctx* c, const double* u, double* N) {
  if (!c) return IBR_EINVAL;
  return guard(c, [&] {
    if (!u || !N) throw Status(IBR_EINVAL, "u and N are required");
    IBR_HIP(hipSetDevice(c->p.device));
    const int d = c->dim;
    hipStream_t s = c->stream;
    if (c->p.advection == IBR_ADVECT_SL && c->steady)
      throw Status(IBR_EINVAL, "semi-Lagrangian advection needs dt > 0 (unsteady)");
    IBR_HIP(hipMemcpyAsync(c->Nprev, u, (size_t)d * c->C * sizeof(double), hipMemcpyHostToDevice, s));
    if (c->p.advection == IBR_ADVECT_SL)
      launch_advect_sl(d, c->logn, c->Nprev, c->Ncur, c->p.dt / c->h, 1.0 / c->p.dt, s, c->wm);
    else
      launch_advect(d, c->logn, c->Nprev, c->Ncur, 0.5 / c->h, s, c->wm);
    IBR_HIP(hipMemcpyAsync(N, c->Ncur, (size_t)d * c->C * sizeof(double), hipMemcpyDeviceToHost, s));
    c->have_prev = false;
    sync(c);
  });
}

}  // extern "C"
