// Per-body approximate mobility blocks (Sec. 4, eq. M_tilde_ij) and their
// dense solve (Sec. 5.3).  Each body's block is assembled from f(r), g(r),
// factored by Cholesky (shifted by s f(0) I when it is not positive definite)
// and turned into an explicit inverse, so that every preconditioner
// application is one batched matrix-vector product.
//
// Block p is row-major dN_p x dN_p at M + moff[p].
#include <algorithm>

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

// Fitted f(r), g(r) (Sec. 4.2 fitting procedure, Appendix A forms; x = r/h).
// Steady: ft = 8 pi eta r (f + shift), gt = 8 pi eta r g.  Finite beta:
// f = -(beta/(eta h)) ft_b / (4 pi x^3), g = (beta/(eta h)) 3 gt_b / (4 pi x^3),
// and f(0) = phi0 beta / (eta h), g(0) = 0.
__device__ void mob_fg_fit(double r, const MobParams& p, double& f, double& g) {
  const double x = r / p.h;
  if (p.fit == 3) {
    // 2D steady: f = f(0) - f~ / (4 pi eta), g = g~ / (4 pi eta)
    if (x < 1e-3) {
      f = p.self0 + p.mean_mode;
      g = 0.0;
      return;
    }
    const double* c = p.f2s;
    const double c4 = 1.0 / (4.0 * kPi * p.eta);
    const double x2 = x * x, x3 = x2 * x, lx = log(x);
    const double ft = (c[0] * x2 + c[1] * x3 + c[2] * x3 * lx) / (1.0 + c[3] * x + c[4] * x2 + c[2] * x3);
    const double gt = (c[5] * x2 + c[6] * x3) / (1.0 + c[7] * x + c[8] * x2 + c[6] * x3);
    f = p.self0 - c4 * ft + p.mean_mode;
    g = c4 * gt;
    return;
  }
  if (p.fit == 4) {
    // 2D finite beta: f = -(beta / (2 pi eta x^2)) f~, g = (beta / (pi eta x^2)) g~
    const double be = p.beta / p.eta;
    if (x < 1e-3) {
      f = p.phi0 * be + p.mean_mode;
      g = 0.0;
      return;
    }
    const double x2 = x * x, x3 = x2 * x, x4 = x2 * x2, lx = log(x), sb = sqrt(p.beta);
    double ft = 0.0, gt = 0.0;
    for (int q = 0; q < 2; ++q) {
      const double w = q == 0 ? 1.0 - p.tw : p.tw;
      if (w == 0.0) continue;
      const double* c = p.f2r[q];
      const double ftq = x3 * lx / (p.beta * (c[0] + 2.0 * x)) * exp(-c[4] * x / sb) +
                         (c[1] * x2 + c[2] * x3 + c[3] * x4) / (1.0 + c[5] * x2 + c[6] * x3 + c[3] * x4);
      const double gtq = x3 / (p.beta * (c[7] + 4.0 * x)) * exp(-c[11] * x / sb) +
                         x3 / (exp(-c[12] * x) * (c[8] + c[9] * x + c[10] * x2) + x3);
      ft += w * ftq;
      gt += w * gtq;
    }
    f = -be * ft / (2.0 * kPi * x2) + p.mean_mode;
    g = be * gt / (kPi * x2);
    return;
  }
  if (p.fit == 1) {
    const double* b = p.fs;
    const double c = 1.0 / (8.0 * kPi * p.eta * p.h);
    if (x < 0.8) {
      // ft / (8 pi eta r) = 1 / (8 pi eta h (3a/4h + b0 x^2)): finite at x = 0
      f = c / (0.75 * p.ah + b[0] * x * x);
    } else {
      const double x2 = x * x, x4 = x2 * x2;
      const double ft = b[1] * x * exp(-b[2] * x) + (b[3] * x2 + x4) / (1.0 + b[4] * x2 + x4);
      f = c * ft / x;
    }
    f -= p.periodic_shift;
    f += p.mean_mode;
    const double x2 = x * x;
    g = c * x2 / (b[5] + b[6] * x2 + x2 * x);
    return;
  }
  const double pre = p.beta / (p.eta * p.h);
  if (x < 1e-3) {
    f = p.phi0 * pre + p.mean_mode;
    g = 0.0;
    return;
  }
  const double x2 = x * x, x3 = x2 * x, x4 = x2 * x2, x5 = x4 * x, x7 = x5 * x2;
  const double bq = p.beta, ph = p.phi0, sb = sqrt(bq);
  double ft = 0.0, gt = 0.0;
  for (int q = 0; q < 2; ++q) {
    const double w = q == 0 ? 1.0 - p.tw : p.tw;
    if (w == 0.0) continue;
    // the forms of row q at beta itself
    const double* a = p.fa[q];
    const double* b = p.fb[q];
    const double ftq = ph * (-4.0 * kPi * x3 + a[4] * (x5 - x7 * exp(-a[3] * x / sb) / (2.0 * bq))) /
                           (1.0 + a[0] * x + a[1] * x2 + a[2] * x3 + a[4] * ph * x5) +
                       (a[5] * x4 * exp(-a[6] * x) + a[7] * x4) / (1.0 + a[8] * x3 + a[9] * x5);
    const double gtq = ph * b[5] * (x5 + x7 * exp(-b[0] * x / sb) / (6.0 * bq)) /
                       (1.0 + b[1] * x + b[2] * x2 + b[3] * x3 + b[4] * x4 + b[5] * ph * x5);
    ft += w * ftq;
    gt += w * gtq;
  }
  f = -pre * ft / (4.0 * kPi * x3) + p.mean_mode;
  g = pre * 3.0 * gt / (4.0 * kPi * x3);
}

// f(r), g(r) of the approximate mobility (same forms as the documented reading
// of Sec. 4 / Appendices A and B), or the fitted forms.
__device__ void mob_fg(double r, const MobParams& p, double& f, double& g) {
  if (p.fit) {
    mob_fg_fit(r, p, f, g);
    return;
  }
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

// Batched blocked right-looking Cholesky of M_p + shift_p f0 I over all
// bodies with 64-column panels; per panel three launches cover every body:
//   diag:  one workgroup per body factors the 64 x 64 diagonal block in LDS
//          (16 x 16 tiles: register factor of the diagonal tile, row tiles by
//          substitution, trailing tiles on MFMA) and inverts it (the
//          diagonal block of X = L^-1);
//   trsm:  one workgroup per 64-row block below: L_Ip = A_Ip (L_pp^-1)^T on
//          MFMA with both operands in LDS;
//   syrk:  one workgroup per pair of 64-row blocks I >= J below: A_IJ -=
//          L_Ip L_Jp^T on MFMA, each wavefront a 32 x 32 quadrant (2 x 2
//          tiles, 16 k-steps per tile).
// A pivot <= pivot_tol f0 marks the body failed (it is factored again with a
// larger shift).  The inverse then needs only the off-diagonal blocks of X
// and Minv = X^T X, both as 64 x 64 block products on MFMA.
constexpr int kBlk = 64;   // block edge
constexpr int kSld = 66;   // LDS row stride in doubles (MFMA operand reads 2-way at most per bank)

// L = lower(M) + shift on the diagonal, identity on the padding rows.
__global__ void __launch_bounds__(64) k_chol_init(const int* __restrict__ off, int dim,
                                                  const int64_t* __restrict__ moff, const double* __restrict__ M,
                                                  double* __restrict__ Lf, const int* __restrict__ active,
                                                  const double* __restrict__ shift, double f0, int* __restrict__ fail) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int i = blockIdx.x;
  if (i >= ld) return;
  if (i == 0 && threadIdx.x == 0) fail[b] = 0;
  const double* A = M + moff[b];
  double* L = Lf + moff[b];
  const double sh = shift[b] * f0;
  for (int j = threadIdx.x; j < ld; j += blockDim.x) {
    double v = 0.0;
    if (j <= i) {
      if (i < n) v = A[(int64_t)i * ld + j] + (i == j ? sh : 0.0);
      else if (i == j) v = 1.0;
    }
    L[(int64_t)i * ld + j] = v;
  }
}

// A kBlk x kBlk block of the row-major matrix G (leading dimension ld) from
// row r0, column c0 into LDS S (stride kSld); entries outside rows < rmax,
// columns < cmax (and, with lower, above the diagonal) are zero.
// 256 threads: each issues its 16 global loads before its LDS stores, so
// they are in flight together.  block_fetch / block_put split the two halves
// so that the loads of the next block can overlap the products on this one.
constexpr int kPer = kBlk * kBlk / 256;
__device__ inline void block_fetch(double v[kPer], const double* __restrict__ G, int ld, int r0, int c0, int rmax,
                                   int cmax, bool lower = false) {
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + 256 * u;
    const int i = idx >> 6, j = idx & 63;
    v[u] = 0.0;
    if (r0 + i < rmax && c0 + j < cmax && (!lower || c0 + j <= r0 + i)) v[u] = G[(int64_t)(r0 + i) * ld + c0 + j];
  }
}
__device__ inline void block_put(double* S, const double v[kPer]) {
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int idx = threadIdx.x + 256 * u;
    S[(idx >> 6) * kSld + (idx & 63)] = v[u];
  }
}
__device__ inline void lds_load_block(double* S, const double* __restrict__ G, int ld, int r0, int c0, int rmax,
                                      int cmax, bool lower = false) {
  double v[kPer];
  block_fetch(v, G, ld, r0, c0, rmax, cmax, lower);
  block_put(S, v);
}

// Workgroup -> (body, item) so that all workgroups of one body run on one
// XCD (the hardware hands consecutive workgroups to the 8 XCDs in turn): a
// body's panel and blocks are then re-read from that XCD's L2.  Grid:
// 8 * ceil(nb / 8) * nitems workgroups in x; false for the padding ones.
__device__ inline bool body_item(int nb, int nitems, int& body, int& item) {
  const int id = blockIdx.x;
  const int xcd = id % kXcds, k = id / kXcds;
  body = xcd + kXcds * (k / nitems);
  item = k % nitems;
  return body < nb;
}

// acc += A B^T on the 16 x 16 tile (ti, tj): A[i][k] = A[i * kSld + k],
// B^T given as Bt[j][k] = Bt[j * kSld + k]; K a multiple of 4.
__device__ inline dvec4 mma_abt(dvec4 acc, const double* A, const double* Bt, int ti, int tj, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  const double* a = A + (ti * 16 + r) * kSld + kq;
  const double* bt = Bt + (tj * 16 + r) * kSld + kq;
  for (int k0 = 0; k0 < K; k0 += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k0], bt[k0], acc, 0, 0, 0);
  return acc;
}
// acc += A B on the tile (ti, tj): A[i][k] = A[i * kSld + k], B[k][j] = B[k * kSld + j].
__device__ inline dvec4 mma_ab(dvec4 acc, const double* A, const double* B, int ti, int tj, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  const double* a = A + (ti * 16 + r) * kSld + kq;
  const double* bb = B + kq * kSld + tj * 16 + r;
  for (int k0 = 0; k0 < K; k0 += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k0], bb[k0 * kSld], acc, 0, 0, 0);
  return acc;
}
// acc += A^T B on the tile (ti, tj): A[k][i] = A[k * kSld + i], B[k][j] = B[k * kSld + j].
__device__ inline dvec4 mma_atb(dvec4 acc, const double* A, const double* B, int ti, int tj, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  const double* a = A + kq * kSld + ti * 16 + r;
  const double* bb = B + kq * kSld + tj * 16 + r;
  for (int k0 = 0; k0 < K; k0 += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k0 * kSld], bb[k0 * kSld], acc, 0, 0, 0);
  return acc;
}
// The same products on a 2 x 2 quadrant of tiles (ti0, ti0+1) x (tj0, tj0+1):
// per k-step two A and two B operands feed four independent accumulators.
__device__ inline void mma_abt_2x2(dvec4 acc[2][2], const double* A, const double* Bt, int ti0, int tj0, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  const double* a0 = A + (ti0 * 16 + r) * kSld + kq;
  const double* a1 = a0 + 16 * kSld;
  const double* b0 = Bt + (tj0 * 16 + r) * kSld + kq;
  const double* b1 = b0 + 16 * kSld;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double x0 = a0[k0], x1 = a1[k0], y0 = b0[k0], y1 = b1[k0];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
  }
}
__device__ inline void mma_ab_2x2(dvec4 acc[2][2], const double* A, const double* B, int ti0, int tj0, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  const double* a0 = A + (ti0 * 16 + r) * kSld + kq;
  const double* a1 = a0 + 16 * kSld;
  const double* b0 = B + kq * kSld + tj0 * 16 + r;
  const double* b1 = b0 + 16;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double x0 = a0[k0], x1 = a1[k0], y0 = b0[k0 * kSld], y1 = b1[k0 * kSld];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
  }
}
__device__ inline void mma_atb_2x2(dvec4 acc[2][2], const double* A, const double* B, int ti0, int tj0, int K) {
  const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
  const double* a0 = A + kq * kSld + ti0 * 16 + r;
  const double* a1 = a0 + 16;
  const double* b0 = B + kq * kSld + tj0 * 16 + r;
  const double* b1 = b0 + 16;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double x0 = a0[k0 * kSld], x1 = a1[k0 * kSld], y0 = b0[k0 * kSld], y1 = b1[k0 * kSld];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
  }
}

// Tile (ti, tj) of a 16 x 16 accumulator to / from LDS (stride kSld).
__device__ inline void tile_store(double* S, int ti, int tj, dvec4 acc) {
  const int lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) S[(ti * 16 + 4 * q + rq) * kSld + tj * 16 + c] = acc[q];
}
__device__ inline dvec4 tile_load(const double* S, int ti, int tj) {
  const int lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
  dvec4 acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = S[(ti * 16 + 4 * q + rq) * kSld + tj * 16 + c];
  return acc;
}

// Diagonal block of panel c0 (width W = min(64, ld - c0)): factor and invert.
// 256 threads.  LDS: D (the block, then L_pp; its strictly upper tiles are
// the wavefronts' scratch tiles of the inversion), X (the inverse).
__global__ void __launch_bounds__(256) k_chol_diag(const int* __restrict__ off, int dim,
                                                   const int64_t* __restrict__ moff, double* __restrict__ Lf,
                                                   double* __restrict__ Xf, const int* __restrict__ active, int c0,
                                                   double f0, double pivot_tol, int* __restrict__ fail) {
  __shared__ double D[kBlk * kSld];
  __shared__ double X[kBlk * kSld];
  __shared__ double rdiag[kBlk];  // 1 / L_jj: the substitutions multiply instead of dividing
  __shared__ double colbuf[2][16];  // the pivot column of the register factor, double-buffered
  __shared__ int bad_s;
  const int b = blockIdx.x;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  if (c0 >= ld) return;
  const int W = min(kBlk, ld - c0);
  const int nt = W / 16;
  double* L = Lf + moff[b];
  double* Xg = Xf + moff[b];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15;
  if (threadIdx.x == 0) bad_s = 0;
  lds_load_block(D, L, ld, c0, c0, c0 + W, c0 + W, true);
  for (int idx = threadIdx.x; idx < kBlk * kSld; idx += blockDim.x) X[idx] = 0.0;
  __syncthreads();
  for (int q = 0; q < nt; ++q) {
    const int q0 = 16 * q;
    // diagonal tile in registers of wavefront 0: lane r (mod 16) holds row r.
    // Step jj broadcasts column jj through LDS (one write, then independent
    // reads of all its entries; lane-to-lane shuffles here were serialised,
    // about 800 cycles per step)
    if (wv == 0) {
      double row[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) row[c] = c <= r16 ? D[(q0 + r16) * kSld + q0 + c] : 0.0;
      bool bad = false;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        double* cb = colbuf[jj & 1];
        if (lane < 16) cb[lane] = row[jj];
        wave_sync();
        double cv[16];
#pragma unroll
        for (int c = jj; c < 16; ++c) cv[c] = cb[c];
        const double d = cv[jj];
        bad = bad || !(d > pivot_tol * f0);
        const double sd = sqrt(d > 0.0 ? d : 1.0);
        const double rs = 1.0 / sd;
        if (lane == jj) rdiag[q0 + jj] = rs;
        if (r16 == jj) row[jj] = sd;
        else if (r16 > jj) row[jj] = row[jj] * rs;
#pragma unroll
        for (int c = jj + 1; c < 16; ++c) {
          const double lc = cv[c] * rs;
          if (r16 >= c) row[c] -= row[jj] * lc;
        }
      }
      if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) D[(q0 + r16) * kSld + q0 + c] = c <= r16 ? row[c] : 0.0;
      }
      if (lane == 0 && bad) bad_s = 1;
    }
    __syncthreads();
    // row tiles below: x L_qq^T = a, one row per lane (16 lanes of a wavefront per tile)
    for (int rt = q + 1 + wv; rt < nt; rt += 4) {
      if (lane < 16) {
        double* Lr = D + (16 * rt + lane) * kSld + q0;
        double x[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) x[c] = Lr[c];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          double t = x[c];
#pragma unroll
          for (int k = 0; k < c; ++k) t -= x[k] * D[(q0 + c) * kSld + q0 + k];
          x[c] = t * rdiag[q0 + c];
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) Lr[c] = x[c];
      }
    }
    __syncthreads();
    // trailing tiles (rt, st), q < st <= rt < nt: D -= L_rt,q L_st,q^T (K = 16 at column q0)
    int cnt = 0;
    for (int rt = q + 1; rt < nt; ++rt)
      for (int st = q + 1; st <= rt; ++st, ++cnt) {
        if (cnt % 4 != wv) continue;
        dvec4 acc = tile_load(D, rt, st);
        dvec4 m = {0.0, 0.0, 0.0, 0.0};
        m = mma_abt(m, D + q0, D + q0, rt, st, 16);
        acc -= m;
        tile_store(D, rt, st, acc);
      }
    __syncthreads();
  }
  // inverse of the lower-triangular L_pp: diagonal tiles (lane c < 16 solves column c)
  for (int q = wv; q < nt; q += 4) {
    if (lane < 16) {
      const int q0 = 16 * q, c = lane;
      double col[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double v = i == c ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) v -= D[(q0 + i) * kSld + q0 + k] * col[k];
        col[i] = i < c ? 0.0 : v * rdiag[q0 + i];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) X[(q0 + i) * kSld + q0 + c] = col[i];
    }
  }
  __syncthreads();
  // X_rs = -X_rr sum_{k=s}^{r-1} L_rk X_ks, row tile by row tile.  Scratch
  // tile of wavefront w: the strictly upper tile (0, w+1) of D, or (1, 3).
  const int sti = wv == 3 ? 1 : 0, stj = wv == 3 ? 3 : wv + 1;
  double* scratch = D + 16 * sti * kSld + 16 * stj;
  for (int rt = 1; rt < nt; ++rt) {
    for (int st = wv; st < rt; st += 4) {
      dvec4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k = st; k < rt; ++k) {
        // L_rk X_ks: A = D tile (rt, k), B = X tile (k, st), K = 16
        acc = mma_ab(acc, D + 16 * k, X + 16 * k * kSld, rt, st, 16);
      }
      tile_store(scratch, 0, 0, acc);
      dvec4 res = {0.0, 0.0, 0.0, 0.0};
      res = mma_ab(res, X + 16 * rt, scratch, rt, 0, 16);
      tile_store(X, rt, st, -res);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < W * W; idx += blockDim.x) {
    const int i = idx / W, j = idx - (idx / W) * W;
    if (j <= i) {
      L[(int64_t)(c0 + i) * ld + c0 + j] = D[i * kSld + j];
      Xg[(int64_t)(c0 + i) * ld + c0 + j] = X[i * kSld + j];
    } else {
      Xg[(int64_t)(c0 + i) * ld + c0 + j] = 0.0;
    }
  }
  if (threadIdx.x == 0 && bad_s) fail[b] = 1;
}

// Panel rows below the diagonal block: L_Ip = A_Ip (L_pp^-1)^T, one workgroup
// per 64-row block I (rows c0 + W + 64 blockIdx.x ..), each wavefront 16 rows.
__global__ void __launch_bounds__(256) k_chol_trsm(const int* __restrict__ off, int dim,
                                                   const int64_t* __restrict__ moff, double* __restrict__ Lf,
                                                   const double* __restrict__ Xf, const int* __restrict__ active,
                                                   int c0, int nb, int nitems) {
  __shared__ double A[kBlk * kSld];
  __shared__ double Xs[kBlk * kSld];
  int b, item;
  if (!body_item(nb, nitems, b, item)) return;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  if (c0 >= ld) return;
  const int W = min(kBlk, ld - c0);
  const int r0 = c0 + W + kBlk * item;
  if (r0 >= ld) return;
  double* L = Lf + moff[b];
  const double* Xg = Xf + moff[b];
  lds_load_block(A, L, ld, r0, c0, ld, c0 + W);
  lds_load_block(Xs, Xg, ld, c0, c0, c0 + W, c0 + W, true);
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
  // wavefront w: the 2 x 2 quadrant (rows 32 (w >> 1), columns 32 (w & 1)) of the 64 x W product
  const int qi = wv >> 1, qj = wv & 1;
  if (32 * qj >= W) return;
  dvec4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) acc[a][e] = dvec4{0.0, 0.0, 0.0, 0.0};
  mma_abt_2x2(acc, A, Xs, 2 * qi, 2 * qj, W);
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) {
      const int ti = 2 * qi + a, tj = 2 * qj + e;
      if (r0 + 16 * ti >= ld || 16 * tj >= W) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) L[(int64_t)(r0 + 16 * ti + 4 * q + rq) * ld + c0 + 16 * tj + c] = acc[a][e][q];
    }
}

// Unrank t -> (I, J), 0 <= J <= I, in row-major lower-triangular order.
__device__ inline void unrank_lower(int t, int& I, int& J) {
  I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  J = t - I * (I + 1) / 2;
}

// Trailing update: A_IJ -= L_Ip L_Jp^T for 64-row blocks I >= J below the
// panel; each wavefront a 32 x 32 quadrant, the lower triangle only on I == J.
__global__ void __launch_bounds__(256) k_chol_syrk(const int* __restrict__ off, int dim,
                                                   const int64_t* __restrict__ moff, double* __restrict__ Lf,
                                                   const int* __restrict__ active, int c0, int nb, int nitems) {
  __shared__ double Ai[kBlk * kSld];
  __shared__ double Aj[kBlk * kSld];
  int b, item;
  if (!body_item(nb, nitems, b, item)) return;
  if (!active[b]) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  if (c0 >= ld) return;
  const int W = min(kBlk, ld - c0);
  const int base = c0 + W;
  const int nblk = (ld - base + kBlk - 1) / kBlk;
  if (item >= nblk * (nblk + 1) / 2) return;
  int I, J;
  unrank_lower(item, I, J);
  const int ri = base + kBlk * I, rj = base + kBlk * J;
  double* L = Lf + moff[b];
  lds_load_block(Ai, L, ld, ri, c0, ld, c0 + W);
  if (I != J) lds_load_block(Aj, L, ld, rj, c0, ld, c0 + W);
  __syncthreads();
  const double* Bj = I != J ? Aj : Ai;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
  const int qi = wv >> 1, qj = wv & 1;  // quadrant
  if (I == J && qj > qi) return;        // strictly upper quadrant of a diagonal block
  dvec4 m[2][2];
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) m[a][e] = dvec4{0.0, 0.0, 0.0, 0.0};
  mma_abt_2x2(m, Ai, Bj, 2 * qi, 2 * qj, W);
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) {
      const int ti = 2 * qi + a, tj = 2 * qj + e;
      if (I == J && tj > ti) continue;
      const int row0 = ri + 16 * ti, col0 = rj + 16 * tj;
      if (row0 >= ld || col0 >= ld) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + 4 * q + rq, col = col0 + c;
        if (I != J || ti != tj || col <= row) L[(int64_t)row * ld + col] -= m[a][e][q];
      }
    }
}

// X = L^-1 below the diagonal blocks (those were inverted by k_chol_diag):
// one workgroup per 64-column block J and body walks the row blocks
//   X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ,   I = J+1, J+2, ...
// as a chain of steps (each product L_IK X_KJ, then the product with X_II),
// each wavefront a 32 x 32 quadrant of the 64 x 64 products.  The operands
// of the next step are loaded into registers while this step's products run
// (the X_KJ a step needs was written by an earlier step, before a barrier).
__global__ void __launch_bounds__(256) k_tri_inv(const int* __restrict__ off, int dim,
                                                 const int64_t* __restrict__ moff, const double* __restrict__ Lf,
                                                 double* __restrict__ Xf, int nb, int nitems) {
  __shared__ double A[kBlk * kSld];
  __shared__ double B[kBlk * kSld];
  int b, J;
  if (!body_item(nb, nitems, b, J)) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int nblk = (ld + kBlk - 1) / kBlk;
  if (J + 1 >= nblk) return;
  const double* L = Lf + moff[b];
  double* X = Xf + moff[b];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
  const int qi = wv >> 1, qj = wv & 1;
  const int cj = kBlk * J;
  // step (I, K): K < I is the product L_IK X_KJ, K == I the product with X_II
  double va[kPer], vb[kPer];
  auto fetch = [&](int I, int K) {
    if (K < I) {
      block_fetch(va, L, ld, kBlk * I, kBlk * K, ld, ld);
      block_fetch(vb, X, ld, kBlk * K, cj, ld, ld);
    } else {
      block_fetch(va, X, ld, kBlk * I, kBlk * I, ld, ld, true);
    }
  };
  int I = J + 1, K = J;
  fetch(I, K);
  block_put(A, va);
  block_put(B, vb);
  __syncthreads();
  dvec4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) acc[a][e] = dvec4{0.0, 0.0, 0.0, 0.0};
  while (true) {
    int In = I, Kn = K + 1;
    if (K == I) {
      In = I + 1;
      Kn = J;
    }
    const bool next = In < nblk;
    if (next) fetch(In, Kn);
    if (K < I) {
      mma_ab_2x2(acc, A, B, 2 * qi, 2 * qj, kBlk);
    } else {
      // the sum into LDS B (its last operand was read before the previous barrier), times X_II
      for (int a = 0; a < 2; ++a)
        for (int e = 0; e < 2; ++e) tile_store(B, 2 * qi + a, 2 * qj + e, acc[a][e]);
      __syncthreads();
      dvec4 res[2][2];
      for (int a = 0; a < 2; ++a)
        for (int e = 0; e < 2; ++e) res[a][e] = dvec4{0.0, 0.0, 0.0, 0.0};
      mma_ab_2x2(res, A, B, 2 * qi, 2 * qj, kBlk);
      const int ri = kBlk * I;
      for (int a = 0; a < 2; ++a)
        for (int e = 0; e < 2; ++e) {
          acc[a][e] = dvec4{0.0, 0.0, 0.0, 0.0};
          const int row0 = ri + 16 * (2 * qi + a), col0 = cj + 16 * (2 * qj + e);
          if (row0 >= ld || col0 >= ld) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) X[(int64_t)(row0 + 4 * q + rq) * ld + col0 + c] = -res[a][e][q];
        }
    }
    if (!next) break;
    // every wavefront has read this step's LDS operands (and the X_IJ just
    // stored is visible to the loads of later steps)
    __syncthreads();
    block_put(A, va);
    if (Kn < In) block_put(B, vb);
    __syncthreads();
    I = In;
    K = Kn;
  }
}

// Minv = X^T X for X = L^-1 lower triangular: one workgroup per 64 x 64 block
// (I >= J), sum over K >= I of X_KI^T X_KJ, mirrored into the upper triangle.
// (Loading the next K's blocks during the products, as k_tri_inv does, took
// 254 registers and ran 2.2 times slower here: the plain loop stays.)
__global__ void __launch_bounds__(256) k_xtx(const int* __restrict__ off, int dim, const int64_t* __restrict__ moff,
                                             const double* __restrict__ Xf, double* __restrict__ Minv, int nb,
                                             int nitems) {
  __shared__ double A[kBlk * kSld];
  __shared__ double B[kBlk * kSld];
  int b, item;
  if (!body_item(nb, nitems, b, item)) return;
  const int n = dim * (off[b + 1] - off[b]);
  const int ld = pad16(n);
  const int nblk = (ld + kBlk - 1) / kBlk;
  if (item >= nblk * (nblk + 1) / 2) return;
  int I, J;
  unrank_lower(item, I, J);
  const double* X = Xf + moff[b];
  double* Mb = Minv + moff[b];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
  const int qi = wv >> 1, qj = wv & 1;
  const int ri = kBlk * I, rj = kBlk * J;
  dvec4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) acc[a][e] = dvec4{0.0, 0.0, 0.0, 0.0};
  for (int K = I; K < nblk; ++K) {
    const int rk = kBlk * K;
    __syncthreads();
    lds_load_block(A, X, ld, rk, ri, ld, ld);
    lds_load_block(B, X, ld, rk, rj, ld, ld);
    __syncthreads();
    mma_atb_2x2(acc, A, B, 2 * qi, 2 * qj, kBlk);
  }
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 2; ++e) {
      const int row0 = ri + 16 * (2 * qi + a), col0 = rj + 16 * (2 * qj + e);
      if (row0 >= ld || col0 >= ld) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + 4 * q + rq, col = col0 + c;
        Mb[(int64_t)row * ld + col] = acc[a][e][q];
        Mb[(int64_t)col * ld + row] = acc[a][e][q];
      }
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

// Workgroups of a body_item grid: 8 * ceil(nb / 8) * nitems.
static unsigned body_grid(int nb, int nitems) { return (unsigned)(kXcds * ((nb + kXcds - 1) / kXcds) * nitems); }

void launch_chol(int nb, const int* offsets, int dim, const int64_t* moff, const double* M, double* Lf, double* Xf,
                 const int* active, const double* shift, double f0, double pivot_tol, int* fail, int max_rows,
                 hipStream_t s) {
  const int ldmax = (max_rows + 15) & ~15;
  hipLaunchKernelGGL(k_chol_init, dim3(ldmax, nb), dim3(64), 0, s, offsets, dim, moff, M, Lf, active, shift, f0,
                     fail);
  for (int c0 = 0; c0 < ldmax; c0 += kBlk) {
    const int W = std::min(kBlk, ldmax - c0);
    const int rows = ldmax - c0 - W;
    const int nblk = (rows + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(k_chol_diag, dim3(nb), dim3(256), 0, s, offsets, dim, moff, Lf, Xf, active, c0, f0, pivot_tol,
                       fail);
    if (nblk > 0) {
      const int np = nblk * (nblk + 1) / 2;
      hipLaunchKernelGGL(k_chol_trsm, dim3(body_grid(nb, nblk)), dim3(256), 0, s, offsets, dim, moff, Lf, Xf, active,
                         c0, nb, nblk);
      hipLaunchKernelGGL(k_chol_syrk, dim3(body_grid(nb, np)), dim3(256), 0, s, offsets, dim, moff, Lf, active, c0,
                         nb, np);
    }
  }
}

void launch_chol_inverse(int nb, const int* offsets, int dim, const int64_t* moff, double* Lf, double* Minv,
                         double* X, int max_n, hipStream_t s) {
  const int nblk = (max_n + kBlk - 1) / kBlk;
  if (nblk > 1)
    hipLaunchKernelGGL(k_tri_inv, dim3(body_grid(nb, nblk - 1)), dim3(256), 0, s, offsets, dim, moff, Lf, X, nb,
                       nblk - 1);
  const int np = nblk * (nblk + 1) / 2;
  hipLaunchKernelGGL(k_xtx, dim3(body_grid(nb, np)), dim3(256), 0, s, offsets, dim, moff, X, Minv, nb, np);
}

void launch_mob_apply(int nb, const int* offsets, int dim, const int64_t* moff, const double* Minv,
                      const double* dU, double* lam, int max_rows, hipStream_t s) {
  const unsigned g = (unsigned)((max_rows + 3) / 4);
  hipLaunchKernelGGL(k_mob_apply, dim3(g, nb), dim3(256), 0, s, offsets, dim, moff, Minv, dU, lam);
}

}  // namespace ibr
