"""Analytic approximate mobility M~ of Sec. 4 (eq. M_tilde_ij), per body.

    M~_ij = f(r_ij) I + g(r_ij) r^_ij (x) r^_ij,  r_ij = R_i - R_j (minimum image)

The paper's fitted coefficients are published outside the paper, so M~ is built
from the analytic forms the paper gives (a documented reading; M~ only changes
iteration counts, never the converged answer):

* 3D steady Stokes: the RPY tensor (eq. RPYTensor) with the four-point kernel's
  hydrodynamic radius a = 1.25 h (Sec. 4.1 footnote), shifted by the periodic
  correction -2.84 / (6 pi eta l) of Appendix A for a periodic box of side l.
* 3D finite beta: self term f(0) = 1 / (1/f_0(0) + 1/f_inf(0)), which moves
  between the inviscid limit f_0(0) = ((d-1)/d)(dt/rho)/V_m (eq. f_0_inviscid)
  and Stokes' drag f_inf(0) = 1/(6 pi eta a); V_m = (8/3)^d h^d for the
  four-point kernel (its squared weights sum to 3/8 per dimension).  For
  r >= 2a the Brinkmanlet (eq. Brinkmanlet_3D) with alpha^2 = rho/(eta dt);
  for r < 2a a linear blend from (f(0), 0) to the Brinkmanlet values at 2a.
* 2D steady Stokes (Appendix B): f(0) = ln(l / (3.708 a)) / (4 pi eta) and the
  regularised logarithm f(r) = f(0) - ln(1 + r^2/a^2) / (8 pi eta),
  g(r) = r^2 / ((r^2 + a^2) 4 pi eta), which has the far-field behaviour of
  eq. fg_asympt_2D.
* 2D finite beta: the same self-term blend with d = 2 and the 2D inviscid dipole
  (eq. fg_inv_2D) for r >= 2a, blended linearly below 2a.

If the Cholesky factorisation of a block fails (Sec. 5.3 filters small or
negative eigenvalues with an SVD pseudo-inverse), the block is regularised as
M~ + s f(0) I for the first s in SHIFTS that factors with every pivot above
PIVOT_TOL f(0); ``factor_block`` implements that reading.
"""
import math

import numpy as np

A3D_FACTOR = 1.25    # hydrodynamic radius of a four-point marker in 3D, units of h
A2D_FACTOR = 1.04    # 2D four-point marker radius in f(0) = ln(l/(3.708 a))/(4 pi eta), units of h
PERIODIC_3D = 2.84   # periodic correction coefficient of the Oseen tensor (Appendix A)


def rpy(r, a, eta):
    """RPY f(r), g(r) (eq. RPYTensor)."""
    r = np.asarray(r, dtype=np.float64)
    c = 1.0 / (6.0 * math.pi * eta * a)
    far = r > 2.0 * a
    rs = np.where(far, r, 1.0)
    f = np.where(far, c * (0.75 * a / rs + 0.5 * a ** 3 / rs ** 3), c * (1.0 - 9.0 * r / (32.0 * a)))
    g = np.where(far, c * (0.75 * a / rs - 1.5 * a ** 3 / rs ** 3), c * (3.0 * r / (32.0 * a)))
    return f, g


def brinkmanlet(r, alpha, eta):
    """Brinkman Green's function f_B, g_B (eq. Brinkmanlet_3D), r > 0."""
    r = np.asarray(r, dtype=np.float64)
    ar = alpha * r
    e = np.exp(-ar) / (4.0 * math.pi * eta * r)
    f = e * (1.0 / ar ** 2 + 1.0 / ar + 1.0) - 1.0 / (4.0 * math.pi * eta * alpha ** 2 * r ** 3)
    g = -e * (3.0 / ar ** 2 + 3.0 / ar + 1.0) + 3.0 / (4.0 * math.pi * eta * alpha ** 2 * r ** 3)
    return f, g


def marker_volume(d, h):
    return (8.0 / 3.0) ** d * h ** d


def self_inviscid(d, h, rho, dt):
    return (d - 1.0) / d * (dt / rho) / marker_volume(d, h)


def params_for(d, h, L, rho, eta, dt):
    """Scalars that define f, g for a box of side L."""
    steady = rho == 0.0
    if d == 3:
        a = A3D_FACTOR * h
        finf = 1.0 / (6.0 * math.pi * eta * a)
    else:
        a = A2D_FACTOR * h
        finf = math.log(L / (3.708 * a)) / (4.0 * math.pi * eta)
    p = {"d": d, "a": a, "eta": eta, "L": L, "steady": steady, "finf0": finf}
    if not steady:
        f0 = self_inviscid(d, h, rho, dt)
        p["f00"] = 1.0 / (1.0 / f0 + 1.0 / finf)
        p["alpha"] = math.sqrt(rho / (eta * dt))
        p["dt_rho"] = dt / rho
    return p


def fg(r, p):
    """f(r), g(r) of the approximate mobility for parameters from ``params_for``."""
    r = np.asarray(r, dtype=np.float64)
    d, a, eta = p["d"], p["a"], p["eta"]
    if p["steady"]:
        if d == 3:
            f, g = rpy(r, a, eta)
            return f - PERIODIC_3D / (6.0 * math.pi * eta * p["L"]), g
        c = 1.0 / (4.0 * math.pi * eta)
        f = p["finf0"] - 0.5 * c * np.log1p(r * r / (a * a))
        g = c * r * r / (r * r + a * a)
        return f, g
    f00 = p["f00"]
    r2a = 2.0 * a
    if d == 3:
        fb = lambda s: brinkmanlet(s, p["alpha"], eta)  # noqa: E731
    else:
        def fb(s):
            s = np.asarray(s, dtype=np.float64)
            return (-p["dt_rho"] / (2.0 * math.pi * s * s), p["dt_rho"] / (math.pi * s * s))
    near = r < r2a
    rs = np.where(near, r2a, r)
    ff, gf = fb(rs)
    f2a, g2a = fb(np.array(r2a))
    t = r / r2a
    f = np.where(near, f00 + t * (f2a - f00), ff)
    g = np.where(near, t * g2a, gf)
    return f, g


def self_term(p):
    f, _ = fg(np.array(0.0), p)
    return float(f)


def block(Rb, p):
    """Dense M~ for one body's markers Rb [Np, d] (minimum-image pair vectors)."""
    Np, d = Rb.shape
    L = p["L"]
    dr = Rb[:, None, :] - Rb[None, :, :]
    dr = dr - L * np.round(dr / L)
    r = np.sqrt((dr ** 2).sum(axis=2))
    f, g = fg(r, p)
    rhat = np.where(r[..., None] > 0, dr / np.where(r > 0, r, 1.0)[..., None], 0.0)
    M = f[:, :, None, None] * np.eye(d)[None, None] + g[:, :, None, None] * rhat[:, :, :, None] * rhat[:, :, None, :]
    return M.transpose(0, 2, 1, 3).reshape(Np * d, Np * d)


SHIFTS = (0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.3, 0.4, 0.5, 0.7, 1.0, 1.5, 2.0, 3.0, 5.0, 10.0, 20.0, 50.0)
PIVOT_TOL = 1e-8


def factor_block(M, f0):
    """Cholesky factor of M + s f0 I for the first shift s in SHIFTS that factors.

    A factorisation counts as failed when a pivot (squared diagonal of the
    factor) is not above PIVOT_TOL * f0.  Returns (L, s).
    """
    for s in SHIFTS:
        try:
            Lc = np.linalg.cholesky(M + s * f0 * np.eye(M.shape[0]))
        except np.linalg.LinAlgError:
            continue
        if np.min(np.diag(Lc)) ** 2 > PIVOT_TOL * f0:
            return Lc, s
    raise np.linalg.LinAlgError("mobility block could not be factored")


def blocks_for_problem(prob, R=None):
    R = prob.R if R is None else R
    p = params_for(prob.dim, prob.h, prob.L, prob.rho, prob.eta, prob.dt)
    out = []
    for b in range(prob.nbodies):
        Rb = R[prob.offsets[b]:prob.offsets[b + 1]]
        out.append(block(Rb, p))
    return out, p
