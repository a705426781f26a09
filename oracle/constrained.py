"""Exact solution of the rigidly constrained Stokes system, Secs. 3.2-3.4.

The system (eq. constrained_Stokes; eq. constrained_periodic for periodic
steady Stokes, where S is replaced by S' and <v> = 0 is imposed) is

    A v + G pi - S Lambda = g
    -D v                  = hp
    -J v                  = W

Sec. 3.3 eliminates the fluid: the unconstrained solution (v~, pi~) of
eq. Stokes_saddle with right-hand side (g, hp), then the mobility system
(eq. lambda_sol)

    M Lambda = -(W + J v~),     M = J L^-1 S     (eq. mob_def),

then v = v~ + L^-1 S Lambda (and the matching pressure).  L^-1 is applied
exactly by the Fourier solve of ``stokes``.  M is formed densely from its dN
columns (unit marker forces) when dN is small, otherwise the mobility system is
solved by conjugate gradients, M being symmetric positive definite.

For prescribed rigid motion W = -V with V_i = U_p + Omega_p x (R_i - X_p).
Outputs follow the paper's sign: Lambda is the force the markers apply to the
fluid, F_p = sum Lambda_i and T_p = sum (R_i - X_p) x Lambda_i; the pressure is
returned with zero mean.
"""
from dataclasses import dataclass

import numpy as np

from . import ib, stokes


@dataclass
class Solution:
    v: np.ndarray      # [d, n..]
    p: np.ndarray      # [n..]
    lam: np.ndarray    # [N, d]
    F: np.ndarray      # [nb, d]
    T: np.ndarray      # [nb, 1 or 3]
    cg_iters: int = 0


class System:
    """Operators of one problem: c0 = rho/dt (0 when steady), eta, h, markers."""

    def __init__(self, dim, n, h, c0, eta, R):
        self.d = dim
        self.n = n
        self.h = h
        self.c0 = c0
        self.eta = eta
        self.R = np.asarray(R, dtype=np.float64)
        self.steady = c0 == 0.0
        self.W = ib.all_weights(self.R, n, h)   # tap indices and weights, fixed with R

    @classmethod
    def from_problem(cls, prob, R=None):
        c0 = 0.0 if prob.steady else prob.rho / prob.dt
        return cls(prob.dim, prob.n, prob.h, c0, prob.eta, prob.R if R is None else R)

    # S (or S' when steady periodic)
    def spread(self, lam):
        if self.steady:
            return ib.spread_periodic_steady(lam, self.R, self.n, self.h, self.W)
        return ib.spread(lam, self.R, self.n, self.h, self.W)

    def interp(self, v):
        return ib.interp(v, self.R, self.h, self.W)

    def stokes(self, f, hp=None):
        return stokes.solve(f, hp, self.c0, self.eta, self.h, self.d)

    def mobility_apply(self, lam):
        """M Lambda = J L^-1 S Lambda."""
        v, _ = self.stokes(self.spread(lam))
        return self.interp(v)

    def mobility_dense(self, batch=32):
        """Dense [dN, dN] mobility, column (i, alpha) = M applied to a unit force."""
        N, d = self.R.shape
        M = np.zeros((N * d, N * d))
        cols = [(i, a) for i in range(N) for a in range(d)]
        for s in range(0, len(cols), batch):
            chunk = cols[s:s + batch]
            f = np.zeros((len(chunk), d) + (self.n,) * d)
            for b, (i, a) in enumerate(chunk):
                lam = np.zeros((N, d))
                lam[i, a] = 1.0
                f[b] = self.spread(lam)
            v, _ = self.stokes(f)
            for b, (i, a) in enumerate(chunk):
                M[:, i * d + a] = self.interp(v[b]).reshape(-1)
        return M

    def solve_mobility(self, rhs, dense_limit=2400, tol=1e-14, maxiter=5000):
        """Solve M Lambda = rhs ([N, d]); returns (Lambda, cg iterations or 0)."""
        N, d = self.R.shape
        if N * d <= dense_limit:
            M = self.mobility_dense()
            lam = np.linalg.solve(M, rhs.reshape(-1))
            return lam.reshape(N, d), 0
        # conjugate gradients on the SPD mobility
        b = rhs.reshape(-1)
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        bnorm = np.sqrt(b @ b)
        it = 0
        while np.sqrt(rr) > tol * bnorm and it < maxiter:
            Ap = self.mobility_apply(p.reshape(N, d)).reshape(-1)
            alpha = rr / (p @ Ap)
            x += alpha * p
            r -= alpha * Ap
            rr_new = r @ r
            p = r + (rr_new / rr) * p
            rr = rr_new
            it += 1
        return x.reshape(N, d), it


def solve(sysm: System, g, hp, W, offsets, centres, **kw) -> Solution:
    """Exact solution for right-hand side (g, hp, W); g, hp may be None (zero)."""
    d, n = sysm.d, sysm.n
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    vt, pt = sysm.stokes(g, hp)
    rhs = -(W + sysm.interp(vt))
    lam, its = sysm.solve_mobility(rhs, **kw)
    vl, pl = sysm.stokes(sysm.spread(lam))
    v = vt + vl
    p = pt + pl
    p = p - p.mean()
    L = n * sysm.h
    F, T = ib.body_force_torque(lam, sysm.R, offsets, centres, L)
    return Solution(v=v, p=p, lam=lam, F=F, T=T, cg_iters=its)


def solve_problem(prob, g=None, hp=None, **kw) -> Solution:
    """Exact solution of a prescribed-motion problem (W = -V)."""
    sysm = System.from_problem(prob)
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    return solve(sysm, g, hp, -V, prob.offsets, prob.centres, **kw)


def residual(sysm: System, v, p, lam, g, hp, W):
    """Blocks of b - K x for the system as written (S' when steady periodic)."""
    from . import grid
    d, n = sysm.d, sysm.n
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    if hp is None:
        hp = np.zeros((n,) * d)
    rm, rc = grid.stokes_apply(v, p, sysm.c0, sysm.eta, sysm.h)
    rm = g - (rm - sysm.spread(lam))
    rc = hp - rc
    rl = W - (-sysm.interp(v))
    return rm, rc, rl
