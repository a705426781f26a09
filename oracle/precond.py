"""Preconditioners of Sec. 5: P_S^-1 (eq. P1_practical), the inner Stokes GMRES
and the Schur-complement preconditioner of Sec. 5.1.

P_S^-1 applied to (g, hp), Sec. 5.2:
    v*  = A~^-1 g                     one V-cycle per velocity component
    q   = -D v* - hp
    phi = L~_p^-1 q                   one Poisson V-cycle, L_p = h^2 D G
    v   = v* + h^2 G phi
    pi  = B~^-1 q = -(rho h^2/dt) phi + eta q     (steady: eta q)
With exact sub-solves this is the exact inverse of the periodic Stokes operator.

Inner solver (Sec. 5.2): GMRES on [[A, G], [-D, 0]] with right preconditioner
P_S^-1, zero initial guess and a fixed number N_s of iterations (Arnoldi by
modified Gram-Schmidt, least squares by a dense solve of the small Hessenberg
problem).

Schur-complement preconditioner for a residual (r_v, r_p, r_L), Sec. 5.1:
    1. (v, pi) = inner solve of the fluid problem with (r_v, r_p)
    2. dU = -(J v + r_L)
    3. Lambda = M~^-1 dU, block by block (per body)
    4. (full variant only) re-solve the fluid problem with r_v + S' Lambda
With free bodies (module ``free``) step 3 becomes, for each free body, the
per-body block Sec. 8 proposes: the small saddle problem
M~ Lambda - K U = dU, K* Lambda = r_U, solved as U = N~ (r_U - K* M~^-1 dU),
Lambda = M~^-1 (dU + K U) with N~ = (K* M~^-1 K)^-1; prescribed bodies pass
their body rows through (z_U = r_U).
"""
import numpy as np

from . import free as free_mod
from . import grid, mobility, multigrid, stokes


class MGParams:
    """V-cycle sweeps; exact=True swaps each V-cycle for the exact periodic solve."""

    def __init__(self, nu_pre=2, nu_post=2, nu_coarse=4, exact=False):
        self.nu_pre = nu_pre
        self.nu_post = nu_post
        self.nu_coarse = nu_coarse
        self.exact = exact


def ps_inv(g, hp, c0, eta, h, mg=None):
    """P_S^-1 (g, hp)."""
    mg = mg or MGParams()
    d = g.shape[0]

    def cyc(b, a0, a1):
        if mg.exact:
            return stokes.helmholtz_solve(b, a0, a1)
        return multigrid.vcycle(b, a0, a1, mg.nu_pre, mg.nu_post, mg.nu_coarse)

    vstar = np.stack([cyc(g[a], c0, eta / (h * h)) for a in range(d)])
    q = -grid.div(vstar, h) - hp
    # L_p phi = q with L_p the dimensionless Laplacian  <=>  (0 - 1 L) phi = -q
    phi = cyc(-q, 0.0, 1.0)
    v = vstar + h * h * grid.grad(phi, h)
    p = -(c0 * h * h) * phi + eta * q
    return v, p


def stokes_gmres(g, hp, c0, eta, h, ns, mg=None):
    """Right-preconditioned GMRES(ns) for the unconstrained Stokes system, x0 = 0."""
    d = g.shape[0]
    shape_v, shape_p = g.shape, hp.shape

    def pack(v, p):
        return np.concatenate([v.reshape(-1), p.reshape(-1)])

    def unpack(x):
        nv = g.size
        return x[:nv].reshape(shape_v), x[nv:].reshape(shape_p)

    b = pack(g, hp)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(g), np.zeros_like(hp)
    Q = [b / beta]
    Z = []
    H = np.zeros((ns + 1, ns))
    k_used = 0
    for j in range(ns):
        zv, zp = ps_inv(*unpack(Q[j]), c0, eta, h, mg)
        Z.append(pack(zv, zp))
        wv, wp = grid.stokes_apply(zv, zp, c0, eta, h)
        w = pack(wv, wp)
        for i in range(j + 1):
            H[i, j] = w @ Q[i]
            w = w - H[i, j] * Q[i]
        H[j + 1, j] = np.linalg.norm(w)
        k_used = j + 1
        if H[j + 1, j] == 0.0:
            break
        Q.append(w / H[j + 1, j])
    e1 = np.zeros(k_used + 1)
    e1[0] = beta
    y, *_ = np.linalg.lstsq(H[:k_used + 1, :k_used], e1, rcond=None)
    x = sum(y[i] * Z[i] for i in range(k_used))
    return unpack(x)


class SchurPreconditioner:
    """Sec. 5.1 preconditioner for one problem (steady periodic uses S')."""

    def __init__(self, sysm, offsets, mob_blocks, mob_params, ns=2, full=False, mg=None, free=None,
                 centres=None):
        self.s = sysm
        self.offsets = offsets
        self.ns = ns
        self.full = full
        self.mg = mg or MGParams()
        f0 = mobility.self_term(mob_params)
        self.factors = []
        self.shifts = []
        for M in mob_blocks:
            Lc, sh = mobility.factor_block(M, f0)
            self.factors.append(Lc)
            self.shifts.append(sh)
        # free bodies: K_p, Y_p = M~_p^-1 K_p and N~_p = (K_p* Y_p)^-1
        self.free = None if free is None or not np.any(free) else [bool(f) for f in free]
        self.body_blocks = {}
        if self.free:
            L = sysm.n * sysm.h
            for b, fr in enumerate(self.free):
                if not fr:
                    continue
                lo, hi = offsets[b], offsets[b + 1]
                d = sysm.d
                Kb = free_mod.rigid_matrix(sysm.R, offsets, centres, L, [b])[lo * d:hi * d]
                Lc = self.factors[b]
                Y = np.linalg.solve(Lc.T, np.linalg.solve(Lc, Kb))
                self.body_blocks[b] = (Kb, Y, np.linalg.inv(Kb.T @ Y))

    def mobility_solve(self, dU):
        lam = np.zeros_like(dU)
        d = dU.shape[1]
        for b, Lc in enumerate(self.factors):
            lo, hi = self.offsets[b], self.offsets[b + 1]
            rhs = dU[lo:hi].reshape(-1)
            y = np.linalg.solve(Lc, rhs)
            lam[lo:hi] = np.linalg.solve(Lc.T, y).reshape(-1, d)
        return lam

    def apply(self, rv, rp, rl, ru=None):
        """z = P r.  With free bodies ru [nb, d + rotations] holds the body
        rows of r (force then torque rows per body) and the body rows of z
        are returned as a fourth value in the same layout."""
        s = self.s
        v, p = stokes_gmres(rv, rp, s.c0, s.eta, s.h, self.ns, self.mg)
        dU = -(s.interp(v) + rl)
        lam = self.mobility_solve(dU)
        zu = None
        if self.free:
            zu = np.array(ru, dtype=np.float64, copy=True)
            d = s.d
            for b, (Kb, Y, Nb) in self.body_blocks.items():
                lo, hi = self.offsets[b], self.offsets[b + 1]
                t = lam[lo:hi].reshape(-1)
                U = Nb @ (ru[b] - Kb.T @ t)
                lam[lo:hi] = (t + Y @ U).reshape(-1, d)
                zu[b] = U
        if self.full:
            v, p = stokes_gmres(rv + s.spread(lam), rp, s.c0, s.eta, s.h, self.ns, self.mg)
        if self.free:
            return v, p, lam, zu
        return v, p, lam


def for_problem(prob, sysm, ns=2, full=False, mg=None, R=None, free=None):
    blocks, p = mobility.blocks_for_problem(prob, R=R)
    return SchurPreconditioner(sysm, prob.offsets, blocks, p, ns=ns, full=full, mg=mg, free=free,
                               centres=prob.centres)

