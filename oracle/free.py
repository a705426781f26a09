"""Free kinematics: rigid bodies that move under applied forces and torques.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 2 poses the problem: instead of a prescribed motion, a body is subject to
a specified external force F and torque T (gravity in sedimentation), and its
linear and angular velocities are unknowns.  Sec. 8 names the enlarged
saddle-point system this leads to, whose extra Schur complement is the body
mobility N = (K* M^-1 K)^-1, and proposes one block per body for its
approximation.  The system itself is not printed in the text available here,
so this module writes it out from those statements (the reading used
throughout):

    A v + G pi - S Lambda        = g
    -D v                         = hp
    -J v + K U                   = W
    K* Lambda                    = f

U_p = (u_p, omega_p) holds the velocities of free body p; K maps them to the
rigid velocity of its markers, (K U)_i = u_p + omega_p x (R_i - X_p); its
adjoint K* sums marker forces into the body force and torque
[sum Lambda_i, sum (R_i - X_p) x Lambda_i]; f_p = (F_p, T_p) is the applied
load, so that at the solution each free body hands exactly its applied load
to the fluid (Lambda is the force on the fluid, as everywhere here).  Markers
of free bodies carry W_i = 0 (no prescribed slip); bodies with prescribed
motion keep W_i = -V_i and have no unknown in U.  For periodic steady Stokes
S is S' (eq. constrained_periodic), so a net applied load is balanced by the
uniform back-flow of Sec. 3.4.

Eliminating the fluid as in Sec. 3.3 (v~ the unconstrained solution for
(g, hp), M = J L^-1 S):

    M Lambda - K U = -(W + J v~)  =: r,      K* Lambda = f,

which the oracle solves as written, as one dense bordered system
[[M, -K], [K*, 0]] when the mobility is small enough to form, otherwise by
conjugate gradients on M for r and for each column of K followed by
U = N (f - K* M^-1 r), Lambda = M^-1 (r + K U).  Then v = v~ + L^-1 S Lambda.
"""
import numpy as np

from . import constrained, ib


def rotation_dofs(d):
    return 3 if d == 3 else 1


def rigid_matrix(R, offsets, centres, L, bodies):
    """K as a dense [N d, q len(bodies)] matrix, q = d + rotations; the
    columns of body p are its d translations, then its rotations (about the
    z axis in 2D, about x, y, z in 3D), each evaluated on its own markers."""
    N, d = R.shape
    nr = rotation_dofs(d)
    q = d + nr
    K = np.zeros((N * d, q * len(bodies)))
    for j, p in enumerate(bodies):
        lo, hi = offsets[p], offsets[p + 1]
        r = ib.min_image(R[lo:hi] - centres[p], L)
        for i in range(lo, hi):
            ri = r[i - lo]
            for a in range(d):
                K[i * d + a, j * q + a] = 1.0
            if d == 2:
                # omega e_z x r = (-omega r_y, omega r_x)
                K[i * d + 0, j * q + 2] = -ri[1]
                K[i * d + 1, j * q + 2] = ri[0]
            else:
                # e_b x r for b = x, y, z
                K[i * d + 1, j * q + 3] = -ri[2]
                K[i * d + 2, j * q + 3] = ri[1]
                K[i * d + 0, j * q + 4] = ri[2]
                K[i * d + 2, j * q + 4] = -ri[0]
                K[i * d + 0, j * q + 5] = -ri[1]
                K[i * d + 1, j * q + 5] = ri[0]
    return K


def constraint_rhs(R, offsets, centres, U, Omega, L, free):
    """W: -V_i on the markers of prescribed bodies, 0 on those of free bodies."""
    W = -ib.marker_velocities(R, offsets, centres, U, Omega, L)
    b = ib.body_of(offsets)
    W[np.asarray(free, dtype=bool)[b]] = 0.0
    return W


def load_vector(F, T, bodies):
    """f stacked body by body as [F_p, T_p]."""
    return np.concatenate([np.concatenate([F[p], T[p]]) for p in bodies])


def _cg(apply, b, tol, maxiter):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    bn = np.sqrt(b @ b)
    it = 0
    while np.sqrt(rr) > tol * bn and it < maxiter:
        Ap = apply(p)
        alpha = rr / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rn = r @ r
        p = r + (rn / rr) * p
        rr = rn
        it += 1
    return x


def solve(sysm, g, hp, W, offsets, centres, free, F, T, dense_limit=2400, tol=1e-14, maxiter=5000):
    """Exact solution of the free-kinematics system.

    free[p] != 0 marks body p free with applied force F[p] and torque T[p]
    (ignored for prescribed bodies).  Returns (Solution, Ufree [nb, d],
    Omfree [nb, 1|3]) with zeros in the rows of prescribed bodies.
    """
    d, n = sysm.d, sysm.n
    N = sysm.R.shape[0]
    L = n * sysm.h
    nb = len(offsets) - 1
    bodies = [p for p in range(nb) if free[p]]
    nr = rotation_dofs(d)
    q = d + nr
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    vt, pt = sysm.stokes(g, hp)
    r = -(W + sysm.interp(vt)).reshape(-1)
    K = rigid_matrix(sysm.R, offsets, centres, L, bodies)
    f = load_vector(F, T, bodies) if bodies else np.zeros(0)
    nu = K.shape[1]
    if N * d <= dense_limit:
        M = sysm.mobility_dense()
        big = np.zeros((N * d + nu, N * d + nu))
        big[:N * d, :N * d] = M
        big[:N * d, N * d:] = -K
        big[N * d:, :N * d] = K.T
        x = np.linalg.solve(big, np.concatenate([r, f]))
        lam, Uq = x[:N * d], x[N * d:]
    else:
        apply = lambda z: sysm.mobility_apply(z.reshape(N, d)).reshape(-1)
        Mr = _cg(apply, r, tol, maxiter)
        MK = np.stack([_cg(apply, K[:, j].copy(), tol, maxiter) for j in range(nu)], axis=1) if nu else \
            np.zeros((N * d, 0))
        Ninv = K.T @ MK
        Uq = np.linalg.solve(Ninv, f - K.T @ Mr) if nu else np.zeros(0)
        lam = Mr + MK @ Uq
    lam = lam.reshape(N, d)
    vl, pl = sysm.stokes(sysm.spread(lam))
    v = vt + vl
    p = pt + pl
    p = p - p.mean()
    Fo, To = ib.body_force_torque(lam, sysm.R, offsets, centres, L)
    Uf = np.zeros((nb, d))
    Of = np.zeros((nb, nr))
    for j, b in enumerate(bodies):
        Uf[b] = Uq[j * q:j * q + d]
        Of[b] = Uq[j * q + d:(j + 1) * q]
    return constrained.Solution(v=v, p=p, lam=lam, F=Fo, T=To), Uf, Of


def solve_problem(prob, free, F, T, g=None, hp=None, **kw):
    """Free-kinematics solve of a synthetic problem: bodies with free[p] move
    under (F[p], T[p]), the others with their prescribed U, Omega."""
    sysm = constrained.System.from_problem(prob)
    W = constraint_rhs(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L, free)
    return solve(sysm, g, hp, W, prob.offsets, prob.centres, free, F, T, **kw)
