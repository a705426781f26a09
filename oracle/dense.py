"""The constrained system assembled as a dense matrix and solved by LAPACK.

This is the independent check of ``constrained``: the operator of
eq. constrained_Stokes (eq. constrained_periodic when steady and periodic) is
built column by column from the stencil definitions in ``grid`` and ``ib``,
without any Fourier transform, and bordered with the gauge conditions that make
it nonsingular:

    mean(pi) = 0                       (the pressure null space)
    <v^alpha> = 0 for every alpha      (periodic steady Stokes only, Sec. 3.4)

The border adds one Lagrange-multiplier column per gauge row, spanning the
directions missing from the range (uniform momentum per component and uniform
continuity), so a consistent right-hand side gives multipliers equal to zero.
Only small grids are practical (16^2 in 2D, 8^3 in 3D).
"""
import numpy as np

from . import grid, ib


def unknown_sizes(d, n, N):
    C = n ** d
    return d * C, C, d * N


def apply_operator(sysm, x):
    """K x for the stacked vector x = [v (d*C), pi (C), Lambda (d*N)]."""
    d, n = sysm.d, sysm.n
    nv, npr, nl = unknown_sizes(d, n, sysm.R.shape[0])
    v = x[:nv].reshape((d,) + (n,) * d)
    p = x[nv:nv + npr].reshape((n,) * d)
    lam = x[nv + npr:].reshape(-1, d)
    rm, rc = grid.stokes_apply(v, p, sysm.c0, sysm.eta, sysm.h)
    rm = rm - sysm.spread(lam)
    rl = -sysm.interp(v)
    return np.concatenate([rm.reshape(-1), rc.reshape(-1), rl.reshape(-1)])


def assemble(sysm):
    d, n = sysm.d, sysm.n
    nv, npr, nl = unknown_sizes(d, n, sysm.R.shape[0])
    tot = nv + npr + nl
    K = np.zeros((tot, tot))
    e = np.zeros(tot)
    for j in range(tot):
        e[j] = 1.0
        K[:, j] = apply_operator(sysm, e)
        e[j] = 0.0
    return K


def gauge_rows(sysm):
    d, n = sysm.d, sysm.n
    C = n ** d
    nv, npr, nl = unknown_sizes(d, n, sysm.R.shape[0])
    tot = nv + npr + nl
    rows = []
    r = np.zeros(tot)
    r[nv:nv + npr] = 1.0 / C
    rows.append(r)
    if sysm.steady:
        for a in range(d):
            r = np.zeros(tot)
            r[a * C:(a + 1) * C] = 1.0 / C
            rows.append(r)
    return np.array(rows)


def solve(sysm, g, hp, W):
    """Dense LAPACK solve; returns (v, pi, Lambda, gauge multipliers)."""
    d, n = sysm.d, sysm.n
    N = sysm.R.shape[0]
    nv, npr, nl = unknown_sizes(d, n, N)
    K = assemble(sysm)
    Cg = gauge_rows(sysm)
    ng = Cg.shape[0]
    big = np.zeros((K.shape[0] + ng, K.shape[0] + ng))
    big[:K.shape[0], :K.shape[0]] = K
    big[K.shape[0]:, :K.shape[0]] = Cg
    big[:K.shape[0], K.shape[0]:] = Cg.T
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    if hp is None:
        hp = np.zeros((n,) * d)
    rhs = np.concatenate([g.reshape(-1), hp.reshape(-1), W.reshape(-1), np.zeros(ng)])
    x = np.linalg.solve(big, rhs)
    v = x[:nv].reshape((d,) + (n,) * d)
    p = x[nv:nv + npr].reshape((n,) * d)
    lam = x[nv + npr:nv + npr + nl].reshape(N, d)
    return v, p, lam, x[nv + npr + nl:]


def solve_free(sysm, g, hp, W, offsets, centres, free, F, T):
    """The free-kinematics system (see ``free``) assembled densely and solved
    by LAPACK: the constrained operator above, bordered by one column per
    rigid degree of freedom of each free body (the marker velocities of a unit
    translation or rotation, from ``ib.marker_velocities``) and one row per
    degree of freedom (its force or torque, from ``ib.body_force_torque``),
    plus the gauge rows.  Returns (v, pi, Lambda, U [nb, d], Omega [nb, 1|3])
    with zero velocities in the rows of prescribed bodies."""
    d, n = sysm.d, sysm.n
    N = sysm.R.shape[0]
    L = n * sysm.h
    nb = len(offsets) - 1
    nr = 3 if d == 3 else 1
    nv, npr, nl = unknown_sizes(d, n, N)
    K0 = assemble(sysm)
    base = K0.shape[0]
    dofs = [(p, k) for p in range(nb) if free[p] for k in range(d + nr)]
    nu = len(dofs)
    Cg = gauge_rows(sysm)
    ng = Cg.shape[0]
    tot = base + nu + ng
    big = np.zeros((tot, tot))
    big[:base, :base] = K0
    for j, (p, k) in enumerate(dofs):
        U = np.zeros((nb, d))
        Om = np.zeros((nb, nr))
        if k < d:
            U[p, k] = 1.0
        else:
            Om[p, k - d] = 1.0
        col = ib.marker_velocities(sysm.R, offsets, centres, U, Om, L)
        big[nv + npr:base, base + j] = col.reshape(-1)
    for i in range(nl):
        lam = np.zeros(nl)
        lam[i] = 1.0
        Fu, Tu = ib.body_force_torque(lam.reshape(N, d), sysm.R, offsets, centres, L)
        for j, (p, k) in enumerate(dofs):
            big[base + j, nv + npr + i] = Fu[p, k] if k < d else Tu[p, k - d]
    big[base + nu:, :base] = Cg
    big[:base, base + nu:] = Cg.T
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    if hp is None:
        hp = np.zeros((n,) * d)
    f = np.array([F[p, k] if k < d else T[p, k - d] for p, k in dofs])
    rhs = np.concatenate([g.reshape(-1), hp.reshape(-1), W.reshape(-1), f, np.zeros(ng)])
    x = np.linalg.solve(big, rhs)
    v = x[:nv].reshape((d,) + (n,) * d)
    p_ = x[nv:nv + npr].reshape((n,) * d)
    lam = x[nv + npr:base].reshape(N, d)
    Uo = np.zeros((nb, d))
    Oo = np.zeros((nb, nr))
    for j, (p, k) in enumerate(dofs):
        if k < d:
            Uo[p, k] = x[base + j]
        else:
            Oo[p, k - d] = x[base + j]
    return v, p_, lam, Uo, Oo
