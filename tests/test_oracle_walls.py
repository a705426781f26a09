"""Pins of the slit-channel oracle (``oracle.walls``): no-slip walls at both
ends of the last axis, periodic along the others.

What pins it, other than itself:
* the discrete Laplacian with the walls' extension has the sine / cosine
  eigenvectors its boundary rule implies (closed forms);
* D = -G^T, and D G is the Neumann Laplacian;
* closed-form discrete flows: plane Poiseuille flow under a uniform force
  along the walls, and rest with a hydrostatic pressure under a uniform
  force across them;
* J = J0 E and S = E^T S0 are adjoint, equal the periodic taps away from the
  walls, and interpolate zero tangential velocity at a wall (the property the
  appendix gives for choosing this extension);
* the constrained solve through the mobility equals a dense LAPACK solve of
  the whole system assembled column by column from the stencils;
* mirror symmetry about the midplane, and mobilities that fall as a marker
  approaches a wall;
* the V-cycle with the walls' rules converges to the exact discrete solution.
"""
import math

import numpy as np
import pytest

from oracle import ib, walls
from synthetic import slit_problem, slit_shell


def _sh(n, d):
    return (n,) + (1,) * (d - 1)


@pytest.mark.parametrize("d,n", [(2, 16), (3, 8)])
def test_laplacian_eigenvectors(d, n):
    """Tangential: sin(pi m (k+1/2)/n) (the mirror with the sign reversed),
    normal: sin(pi m k/n) on faces (zero on the walls), Neumann: cos(pi m
    (k+1/2)/n); times a Fourier mode along the periodic axes.  Eigenvalue
    -4 sin^2(pi m / 2n) - 4 sin^2(theta/2)."""
    k = np.arange(n)
    x = np.arange(n)
    th = 2 * math.pi * 3 / n
    per = np.cos(th * x)                        # along the fastest (periodic) axis
    lam_p = -4 * math.sin(th / 2) ** 2
    for m in (1, 2, n - 1):
        lam_z = -4 * math.sin(math.pi * m / (2 * n)) ** 2
        for kind, prof in ((walls.CELL_DIR, np.sin(math.pi * m * (k + 0.5) / n)),
                           (walls.FACE_DIR, np.sin(math.pi * m * k / n)),
                           (walls.CELL_NEU, np.cos(math.pi * m * (k + 0.5) / n))):
            f = prof.reshape(_sh(n, d)) * per.reshape((1,) * (d - 1) + (n,))
            f = np.broadcast_to(f, (n,) * d).copy()
            got = walls.lap(f, kind)
            if kind == walls.CELL_NEU:
                got = -walls.apply_op(f, 0.0, 1.0, kind)    # c0 - c1 L with c1 = 1, negated
            assert np.abs(got - (lam_z + lam_p) * f).max() < 1e-12


def test_div_is_minus_grad_transpose_and_neumann():
    d, n, h = 3, 4, 0.25
    C = n ** d
    G = np.zeros((d * C, C))
    D = np.zeros((C, d * C))
    for j in range(C):
        e = np.zeros(C)
        e[j] = 1
        G[:, j] = walls.grad(e.reshape((n,) * d), h).reshape(-1)
    for j in range(d * C):
        e = np.zeros(d * C)
        e[j] = 1
        D[:, j] = walls.div(e.reshape((d,) + (n,) * d), h).reshape(-1)
    wall = np.zeros((d,) + (n,) * d, dtype=bool)
    wall[d - 1][0] = True
    keep = ~wall.reshape(-1)
    assert np.abs(D[:, keep] + G[keep, :].T).max() < 1e-14   # D = -G^T on the unknowns
    assert np.abs(G[~keep]).max() == 0.0                     # no gradient on the wall faces
    Lneu = np.zeros((C, C))
    for j in range(C):
        e = np.zeros(C)
        e[j] = 1
        Lneu[:, j] = -walls.apply_op(e.reshape((n,) * d), 0.0, 1.0, walls.CELL_NEU).reshape(-1)
    assert np.abs(D @ G - Lneu / h ** 2).max() < 1e-12


@pytest.mark.parametrize("d,n", [(2, 16), (3, 8), (3, 16)])
def test_poiseuille_and_hydrostatic(d, n):
    h, eta = 1.0 / n, 1.3
    L = n * h
    z = (np.arange(n) + 0.5) * h
    f = np.zeros((d,) + (n,) * d)
    f[0] = 2.0
    v, p = walls.solve(f, None, 0.0, eta, h, d)
    # u'' = -f/eta with the reversed mirror at z = 0, L: the parabola shifted by h^2/4
    ex = 2.0 / (2 * eta) * (z * (L - z) + h * h / 4)
    assert np.abs(v[0] - ex.reshape(_sh(n, d))).max() < 1e-12
    assert np.abs(v[1:]).max() < 1e-13 and np.abs(p).max() < 1e-12
    f = np.zeros((d,) + (n,) * d)
    f[d - 1] = 3.0
    v, p = walls.solve(f, None, 0.0, eta, h, d)
    assert np.abs(v).max() < 1e-13
    assert np.abs(p - (3.0 * h * (np.arange(n) - (n - 1) / 2)).reshape(_sh(n, d))).max() < 1e-12


@pytest.mark.parametrize("c0", [0.0, 7.0])
def test_exact_solve_satisfies_operator(c0):
    d, n, h, eta = 3, 8, 1.0 / 8, 0.7
    rng = np.random.default_rng(2)
    f = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    hp -= hp.mean()
    v, p = walls.solve(f, hp, c0, eta, h, d)
    rm, rc = walls.stokes_apply(v, p, c0, eta, h)
    f[d - 1][0] = 0.0
    assert np.abs(rm - f).max() < 1e-12 * np.abs(f).max() * n * n
    assert np.abs(rc - hp).max() < 1e-12
    assert np.abs(v[d - 1][0]).max() == 0.0 and abs(p.mean()) < 1e-14


def test_spread_interp_adjoint_and_wall_property():
    d, n = 3, 16
    h = 1.0 / n
    L = n * h
    rng = np.random.default_rng(4)
    R = rng.uniform(0, L, size=(40, d))
    R[:, 2] = rng.uniform(1e-3, L - 1e-3, size=40)
    R[:10, 2] = rng.uniform(1e-3, 2.5 * h, size=10)          # near the bottom wall
    R[10:20, 2] = L - rng.uniform(1e-3, 2.5 * h, size=10)    # near the top wall
    W = walls.all_weights(R, n, h)
    lam = rng.standard_normal((40, d))
    v = rng.standard_normal((d,) + (n,) * d)
    v[d - 1][0] = 0.0
    Sl = ib.spread(lam, R, n, h, W)
    Jv = ib.interp(v, R, h, W)
    assert abs((Jv * lam).sum() - h ** d * (v * Sl).sum()) < 1e-12 * abs((Jv * lam).sum())
    assert np.abs(Sl[d - 1][0]).max() == 0.0               # nothing spread onto the wall faces
    # away from the walls the taps are the periodic ones
    far = (R[:, 2] > 2.5 * h) & (R[:, 2] < L - 2.5 * h)
    Wp = ib.all_weights(R[far], n, h)
    Wf = walls.all_weights(R[far], n, h)
    for a in range(d):
        assert np.array_equal(Wp[a][0], Wf[a][0]) and np.abs(Wp[a][1] - Wf[a][1]).max() == 0.0
    # a marker on a wall interpolates zero velocity from any field (odd mirror)
    for zw in (1e-13, L - 1e-13):
        Rw = np.array([[0.37, 0.61, zw]])
        assert np.abs(ib.interp(v, Rw, h, walls.all_weights(Rw, n, h))).max() < 1e-11


def _dense_solve(prob):
    """The constrained system assembled column by column and solved by LAPACK
    (wall faces removed from the unknowns, mean(pi) = 0 bordered)."""
    sysm = walls.System(prob.dim, prob.n, prob.h, 0.0, prob.eta, prob.R)
    d, n = prob.dim, prob.n
    C = n ** d
    N = prob.R.shape[0]
    wall = np.zeros((d,) + (n,) * d, dtype=bool)
    wall[d - 1][0] = True
    keep = np.flatnonzero(~wall.reshape(-1))
    nv = keep.size
    tot = nv + C + d * N

    def apply(x):
        vf = np.zeros(d * C)
        vf[keep] = x[:nv]
        v = vf.reshape((d,) + (n,) * d)
        p = x[nv:nv + C].reshape((n,) * d)
        lam = x[nv + C:].reshape(N, d)
        rm, rc = walls.stokes_apply(v, p, 0.0, prob.eta, prob.h)
        rm = (rm - sysm.spread(lam)).reshape(-1)[keep]
        return np.concatenate([rm, rc.reshape(-1), -sysm.interp(v).reshape(-1)])

    K = np.zeros((tot + 1, tot + 1))
    e = np.zeros(tot)
    for j in range(tot):
        e[j] = 1.0
        K[:tot, j] = apply(e)
        e[j] = 0.0
    K[nv:nv + C, tot] = 1.0
    K[tot, nv:nv + C] = 1.0
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    rhs = np.zeros(tot + 1)
    rhs[nv + C:tot] = -V.reshape(-1)          # -J v = W = -V
    x = np.linalg.solve(K, rhs)
    vf = np.zeros(d * C)
    vf[keep] = x[:nv]
    return vf.reshape((d,) + (n,) * d), x[nv:nv + C].reshape((n,) * d), x[nv + C:tot].reshape(N, d)


@pytest.mark.parametrize("d,n,nb", [(2, 16, 2), (3, 8, 1)])
def test_constrained_solve_matches_dense(d, n, nb):
    prob = slit_problem(seed=3, dim=d, n=n, nbodies=nb, radius_h=1.5 if d == 3 else 2.5, wall_gap_h=0.5,
                        gap_h=1.0)
    sol = walls.solve_problem(prob)
    v, p, lam = _dense_solve(prob)
    assert np.abs(sol.v - v).max() < 1e-9 * np.abs(v).max()
    assert np.abs(sol.p - p).max() < 1e-9 * np.abs(p).max()
    assert np.abs(sol.lam - lam).max() < 1e-9 * np.abs(lam).max()


def test_mirror_symmetry_and_wall_mobility():
    """A shell at height H and one at L - H moving along the walls feel the
    same drag; a marker's self-mobility falls toward a wall, along and across
    it, and stays below the periodic box's."""
    a = walls.solve_problem(slit_shell(16, 0, height=0.3))
    b = walls.solve_problem(slit_shell(16, 0, height=0.7))
    assert abs(a.F[0, 0] - b.F[0, 0]) < 1e-9 * abs(a.F[0, 0])
    assert abs(a.F[0, 2]) < 1e-9 * abs(a.F[0, 0]) or np.sign(a.F[0, 2]) == -np.sign(b.F[0, 2])
    n, h = 16, 1.0 / 16
    prev = None
    for z in (0.5, 0.3, 0.2, 0.12, 0.07, 0.03):
        sysm = walls.System(3, n, h, 0.0, 1.0, np.array([[0.41, 0.53, z]]))
        M = sysm.mobility_dense()
        cur = (M[0, 0], M[2, 2])
        if prev is not None:
            assert cur[0] < prev[0] and cur[1] < prev[1]
        prev = cur


@pytest.mark.parametrize("kind", [walls.CELL_DIR, walls.FACE_DIR, walls.CELL_NEU])
@pytest.mark.parametrize("d,n", [(2, 32), (3, 16)])
def test_vcycle_with_walls_converges_to_exact(kind, d, n):
    """Iterating x += V(b - A x) reaches the dense solution of the boundary
    operator, at a rate typical of multigrid (the cycle's restriction,
    prolongation and boundary rules are consistent with the operator)."""
    rng = np.random.default_rng(5)
    b = rng.standard_normal((n,) * d)
    if kind == walls.FACE_DIR:
        b[0] = 0.0
    c0, c1 = (0.0, -1.0) if kind == walls.CELL_NEU else (0.0, 3.0)
    if kind == walls.CELL_NEU:
        b -= b.mean()
    C = n ** d
    A = np.zeros((C, C))
    for j in range(C):
        e = np.zeros(C)
        e[j] = 1
        A[:, j] = walls.apply_op(e.reshape((n,) * d), c0, c1, kind).reshape(-1)
    # the operator of the cycle is c0 - c1 L with the walls' Laplacian
    x = rng.standard_normal((n,) * d)
    if kind == walls.FACE_DIR:
        x[0] = 0
    assert np.abs(walls.apply_op(x, c0, c1, kind) - (c0 * x - c1 * walls.lap(x, kind))).max() < 1e-12
    if kind == walls.FACE_DIR:
        keep = np.ones((n,) * d, dtype=bool)
        keep[0] = False
        keep = keep.reshape(-1)
        ex = np.zeros(C)
        ex[keep] = np.linalg.solve(A[np.ix_(keep, keep)], b.reshape(-1)[keep])
    elif kind == walls.CELL_NEU:
        ex = np.linalg.lstsq(A, b.reshape(-1), rcond=None)[0]
        ex -= ex.mean()
    else:
        ex = np.linalg.solve(A, b.reshape(-1))
    ex = ex.reshape((n,) * d)
    x = np.zeros_like(b)
    errs = []
    for _ in range(30):
        r = b - walls.apply_op(x, c0, c1, kind)
        x = x + walls.vcycle(r, c0, c1, kind)
        if kind == walls.CELL_NEU:
            x -= x.mean()
        errs.append(np.abs(x - ex).max())
    rate = (errs[11] / errs[1]) ** (1.0 / 10)
    assert errs[-1] < 1e-8 * np.abs(ex).max()
    assert rate < 0.45, rate          # about 0.22 in 2D and 0.38 in 3D for every kind


def test_ps_inv_projects():
    """P_S^-1 with the walls keeps the normal component's wall faces at 0 and
    removes most of the divergence defect (one Neumann V-cycle for the
    pressure: the defect left is that cycle's residual)."""
    d, n, h = 3, 16, 1.0 / 16
    rng = np.random.default_rng(6)
    g = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    hp -= hp.mean()
    for c0 in (0.0, 50.0):
        v0 = np.stack([walls.vcycle(g[a], c0, 1.0 / (h * h), walls.kinds(d)[a]) for a in range(d)])
        before = np.abs(-walls.div(v0, h) - hp).max()
        v, pi = walls.ps_inv(g, hp, c0, 1.0, h)
        after = np.abs(-walls.div(v, h) - hp).max()
        assert after < 0.5 * before
        assert np.abs(v[d - 1][0]).max() == 0.0


def test_faxen_series_limits_and_inverse():
    """Faxen's slit series: Stokes' law far from the walls, the drag grows
    with R at fixed H, a sphere at the quarter plane (nearer wall) is less
    mobile than one of the same size at the midplane of the same slit, and
    radius_from_slit_drag inverts the drag."""
    d = 1.0
    for where, H in (("half", d / 2), ("quarter", d / 4)):
        R = 1e-7
        assert abs(walls.faxen_mobility(R, H, where) * 6 * math.pi * R - 1) < 1e-5
        Rs = np.linspace(0.01, 0.3, 30) * H
        drag = [1 / walls.faxen_mobility(r, H, where) for r in Rs]
        assert np.all(np.diff(drag) > 0)
        for r in (0.05 * H, 0.2 * H, 0.4 * H):
            F = 1 / walls.faxen_mobility(r, H, where)
            assert abs(walls.radius_from_slit_drag(F, 1.0, H, where) - r) < 1e-12
    for R in (0.02, 0.06, 0.1):
        assert walls.faxen_mobility(R, d / 4, "quarter") < walls.faxen_mobility(R, d / 2, "half")


def _mirror(v):
    """Mirror image of a face field about the midplane between the walls:
    tangential rows k -> n-1-k, normal faces k -> n-k with the sign reversed
    (face 0 is its own image, the walls swapping)."""
    d, n = v.shape[0], v.shape[1]
    out = v.copy()
    for a in range(d - 1):
        out[a] = v[a][::-1]
    out[d - 1] = 0.0
    out[d - 1][1:] = -v[d - 1][1:][::-1]
    return out


@pytest.mark.parametrize("d,n", [(2, 16), (3, 8)])
def test_wall_advection_interior_rows_and_mirror(d, n):
    """Away from the tangential components' boundary rows the wall advection
    equals the periodic one (the normal component's wall faces hold 0 in
    both), and it commutes with the mirror image about the midplane."""
    from oracle import navier
    h = 1.0 / n
    rng = np.random.default_rng(8)
    v = rng.standard_normal((d,) + (n,) * d)
    v[d - 1][0] = 0.0
    Nw = walls.advection(v, h)
    Np = navier.advection(v, h)
    for a in range(d - 1):
        assert np.abs(Nw[a][1:-1] - Np[a][1:-1]).max() < 1e-13
        assert np.abs(Nw[a][[0, -1]] - Np[a][[0, -1]]).max() > 1e-3
    assert np.abs(Nw[d - 1][1:] - Np[d - 1][1:]).max() < 1e-13 and np.abs(Nw[d - 1][0]).max() == 0.0
    assert np.abs(walls.advection(_mirror(v), h) - _mirror(Nw)).max() < 1e-12


def test_wall_advection_converges_to_the_continuum():
    """A no-slip, divergence-free 2D flow between the walls (stream function
    sin(2 pi x) z^2 (1 - z)^2): the discrete advection term converges at
    second order to (u . grad) u, the boundary rows included."""
    def ux(x, z):
        return np.sin(2 * np.pi * x) * 2 * z * (1 - z) * (1 - 2 * z)

    def uz(x, z):
        return -2 * np.pi * np.cos(2 * np.pi * x) * z ** 2 * (1 - z) ** 2

    e = 1e-6

    def conv(f, x, z):
        return ux(x, z) * (f(x + e, z) - f(x - e, z)) / (2 * e) + uz(x, z) * (f(x, z + e) - f(x, z - e)) / (2 * e)

    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        i = np.arange(n)
        Zx, Xx = np.meshgrid((i + 0.5) * h, i * h, indexing="ij")
        Zz, Xz = np.meshgrid(i * h, (i + 0.5) * h, indexing="ij")
        v = np.stack([ux(Xx, Zx), uz(Xz, Zz)])
        ex = np.stack([conv(ux, Xx, Zx), conv(uz, Xz, Zz)])
        ex[1][0] = 0.0
        errs.append(np.abs(walls.advection(v, h) - ex).max())
    assert np.log2(errs[0] / errs[1]) > 1.8 and np.log2(errs[1] / errs[2]) > 1.8, errs
