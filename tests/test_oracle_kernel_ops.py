"""Pins of the oracle's kernel, MAC operators, J/S and Fourier solver.

Each check is fixed by mathematics or by the paper, not by re-typing the
oracle's formulas: Peskin's defining moment conditions for the kernel,
second-order accuracy of the staggered stencils on analytic fields, D = -G^T
(Sec. 3.2), the adjointness J = h^d S^T (Sec. 3.1), and the Fourier solve
satisfying the stencil equations it claims to invert (Sec. 3.3).
"""
import numpy as np
import pytest

from oracle import grid, ib, kernel, stokes


# ---------------------------------------------------------------- kernel
def test_phi_integer_values():
    # values at integer offsets implied by the even/odd partition with phi(0) max
    assert kernel.phi(0.0) == pytest.approx(0.5, abs=1e-15)
    assert kernel.phi(1.0) == pytest.approx(0.25, abs=1e-15)
    assert kernel.phi(-1.0) == pytest.approx(0.25, abs=1e-15)
    assert kernel.phi(2.0) == 0.0 and kernel.phi(-2.5) == 0.0


def test_phi_moment_conditions(rng):
    r = rng.uniform(-3.0, 3.0, size=200)
    j = np.arange(-6, 7)
    w = kernel.phi(r[:, None] - j[None, :])
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)                  # partition of unity
    even = (j % 2 == 0)
    assert np.allclose(w[:, even].sum(axis=1), 0.5, atol=1e-14)          # even/odd split
    assert np.allclose(((r[:, None] - j) * w).sum(axis=1), 0.0, atol=1e-14)  # first moment
    assert np.allclose((w ** 2).sum(axis=1), 3.0 / 8.0, atol=1e-14)      # sum of squares
    assert (np.count_nonzero(w > 0, axis=1) <= 4).all()


def test_phi_continuous_at_one():
    eps = 1e-9
    assert abs(kernel.phi(1.0 - eps) - kernel.phi(1.0 + eps)) < 1e-8


# ---------------------------------------------------------------- MAC operators
def _dense(op, nin, nout):
    M = np.zeros((nout, nin))
    e = np.zeros(nin)
    for j in range(nin):
        e[j] = 1.0
        M[:, j] = op(e)
        e[j] = 0.0
    return M


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_div_is_minus_grad_transpose(d, n):
    h = 0.3
    C = n ** d
    G = _dense(lambda x: grid.grad(x.reshape((n,) * d), h).reshape(-1), C, d * C)
    D = _dense(lambda x: grid.div(x.reshape((d,) + (n,) * d), h).reshape(-1), d * C, C)
    assert np.array_equal(D, -G.T)


def _coords(n, d, h, stagger_axis=None):
    """Coordinates (x, y[, z]) of cell centres or of faces normal to ``stagger_axis``."""
    c = [(np.arange(n) + 0.5) * h for _ in range(d)]
    if stagger_axis is not None:
        c[stagger_axis] = np.arange(n) * h
    mesh = np.meshgrid(*c[::-1], indexing="ij")  # array axes (z, y, x)
    return mesh[::-1]  # x first


@pytest.mark.parametrize("d", [2, 3])
def test_stencils_second_order(d):
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        X = _coords(n, d, h)
        p = np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1])
        gerr = 0.0
        for a in range(d):
            F = _coords(n, d, h, stagger_axis=a)
            if a == 0:
                exact = 2 * np.pi * np.cos(2 * np.pi * F[0]) * np.cos(2 * np.pi * F[1])
            elif a == 1:
                exact = -2 * np.pi * np.sin(2 * np.pi * F[0]) * np.sin(2 * np.pi * F[1])
            else:
                exact = np.zeros_like(F[0])
            gerr = max(gerr, np.abs(grid.grad(p, h)[a] - exact).max())
        # divergence of a face field v^a = sin(2 pi x_a) evaluated on its faces
        v = np.stack([np.sin(2 * np.pi * _coords(n, d, h, stagger_axis=a)[a]) for a in range(d)])
        dex = sum(2 * np.pi * np.cos(2 * np.pi * X[a]) for a in range(d))
        derr = np.abs(grid.div(v, h) - dex).max()
        lex = -8 * np.pi ** 2 * p
        lerr = np.abs(grid.lap(p) / h ** 2 - lex).max()
        errs.append((gerr, derr, lerr))
    for k in range(3):
        ratio = errs[0][k] / errs[1][k]
        assert 3.6 < ratio < 4.4, (k, errs)


# ---------------------------------------------------------------- J and S
@pytest.mark.parametrize("d,n", [(2, 16), (3, 8)])
def test_adjointness(d, n, rng):
    h = 1.0 / n
    R = rng.uniform(0.0, 1.0, size=(7, d))
    v = rng.standard_normal((d,) + (n,) * d)
    F = rng.standard_normal((7, d))
    lhs = (ib.interp(v, R, h) * F).sum()
    rhs = h ** d * (v * ib.spread(F, R, n, h)).sum()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("d,n", [(2, 16), (3, 8)])
def test_spread_conserves_force(d, n, rng):
    h = 1.0 / n
    R = rng.uniform(0.0, 1.0, size=(5, d))
    F = rng.standard_normal((5, d))
    f = ib.spread(F, R, n, h)
    tot = h ** d * f.reshape(d, -1).sum(axis=1)
    assert np.allclose(tot, F.sum(axis=0), atol=1e-13)
    fp = ib.spread_periodic_steady(F, R, n, h)
    assert np.allclose(fp.reshape(d, -1).sum(axis=1), 0.0, atol=1e-10)


@pytest.mark.parametrize("d", [2, 3])
def test_interp_reproduces_linear_fields(d, rng):
    """The zero first moment makes J exact for linear fields; this pins the face offsets."""
    n = 32
    h = 1.0 / n
    R = rng.uniform(0.35, 0.65, size=(6, d))
    for a in range(d):
        for b in range(d):
            v = np.zeros((d,) + (n,) * d)
            v[a] = 3.0 + 2.0 * _coords(n, d, h, stagger_axis=a)[b]
            got = ib.interp(v, R, h)[:, a]
            assert np.allclose(got, 3.0 + 2.0 * R[:, b], atol=1e-13)


def test_rigid_velocities_and_sums(rng):
    R = rng.uniform(0.2, 0.8, size=(6, 3))
    offsets = np.array([0, 6])
    X = np.array([[0.5, 0.5, 0.5]])
    U = np.array([[0.1, -0.2, 0.3]])
    Om = np.array([[0.4, 0.5, -0.6]])
    V = ib.marker_velocities(R, offsets, X, U, Om, 1.0)
    # relative velocities of a rigid body are Omega x relative positions
    assert np.allclose(V[1] - V[0], np.cross(Om[0], R[1] - R[0]), atol=1e-15)
    lam = rng.standard_normal((6, 3))
    F, T = ib.body_force_torque(lam, R, offsets, X, 1.0)
    assert np.allclose(F[0], lam.sum(axis=0))
    assert np.allclose(T[0], sum(np.cross(R[i] - X[0], lam[i]) for i in range(6)))
    # 2D: a pure rotation about the centre is perpendicular to the radius
    R2 = rng.uniform(0.3, 0.7, size=(4, 2))
    V2 = ib.marker_velocities(R2, np.array([0, 4]), np.array([[0.5, 0.5]]), np.zeros((1, 2)),
                              np.array([[2.0]]), 1.0)
    assert np.allclose((V2 * (R2 - 0.5)).sum(axis=1), 0.0, atol=1e-15)


# ---------------------------------------------------------------- Fourier solve
@pytest.mark.parametrize("d,n,c0", [(2, 16, 0.0), (2, 16, 50.0), (3, 8, 0.0), (3, 8, 20.0)])
def test_fourier_solve_satisfies_stencils(d, n, c0, rng):
    h, eta = 1.0 / n, 0.7
    f = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    hp -= hp.mean()
    if c0 == 0.0:
        f -= f.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    v, p = stokes.solve(f, hp, c0, eta, h, d)
    rm, rc = grid.stokes_apply(v, p, c0, eta, h)
    scale = np.abs(f).max()
    assert np.abs(rm - f).max() < 1e-11 * scale * n * n
    assert np.abs(rc - hp).max() < 1e-11 * scale * n
    assert abs(p.mean()) < 1e-12 * np.abs(p).max()
    if c0 == 0.0:
        assert np.abs(v.reshape(d, -1).mean(axis=1)).max() < 1e-13 * np.abs(v).max()


@pytest.mark.parametrize("d", [2, 3])
def test_helmholtz_solve(d, rng):
    n = 8
    b = rng.standard_normal((n,) * d)
    for c0, c1 in ((0.0, 1.3), (2.0, 0.5)):
        bb = b - b.mean() if c0 == 0.0 else b
        x = stokes.helmholtz_solve(bb, c0, c1)
        assert np.allclose(c0 * x - c1 * grid.lap(x), bb, atol=1e-12)
