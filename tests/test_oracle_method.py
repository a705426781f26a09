"""Pins of the oracle's approximations: M~ (Sec. 4), the V-cycle and P_S^-1
(Sec. 5.2), the Schur preconditioner (Sec. 5.1) and the advection term.

The approximations have no exact value to match, so each is pinned by what the
paper or the mathematics fixes about it: limits and continuity of the analytic
mobilities, SPD of the RPY tensor, rotation covariance; convergence of repeated
V-cycles to the exact periodic solve; exactness of P_S^-1 and of the full Schur
preconditioner when their sub-solves are exact; second-order accuracy of the
advection stencil on a Taylor-Green field.
"""
import math

import numpy as np
import pytest

from oracle import constrained, grid, ib, mobility, multigrid, navier, precond, stokes
from synthetic import fibonacci_sphere, small_problem


# ---------------------------------------------------------------- mobility
def test_rpy_limits_and_continuity():
    a, eta = 0.3, 1.7
    f0, g0 = mobility.rpy(np.array(0.0), a, eta)
    assert float(f0) == pytest.approx(1.0 / (6 * math.pi * eta * a), rel=1e-15)
    assert float(g0) == 0.0
    lo = mobility.rpy(np.array(2 * a * (1 - 1e-12)), a, eta)
    hi = mobility.rpy(np.array(2 * a * (1 + 1e-12)), a, eta)
    assert float(lo[0]) == pytest.approx(float(hi[0]), rel=1e-9)
    assert float(lo[1]) == pytest.approx(float(hi[1]), rel=1e-9)
    r = 1e4 * a
    f, g = mobility.rpy(np.array(r), a, eta)
    oseen = 1.0 / (8 * math.pi * eta * r)
    assert float(f) == pytest.approx(oseen, rel=1e-6) and float(g) == pytest.approx(oseen, rel=1e-6)


def test_rpy_spd_for_arbitrary_configurations(rng):
    """The RPY tensor gives an SPD mobility for every configuration (Sec. 4.1)."""
    a = 1.0
    for trial in range(5):
        R = rng.uniform(0.0, 4.0, size=(40, 3))  # dense cloud with overlapping blobs
        f, g = mobility.rpy(np.sqrt(((R[:, None] - R[None]) ** 2).sum(-1)), a, 1.0)
        dr = R[:, None] - R[None]
        r = np.sqrt((dr ** 2).sum(-1))
        rh = np.where(r[..., None] > 0, dr / np.where(r > 0, r, 1)[..., None], 0)
        M = (f[..., None, None] * np.eye(3) + g[..., None, None] * rh[..., :, None] * rh[..., None, :])
        M = M.transpose(0, 2, 1, 3).reshape(120, 120)
        assert np.linalg.eigvalsh(M).min() > 0


def test_brinkmanlet_limits():
    eta, r = 0.8, 0.7
    f, g = mobility.brinkmanlet(np.array(r), 1e-5, eta)       # alpha -> 0: Stokeslet
    st = 1.0 / (8 * math.pi * eta * r)
    assert float(f) == pytest.approx(st, rel=1e-4) and float(g) == pytest.approx(st, rel=1e-4)
    alpha = 50.0
    f, g = mobility.brinkmanlet(np.array(r), alpha, eta)      # far field: dipole
    dip = 1.0 / (4 * math.pi * eta * alpha ** 2 * r ** 3)
    assert float(f) == pytest.approx(-dip, rel=1e-9) and float(g) == pytest.approx(3 * dip, rel=1e-9)


def test_inviscid_self_mobility_matches_exact_marker():
    """f_0(0) = ((d-1)/d)(dt/rho)/V_m with V_m = (8/3)^3 h^3 (eq. f_0_inviscid)."""
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(4)
    vals = []
    for _ in range(6):
        R = rng.uniform(0, 1, size=(1, 3))
        M = constrained.System(3, n, h, 1.0, 1e-12, R).mobility_dense()   # rho/dt = 1, eta ~ 0
        vals.append(np.trace(M) / 3.0)
    expect = mobility.self_inviscid(3, h, 1.0, 1.0)
    assert np.mean(vals) == pytest.approx(expect, rel=0.03)


def test_mobility_block_rotation_covariance(rng):
    R = fibonacci_sphere(30, 0.1, [0.5, 0.5, 0.5])
    p = mobility.params_for(3, 1.0 / 64, 1.0, 0.0, 1.0, 0.0)
    M = mobility.block(R, p)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Rr = (R - 0.5) @ q.T + 0.5
    Mr = mobility.block(Rr, p)
    Q = np.kron(np.eye(30), q)
    assert np.allclose(Mr, Q @ M @ Q.T, atol=1e-12 * np.abs(M).max())


def test_factor_block_shift_rule():
    M = np.array([[1.0, 2.0], [2.0, 1.0]])            # eigenvalues -1, 3
    L, s = mobility.factor_block(M, 1.0)
    assert s == mobility.SHIFTS[next(i for i, x in enumerate(mobility.SHIFTS) if x > 1.0)]
    assert np.allclose(L @ L.T, M + s * np.eye(2))
    L0, s0 = mobility.factor_block(np.eye(2) * 3.0, 1.0)
    assert s0 == 0.0


# ---------------------------------------------------------------- multigrid
@pytest.mark.parametrize("d,n", [(2, 32), (3, 16)])
@pytest.mark.parametrize("c0,c1", [(0.0, 1.0), (3.0, 0.7)])
def test_vcycle_iteration_converges_to_exact(d, n, c0, c1, rng):
    b = rng.standard_normal((n,) * d)
    if c0 == 0.0:
        b -= b.mean()
    xe = stokes.helmholtz_solve(b, c0, c1)
    x = np.zeros_like(b)
    prev = 1.0
    for it in range(5):
        x = x + multigrid.vcycle(b - multigrid.apply_op(x, c0, c1), c0, c1)
        if c0 == 0.0:
            x -= x.mean()
        err = np.linalg.norm(x - xe) / np.linalg.norm(xe)
        assert err < 0.2 * prev
        prev = err


def test_vcycle_restricted_inverse_mean_zero(rng):
    b = rng.standard_normal((16, 16, 16)) + 5.0
    x = multigrid.vcycle(b, 0.0, 1.0)
    assert abs(x.mean()) < 1e-13


def test_transfer_operators():
    e = np.random.default_rng(0).standard_normal((4, 4, 4))
    # prolongation preserves constants and the mean; restriction averages children
    assert np.allclose(multigrid.prolong(np.ones((4, 4))), 1.0)
    assert multigrid.prolong(e).mean() == pytest.approx(e.mean(), abs=1e-15)
    f = np.arange(64.0).reshape(8, 8)
    assert multigrid.restrict(f)[1, 2] == pytest.approx(f[2:4, 4:6].mean())
    # multilinear interpolation is exact for linear functions away from the wrap
    xc = (np.arange(8) + 0.5) * 2.0
    xf = (np.arange(16) + 0.5)
    lin = multigrid.prolong(np.broadcast_to(xc, (8, 8)).copy())
    assert np.allclose(lin[:, 2:-2], np.broadcast_to(xf, (16, 16))[:, 2:-2])


@pytest.mark.parametrize("d,n,c0", [(2, 16, 0.0), (2, 16, 40.0), (3, 8, 0.0), (3, 8, 30.0)])
def test_ps_inv_exact_subsolves_is_stokes_inverse(d, n, c0, rng):
    h, eta = 1.0 / n, 0.6
    g = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    hp -= hp.mean()
    if c0 == 0.0:
        g -= g.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    v, p = precond.ps_inv(g, hp, c0, eta, h, precond.MGParams(exact=True))
    ve, pe = stokes.solve(g, hp, c0, eta, h, d)
    p = p - p.mean()
    assert np.abs(v - ve).max() < 1e-11 * np.abs(ve).max()
    assert np.abs(p - pe).max() < 1e-10 * np.abs(pe).max()


@pytest.mark.parametrize("c0", [0.0, 30.0])
def test_inner_gmres_reduces_residual(c0, rng):
    d, n, h, eta = 3, 16, 1.0 / 16, 1.0
    g = rng.standard_normal((d,) + (n,) * d)
    if c0 == 0.0:
        g -= g.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    hp = np.zeros((n,) * d)
    res = []
    for ns in (1, 2, 4):
        v, p = precond.stokes_gmres(g, hp, c0, eta, h, ns)
        rm, rc = grid.stokes_apply(v, p, c0, eta, h)
        res.append(np.sqrt(((rm - g) ** 2).sum() + (rc ** 2).sum()))
    assert res[0] < np.linalg.norm(g) and res[1] < res[0] and res[2] < res[1]


@pytest.mark.parametrize("case", [dict(dim=2, n=16, radius_h=3.0),
                                  dict(dim=3, n=8, radius_h=1.5, rho=1.0, dt=0.05, eta=0.3)])
def test_full_schur_with_exact_parts_is_exact(case, rng):
    """With the true mobility and exact fluid solves, the full preconditioner inverts K."""
    prob = small_problem(7, **case)
    sysm = constrained.System.from_problem(prob)
    M = sysm.mobility_dense()
    mp = mobility.params_for(prob.dim, prob.h, prob.L, prob.rho, prob.eta, prob.dt)
    pc = precond.SchurPreconditioner(sysm, prob.offsets, [M], mp, ns=1, full=True,
                                     mg=precond.MGParams(exact=True))
    assert pc.shifts == [0.0]
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    d, n = prob.dim, prob.n
    g = rng.standard_normal((d,) + (n,) * d)
    if prob.steady:
        g -= g.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    hp = np.zeros((n,) * d)
    v, p, lam = pc.apply(g, hp, -V)
    ex = constrained.solve(sysm, g, hp, -V, prob.offsets, prob.centres)
    assert np.abs(v - ex.v).max() < 1e-10 * np.abs(ex.v).max()
    assert np.abs(lam - ex.lam).max() < 1e-9 * np.abs(ex.lam).max()


# ---------------------------------------------------------------- advection
def _face_coords(n, d, h, a):
    c = [(np.arange(n) + 0.5) * h for _ in range(d)]
    c[a] = np.arange(n) * h
    mesh = np.meshgrid(*c[::-1], indexing="ij")
    return mesh[::-1]


def test_advection_second_order_taylor_green():
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        v = np.zeros((2, n, n))
        X = _face_coords(n, 2, h, 0)
        v[0] = np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1])
        Y = _face_coords(n, 2, h, 1)
        v[1] = -np.cos(2 * np.pi * Y[0]) * np.sin(2 * np.pi * Y[1])
        N = navier.advection(v, h)
        # (v.grad)v for this field is (pi sin(4 pi x), pi sin(4 pi y))
        ex0 = np.pi * np.sin(4 * np.pi * X[0])
        ex1 = np.pi * np.sin(4 * np.pi * Y[1])
        errs.append(max(np.abs(N[0] - ex0).max(), np.abs(N[1] - ex1).max()))
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def test_advection_of_uniform_flow_is_zero():
    v = np.ones((3, 8, 8, 8)) * np.array([0.3, -0.2, 0.5])[:, None, None, None]
    assert np.abs(navier.advection(v, 0.1)).max() == 0.0


def test_navier_steps_meet_constraints():
    prob = small_problem(9, 3, 8, radius_h=1.5, rho=1.0, dt=0.5 / 8, eta=0.05, nsteps=2,
                         rotate=False)
    sols = navier.run(prob, 2)
    R = prob.R.copy()
    b = ib.body_of(prob.offsets)
    for s in sols:
        R = np.mod(R + prob.dt * prob.U[b], prob.L)
        Jv = ib.interp(s.v, R, prob.h)
        assert np.allclose(Jv, prob.U[b], atol=1e-10)
        assert np.abs(grid.div(s.v, prob.h)).max() < 1e-9
