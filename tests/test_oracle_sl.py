"""Pins of the oracle's semi-Lagrangian advection (the transport reading of the
advection step, Sec. 3 with Sec. 7.6's unsteady runs).

The transport has no closed form to match, so it is pinned by what the
mathematics fixes: multilinear interpolation is exact for integer shifts and
reproduces multilinear functions; it is a convex combination (a maximum
principle); its face velocity is the one of the centred advective form
(itself pinned by the Taylor-Green convergence); for small steps the term
tends to the first-order upwind difference, and on a smooth field it
converges to (u.grad)u at first order for CFL numbers below and above one;
between the walls it equals the periodic transport of the mirror-extended
field on a channel of twice the height (the definition of the extension E).
"""
import numpy as np
import pytest

from oracle import grid, ib, navier, walls
from synthetic import slit_problem, small_problem


def _tg(n):
    """Taylor-Green field on the 2D MAC faces and its (u.grad)u."""
    h = 1.0 / n
    x = np.arange(n) * h
    v = np.zeros((2, n, n))
    ex = np.zeros((2, n, n))
    # array axes (y, x); v^x at (i h, (j + 1/2) h), v^y at ((i + 1/2) h, j h)
    X, Y = np.meshgrid(x, x + h / 2)
    v[0] = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    ex[0] = np.pi * np.sin(4 * np.pi * X)
    X, Y = np.meshgrid(x + h / 2, x)
    v[1] = -np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    ex[1] = np.pi * np.sin(4 * np.pi * Y)
    return v, ex, h


def test_interp_integer_shift_is_a_roll():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((6, 8, 10))
    idx = np.indices(q.shape).astype(np.float64)
    off = (2, -1, 13)
    s = [idx[ax] + off[ax] for ax in range(3)]
    out = navier.interp_lattice(q, s)
    assert np.array_equal(out, np.roll(q, [-o for o in off], axis=(0, 1, 2)))


def test_interp_reproduces_multilinear_functions():
    rng = np.random.default_rng(1)
    n = 12
    i, j = np.indices((n, n)).astype(np.float64)
    c = rng.standard_normal(4)
    q = c[0] + c[1] * i + c[2] * j + c[3] * i * j
    # points whose cell lies inside the lattice (no wrap)
    si = rng.uniform(0, n - 1, (n, n))
    sj = rng.uniform(0, n - 1, (n, n))
    out = navier.interp_lattice(q, [si, sj])
    ex = c[0] + c[1] * si + c[2] * sj + c[3] * si * sj
    assert np.abs(out - ex).max() < 1e-12


def test_departure_values_obey_the_maximum_principle():
    rng = np.random.default_rng(2)
    n = 8
    v = rng.standard_normal((3, n, n, n))
    for cfl in (0.4, 3.7):
        vd = navier.departure_values(v, 1.0 / n, cfl / n)
        for a in range(3):
            assert vd[a].max() <= v[a].max() + 1e-15
            assert vd[a].min() >= v[a].min() - 1e-15


def test_uniform_flow_has_no_advection():
    v = np.ones((3, 8, 8, 8)) * np.array([0.3, -0.2, 0.5])[:, None, None, None]
    assert np.abs(navier.advection_sl(v, 0.1, 0.37)).max() < 1e-15


def test_face_velocity_is_the_centred_forms():
    """The centred advective form is sum_b ubar^b times the centred difference:
    the transport backtracks along the same face velocity."""
    rng = np.random.default_rng(3)
    n, h = 8, 0.125
    v = rng.standard_normal((3, n, n, n))
    N = navier.advection(v, h)
    for a in range(3):
        u = navier.face_velocity(v, a)
        acc = sum(u[b] * (grid.shift(v[a], 1, 2 - b) - grid.shift(v[a], -1, 2 - b)) / (2 * h)
                  for b in range(3))
        assert np.abs(acc - N[a]).max() < 1e-12


def test_small_steps_tend_to_first_order_upwind():
    rng = np.random.default_rng(4)
    n, h = 8, 0.125
    v = rng.standard_normal((2, n, n))
    up = np.zeros_like(v)
    for a in range(2):
        u = navier.face_velocity(v, a)
        for b in range(2):
            ax = 1 - b
            back = (v[a] - grid.shift(v[a], -1, ax)) / h
            fwd = (grid.shift(v[a], 1, ax) - v[a]) / h
            up[a] += u[b] * np.where(u[b] > 0, back, fwd)
    errs = [np.abs(navier.advection_sl(v, h, dt) - up).max() for dt in (1e-3 * h, 1e-4 * h)]
    assert errs[1] < 1e-3 * np.abs(up).max()
    assert 8 < errs[0] / errs[1] < 12, errs     # the bilinear cross term is O(dt)


@pytest.mark.parametrize("cfl", [0.5, 1.7])
def test_taylor_green_first_order(cfl):
    errs = []
    for n in (16, 32, 64):
        v, ex, h = _tg(n)
        errs.append(np.abs(navier.advection_sl(v, h, cfl * h) - ex).max())
    for k in range(2):
        assert 1.8 < errs[k] / errs[k + 1] < 2.2, errs
    assert errs[-1] < 0.6


@pytest.mark.parametrize("d,n", [(2, 8), (3, 6)])
@pytest.mark.parametrize("cfl", [0.3, 2.5])
def test_walls_transport_is_the_mirror_extended_periodic_one(d, n, cfl):
    """Reflect the channel across its top wall with E's signs (tangential
    components odd about the wall, normal faces odd about the wall faces, the
    wall faces 0): periodic transport on the 2n-high channel restricted to
    the lower half equals the transport between the walls."""
    rng = np.random.default_rng(5)
    v = rng.standard_normal((d,) + (n,) * d)
    v[d - 1][0] = 0.0
    h = 1.0 / n
    ext = [np.concatenate([v[a], -np.flip(v[a], 0)], 0) for a in range(d - 1)]
    ext.append(np.concatenate([v[d - 1], np.zeros((1,) + (n,) * (d - 1)), -np.flip(v[d - 1][1:], 0)], 0))
    ref = navier.departure_values(np.stack(ext), h, cfl * h)[:, :n]
    got = walls.departure_values(v, h, cfl * h)
    assert np.abs(got - ref).max() < 1e-14
    assert np.abs(got[d - 1][0]).max() == 0.0
    N = walls.advection_sl(v, h, cfl * h)
    assert np.abs(N[d - 1][0]).max() == 0.0


def test_sl_steps_meet_constraints():
    prob = small_problem(9, 3, 8, radius_h=1.5, rho=1.0, dt=0.5 / 8, eta=0.05, nsteps=2, rotate=False)
    sols = navier.run(prob, 2, scheme="sl")
    R = prob.R.copy()
    b = ib.body_of(prob.offsets)
    for s in sols:
        R = np.mod(R + prob.dt * prob.U[b], prob.L)
        assert np.allclose(ib.interp(s.v, R, prob.h), prob.U[b], atol=1e-10)
        assert np.abs(grid.div(s.v, prob.h)).max() < 1e-9


def test_sl_steps_between_walls_meet_constraints():
    prob = slit_problem(5, dim=2, n=16, nbodies=1, radius_h=3.0, wall_gap_h=2.0, rotate=False,
                        rho=1.0, dt=0.5 / 16, eta=0.05)
    sols = walls.run(prob, 2, scheme="sl")
    for s in sols:
        assert np.abs(s.v[1][0]).max() == 0.0
        assert np.abs(walls.div(s.v, prob.h)).max() < 1e-9
