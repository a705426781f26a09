"""GPU parity of the semi-Lagrangian advection (the transport reading of the
unsteady step's advection, Sec. 3) against ``oracle.navier`` and
``oracle.walls``, through the C ABI.

* the advection term N = (v - v_departure)/dt on random fields, periodic and
  between walls, 2D and 3D, at CFL numbers below and above one and at a few
  hundred cells of displacement (1e-13 relative);
* a non-finite velocity stays on the lattice (the displacement is clamped)
  and yields a non-finite term;
* three unsteady steps with moving bodies equal the oracle's exact
  trajectory (fp64 1e-8, mixed 1e-6), periodic and between walls;
* at a cell Reynolds number where the centred form with Adams-Bashforth 2
  grows without bound, the transport stays bounded.
"""
import numpy as np
import pytest

from oracle import navier, walls
from synthetic import slit_problem, small_problem

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dim,n", [(2, 32), (2, 128), (3, 16), (3, 32)])
@pytest.mark.parametrize("cfl", [0.4, 2.7, 300.0])
@pytest.mark.parametrize("wall", [0, 1])
def test_sl_advection_matches_oracle(dim, n, cfl, wall):
    from paper_1505_07865_amd import ibr
    print("sl advect", dim, n, cfl, wall, flush=True)
    h = 1.0 / n
    dt = cfl * h
    s = ibr.Solver(dim=dim, n=n, h=h, rho=1.0, dt=dt, walls=wall, advection=ibr.ADVECT_SL)
    u = np.random.default_rng(n + dim).standard_normal((dim,) + (n,) * dim)
    if wall:
        u[dim - 1][0] = 0.0
    N = s.advect(u)
    s.close()
    Ne = (walls if wall else navier).advection_sl(u, h, dt)
    assert _rel(N, Ne) < 1e-13, _rel(N, Ne)
    if wall:
        assert np.abs(N[dim - 1][0]).max() == 0.0


def test_sl_advection_nonfinite_stays_on_lattice():
    from paper_1505_07865_amd import ibr
    n = 16
    s = ibr.Solver(dim=3, n=n, h=1.0 / n, rho=1.0, dt=0.01, advection=ibr.ADVECT_SL)
    u = np.random.default_rng(0).standard_normal((3, n, n, n))
    u[0, 3, 4, 5] = np.nan
    u[1, 7, 2, 9] = np.inf
    N = s.advect(u)
    s.close()
    assert not np.isfinite(N[0, 3, 4, 5]) and not np.isfinite(N[1, 7, 2, 9])
    assert np.isfinite(N[2, 12, 12, 12])      # far from both


def test_sl_advect_needs_unsteady():
    from paper_1505_07865_amd import ibr
    s = ibr.Solver(dim=2, n=32, h=1.0 / 32, advection=ibr.ADVECT_SL)
    with pytest.raises(ibr.IbrError):
        s.advect(np.zeros((2, 32, 32)))
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sl_steps_match_oracle(precision):
    from paper_1505_07865_amd import ibr
    prob = small_problem(17, 3, 16, nbodies=2, radius_h=2.0, rho=1.0, dt=0.5 / 16, eta=0.002, nsteps=3,
                         rotate=False)
    fp64 = precision == "fp64"
    s = ibr.from_problem(prob, rtol=1e-11 if fp64 else 1e-9, precision=ibr.FP64 if fp64 else ibr.MIXED,
                         advection=ibr.ADVECT_SL)
    ex = navier.run(prob, 3, scheme="sl")
    tol = 1e-8 if fp64 else 1e-6
    for k in range(3):
        info = s.step()
        sol = s.solution()
        print("step", k, info["iters"], _rel(sol.u, ex[k].v), flush=True)
        assert _rel(sol.u, ex[k].v) < tol
        assert _rel(sol.F, ex[k].F) < tol
    s.close()


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_sl_steps_between_walls_match_oracle(dim, n):
    from paper_1505_07865_amd import ibr
    prob = slit_problem(5, dim=dim, n=n, nbodies=2, radius_h=2.5 if dim == 3 else 4.0, wall_gap_h=2.0,
                        gap_h=2.0, rotate=False, rho=1.0, dt=0.5 / n, eta=0.005)
    s = ibr.from_problem(prob, rtol=1e-10, advection=ibr.ADVECT_SL)
    ex = walls.run(prob, 3, scheme="sl")
    for k in range(3):
        s.step()
        sol = s.solution()
        assert _rel(sol.u, ex[k].v) < 1e-8, (k, _rel(sol.u, ex[k].v))
        assert _rel(sol.F, ex[k].F) < 1e-8, (k, _rel(sol.F, ex[k].F))
        assert np.abs(sol.u[dim - 1][0]).max() == 0.0
    s.close()


def test_sl_stays_bounded_where_centred_grows():
    """Two spheres crossing a 32^3 box at cell Reynolds number 40 (U h rho /
    eta with U = 1): the centred form's velocity grows by orders of magnitude
    within 30 steps, the transport's stays of the bodies' speed."""
    from paper_1505_07865_amd import ibr
    n = 32
    prob = small_problem(21, 3, n, nbodies=2, radius_h=3.0, rho=1.0, dt=0.9 / n, eta=1.0 / (40 * n),
                         nsteps=30, rotate=False)
    umax = {}
    for name, adv in (("centred", ibr.ADVECT_CENTRED), ("sl", ibr.ADVECT_SL)):
        s = ibr.from_problem(prob, rtol=1e-8, advection=adv)
        peak = 0.0
        for k in range(30):
            try:
                s.step()
            except ibr.IbrError:
                peak = np.inf
                break
            peak = max(peak, float(np.abs(s.solution().u).max()))
        s.close()
        umax[name] = peak
    speed = float(np.abs(prob.U).max())
    print("max|u|", umax, "body speed", speed, flush=True)
    assert umax["sl"] < 3 * speed
    assert umax["centred"] > 10 * umax["sl"]
