"""Pins of the oracle's exact constrained solve (Secs. 3.2-3.4, 7.3, 7.5).

* the Fourier/Schur route equals a dense LAPACK solve of the stencil system
  with gauge rows (two independent constructions of the same linear algebra);
* the mobility M = J L^-1 S is symmetric positive semi-definite (Sec. 3.3);
* the solution satisfies every block of the system, <v> = 0 for periodic
  steady Stokes (Sec. 3.4), D v = 0 and J v = V;
* a single four-point marker has hydrodynamic radius a ~ 1.25 h through the
  periodic drag law (Sec. 4.1 footnote, eq. drag_periodic);
* drag of a disk and of a sphere converges at first order towards the
  geometric radius, R_h -> R_g (Sec. 7.3 and eq. drag_periodic_2D).
"""
import math

import numpy as np
import pytest

from oracle import constrained, dense, hasimoto, ib
from synthetic import disk_ring, fibonacci_sphere, small_problem


def _rhs(prob, rng, with_fluid_rhs):
    d, n = prob.dim, prob.n
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    if not with_fluid_rhs:
        return None, None, -V
    g = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    hp -= hp.mean()
    if prob.steady:
        g -= g.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    return g, hp, -V


CASES = [
    dict(dim=2, n=16, radius_h=3.0),
    dict(dim=2, n=16, radius_h=3.0, rho=1.0, dt=0.02),
    dict(dim=3, n=8, radius_h=1.5),
    dict(dim=3, n=8, radius_h=1.5, rho=1.0, dt=0.05, eta=0.3),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("fluid_rhs", [False, True])
def test_fourier_schur_equals_dense(case, fluid_rhs, rng):
    prob = small_problem(3, **case)
    sysm = constrained.System.from_problem(prob)
    g, hp, W = _rhs(prob, rng, fluid_rhs)
    sol = constrained.solve(sysm, g, hp, W, prob.offsets, prob.centres)
    v, p, lam, mult = dense.solve(sysm, g, hp, W)
    p = p - p.mean()
    assert np.abs(mult).max() < 1e-9 * max(1.0, np.abs(lam).max())   # consistent RHS
    assert np.abs(sol.v - v).max() <= 1e-11 * np.abs(v).max()
    assert np.abs(sol.p - p).max() <= 1e-10 * np.abs(p).max()
    assert np.abs(sol.lam - lam).max() <= 1e-10 * np.abs(lam).max()


@pytest.mark.parametrize("case", CASES)
def test_solution_satisfies_system(case, rng):
    prob = small_problem(5, **case)
    sysm = constrained.System.from_problem(prob)
    g, hp, W = _rhs(prob, rng, True)
    sol = constrained.solve(sysm, g, hp, W, prob.offsets, prob.centres)
    rm, rc, rl = constrained.residual(sysm, sol.v, sol.p, sol.lam, g, hp, W)
    assert np.abs(rm).max() < 1e-9 * np.abs(g).max() * prob.n ** 2
    assert np.abs(rc).max() < 1e-10 * np.abs(hp).max() * prob.n
    assert np.abs(rl).max() < 1e-10 * np.abs(W).max()
    if prob.steady:
        assert np.abs(sol.v.reshape(prob.dim, -1).mean(axis=1)).max() < 1e-12


@pytest.mark.parametrize("d,n,rh", [(2, 32, 5.0), (3, 16, 2.5)])
@pytest.mark.parametrize("steady", [True, False])
def test_mobility_symmetric_psd(d, n, rh, steady):
    prob = small_problem(2, d, n, radius_h=rh, rho=0.0 if steady else 1.0,
                         dt=0.0 if steady else 0.5 / n, eta=1.0 if steady else 0.02)
    M = constrained.System.from_problem(prob).mobility_dense()
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev.min() > -1e-12 * ev.max()


def test_single_marker_hydrodynamic_radius():
    """Four-point kernel: a ~ 1.25 h from periodic drag (Sec. 4.1 footnote)."""
    n = 32
    rng = np.random.default_rng(11)
    radii = []
    for _ in range(4):
        R = rng.uniform(0, 1, size=(1, 3))
        M = constrained.System(3, n, 1.0 / n, 0.0, 1.0, R).mobility_dense()
        F = np.linalg.solve(M, np.array([1.0, 0.0, 0.0]))[0]
        radii.append(hasimoto.radius3d(F, 1.0) * n)
    assert abs(np.mean(radii) - 1.25) < 0.03
    assert np.std(radii) < 0.03  # near translational invariance of the kernel


def _drag_disk(n, R):
    h = 1.0 / n
    nm = int(round(math.pi * R / h))
    pts = disk_ring(nm, R, [0.5, 0.5], 0.1)
    sysm = constrained.System(2, n, h, 0.0, 1.0, pts)
    W = -np.tile([1.0, 0.0], (nm, 1))
    sol = constrained.solve(sysm, None, None, W, np.array([0, nm]), np.array([[0.5, 0.5]]))
    return sol.F[0, 0]


def test_disk_drag_first_order():
    """Hydrodynamic radius of a disk converges to R_g at first order (eq. drag_periodic_2D)."""
    R = 0.125
    ex = []
    for n in (64, 128, 256):
        F = _drag_disk(n, R)
        assert F > 0  # Lambda is the force on the fluid, along the motion
        ex.append(hasimoto.radius2d(F, 1.0) / R - 1.0)
    assert all(e > 0 for e in ex)
    r1, r2 = ex[0] / ex[1], ex[1] / ex[2]
    assert 1.6 < r1 < 2.6 and 1.6 < r2 < 2.6, ex


@pytest.mark.slow
def test_sphere_drag_first_order():
    """A sphere shell at ~2h spacing: R_h/R_g -> 1 at first order (Sec. 7.3)."""
    R = 0.125
    ex = []
    for n in (32, 64):
        h = 1.0 / n
        nm = int(round(math.pi * (R / h) ** 2))
        pts = fibonacci_sphere(nm, R, [0.5, 0.5, 0.5])
        sysm = constrained.System(3, n, h, 0.0, 1.0, pts)
        W = -np.tile([1.0, 0.0, 0.0], (nm, 1))
        sol = constrained.solve(sysm, None, None, W, np.array([0, nm]), np.array([[0.5] * 3]))
        ex.append(hasimoto.radius3d(sol.F[0, 0], 1.0) / R - 1.0)
    assert ex[0] > ex[1] > 0
    assert 1.6 < ex[0] / ex[1] < 2.6, ex


def test_hasimoto_limits():
    # dilute limits: Stokes drag in 3D, and the inverse functions round-trip
    assert hasimoto.drag3d(1e-6, 1.0) / (6 * math.pi * 1e-6) == pytest.approx(1.0, rel=1e-5)
    for rh in (0.05, 0.1, 0.2):
        assert hasimoto.radius3d(hasimoto.drag3d(rh, 1.0), 1.0) == pytest.approx(rh, rel=1e-12)
        assert hasimoto.radius2d(hasimoto.drag2d(rh, 1.0), 1.0) == pytest.approx(rh, rel=1e-12)
