"""Pins of the concentric-spheres Stokes solution (``oracle.shells``).

The flow is defined by its boundary value problem, so it is checked against
that problem directly: no slip on both spheres, the Stokes equations
mu lap u = grad p and div u = 0 at interior points (central differences),
and the drag law of the paper's appendix, which also equals the traction
integrated over the inner sphere.
"""
import math

import numpy as np
import pytest

from oracle import shells


def _dirs(m, seed=0):
    v = np.random.default_rng(seed).standard_normal((m, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("a,b,V", [(1.0, 4.0, 1.0), (0.06, 0.241, -2.0), (0.3, 0.45, 0.5)])
def test_no_slip_on_both_spheres(a, b, V):
    e = np.array([0.6, -0.0, 0.8])
    c = np.array([0.2, 0.1, -0.3])
    D = _dirs(50)
    ua = shells.velocity(c + a * D, c, a, b, V, e)
    ub = shells.velocity(c + b * D, c, a, b, V, e)
    assert np.abs(ua).max() < 1e-12 * abs(V)
    assert np.abs(ub - V * e).max() < 1e-12 * abs(V)


@pytest.mark.parametrize("a,b", [(1.0, 4.0), (0.5, 0.8)])
def test_stokes_equations_between_spheres(a, b):
    mu, V = 1.7, 1.3
    e = np.array([0.0, 0.0, 1.0])
    c = np.zeros(3)
    h = 1e-4 * b
    rng = np.random.default_rng(3)
    for _ in range(12):
        x = c + rng.uniform(a + 0.1 * (b - a), b - 0.1 * (b - a)) * _dirs(1, rng.integers(1 << 30))[0]
        u = lambda y: shells.velocity(y, c, a, b, V, e)
        p = lambda y: shells.pressure(y, c, a, b, V, mu, e)
        lap = sum((u(x + h * q) - 2 * u(x) + u(x - h * q)) / h ** 2 for q in np.eye(3))
        gp = np.array([(p(x + h * q) - p(x - h * q)) / (2 * h) for q in np.eye(3)])
        div = sum((u(x + h * q)[i] - u(x - h * q)[i]) / (2 * h) for i, q in enumerate(np.eye(3)))
        scale = np.abs(gp).max() + np.abs(mu * lap).max()
        assert np.abs(mu * lap - gp).max() < 1e-5 * scale
        assert abs(div) < 1e-6 * abs(V) / (b - a)


@pytest.mark.parametrize("lam", [0.1, 0.25, 0.5, 0.8])
def test_drag_law_and_traction(lam):
    a, mu, V = 1.0, 1.0, 1.0
    b = a / lam
    F = shells.inner_force(a, b, V, mu)
    assert abs(F - 6 * math.pi * mu * a * V * shells.drag_factor(lam)) < 1e-10 * abs(F)
    assert abs(shells.lambda_from_drag(F, a, V, mu) - lam) < 1e-10
    # traction sigma n integrated over a sphere between the two (with no body
    # force, the stress is divergence-free, so every such sphere carries the
    # force on the inner one)
    e = np.array([1.0, 0.0, 0.0])
    c = np.zeros(3)
    m = 4000
    k = np.arange(m) + 0.5
    z = 1 - 2 * k / m
    phi = math.pi * (1 + 5 ** 0.5) * k
    n = np.stack([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z], axis=1)
    rq = a + 0.3 * (b - a)
    h = 1e-5 * a
    X = c + rq * n
    grad = np.stack([(shells.velocity(X + h * q, c, a, b, V, e) - shells.velocity(X - h * q, c, a, b, V, e))
                     / (2 * h) for q in np.eye(3)], axis=2)          # [m, i, j] = d u_i / d x_j
    p = shells.pressure(X, c, a, b, V, mu, e)
    sigma = -p[:, None, None] * np.eye(3) + mu * (grad + grad.transpose(0, 2, 1))
    force = (sigma @ n[:, :, None])[:, :, 0].sum(axis=0) * (4 * math.pi * rq * rq / m)
    assert abs(force[0] - F) < 2e-3 * abs(F)
    assert np.abs(force[1:]).max() < 2e-3 * abs(F)


def test_oracle_concentric_shells_32():
    """The oracle's exact constrained solve of the concentric-shells problem at
    32^3 (12 / 162 markers, cavity at rest, sphere moving with -V): the
    hydrodynamic radii and the velocity error against the analytic flow are
    those of a first-order method at this resolution (the paper's 30^3 run,
    with its six-point kernel and walls, reports R_h / R_g of 1.48 and 0.93
    and a relative L2 velocity error of 6.4e-2)."""
    from oracle import constrained, hasimoto
    from synthetic import concentric_shells, single_shell
    n = 32
    p1 = single_shell(n, 0)
    R1h = hasimoto.radius3d(abs(constrained.solve_problem(p1).F[0, 0]), 1.0)
    p2 = concentric_shells(n, 0)
    sol = constrained.solve_problem(p2)
    assert sol.F[0, 0] < 0                         # the sphere, moving with -V, pushes the fluid along -x
    R2h = R1h / shells.lambda_from_drag(-sol.F[0, 0], R1h)
    assert 1.2 < R1h / p2.radius[0] < 1.6
    assert 0.88 < R2h / p2.radius[1] < 1.0
    err = shells.flow_errors(sol.v, sol.p, n, p2.h, p2.centres[0], R1h, R2h, frame=1.0)
    assert err["v"]["L2"] < 0.1 and err["v"]["L1"] < 0.1
    # with the geometric radii the same flow looks several times less accurate
    err_g = shells.flow_errors(sol.v, sol.p, n, p2.h, p2.centres[0], p2.radius[0], p2.radius[1], frame=1.0)
    assert err_g["v"]["L2"] > 1.5 * err["v"]["L2"]
