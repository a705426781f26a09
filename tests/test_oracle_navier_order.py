"""Temporal order of the oracle's unsteady steps (Sec. 3 and Sec. 7.6:
explicit advection, implicit viscosity and constraint).

``navier.run``'s centred form advances (rho/dt)(v^{n+1} - v^n) =
-rho AB2(N) + eta h^-2 L v^{n+1} - G pi + S Lambda with D v = 0 and J v = V at
t^{n+1}.  With the markers at rest and a vanishing viscosity the constraint
rows form a fixed orthogonal projection P (A is a multiple of the identity),
so one step is v^{n+1} = P (v^n - dt (3/2 N^n - 1/2 N^{n-1})): Adams-Bashforth
2 on the projected ODE v' = -P N(v), globally second order in dt when the
first step is forward Euler and v0 already satisfies the constraints.  A
dropped history term (weights 1, 0), a misplaced one (1/2, 1/2) or an
Adams-Bashforth first step without history all make the scheme first order;
the planted-mistake test below checks that the order test tells them apart.
"""
import dataclasses

import numpy as np
import pytest

from oracle import constrained, navier
from synthetic import small_problem

T_END = 0.1
STEPS = (4, 8, 16, 32)


def _problem():
    p = small_problem(3, 2, 16, radius_h=3.0, rho=1.0, eta=1e-9, dt=T_END / STEPS[0], rotate=False)
    return dataclasses.replace(p, U=np.zeros_like(p.U), Omega=np.zeros_like(p.Omega))


def _initial_velocity(p):
    """A smooth O(1) flow that already satisfies D v = 0 and J v = 0: the
    exact constrained response to a few Fourier modes of forcing."""
    n, h = p.n, p.h
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    g = np.zeros((2, n, n))
    g[0] = np.sin(2 * np.pi * Y) + 0.5 * np.cos(2 * np.pi * (X + 2 * Y))
    g[1] = 0.7 * np.cos(2 * np.pi * X) + 0.4 * np.sin(2 * np.pi * (2 * X - Y))
    sysm = constrained.System(2, n, h, 1.0, p.eta, p.R)
    sol = constrained.solve(sysm, g, None, np.zeros((p.nmarkers, 2)), p.offsets, p.centres)
    return sol.v / np.abs(sol.v).max()


def _successive_differences(p, v0):
    end = {}
    for ns in STEPS:
        q = dataclasses.replace(p, dt=T_END / ns)
        end[ns] = navier.run(q, ns, v0=v0)[-1].v
    return [np.linalg.norm(end[a] - end[2 * a]) for a in STEPS[:-1]]


def test_centred_steps_are_second_order_in_time():
    p = _problem()
    v0 = _initial_velocity(p)
    e = _successive_differences(p, v0)
    ratios = [e[0] / e[1], e[1] / e[2]]
    # the flow changes by O(1) over the interval: the test is not vacuous
    last = navier.run(dataclasses.replace(p, dt=T_END / STEPS[-1]), STEPS[-1], v0=v0)[-1].v
    assert np.linalg.norm(last - v0) > 0.1 * np.linalg.norm(v0)
    assert all(3.5 < r < 4.6 for r in ratios), (e, ratios)


def _planted(kind):
    def rhs(v_n, N_n, N_nm1, rho, dt, first):
        if kind == "no-start":
            hist = np.zeros_like(N_n) if N_nm1 is None else N_nm1
            return (rho / dt) * v_n - rho * (1.5 * N_n - 0.5 * hist)
        if first:
            return (rho / dt) * v_n - rho * N_n
        w0, w1 = {"euler": (1.0, 0.0), "average": (0.5, 0.5)}[kind]
        return (rho / dt) * v_n - rho * (w0 * N_n + w1 * N_nm1)
    return rhs


@pytest.mark.parametrize("kind", ["euler", "average", "no-start"])
def test_order_test_detects_wrong_history_weights(monkeypatch, kind):
    p = _problem()
    v0 = _initial_velocity(p)
    monkeypatch.setattr(navier, "rhs", _planted(kind))
    e = _successive_differences(p, v0)
    ratios = [e[0] / e[1], e[1] / e[2]]
    assert all(r < 2.6 for r in ratios), (kind, e, ratios)
