"""Unsteady Navier-Stokes steps with moving rigid bodies (Sec. 3 and Sec. 7.6).

The paper treats advection explicitly and viscosity implicitly (backward Euler
here, kappa = 1), and solves the constrained system eq. constrained_Stokes at
every step.  Its advection scheme (Adams-Bashforth with a staggered PPM
upwinding) is described only by citation, so this module uses the documented
reading: the centred second-order advective form on the MAC grid with
Adams-Bashforth 2 (forward Euler on the first step):

    N(v)^alpha_c = sum_beta vbar^beta (v^alpha_{c+e_beta} - v^alpha_{c-e_beta}) / (2h)
    vbar^alpha   = v^alpha_c
    vbar^beta    = (v^beta_c + v^beta_{c+e_beta} + v^beta_{c-e_alpha} + v^beta_{c-e_alpha+e_beta}) / 4
    g^{n+1}      = (rho/dt) v^n - rho (3/2 N(v^n) - 1/2 N(v^{n-1}))

Markers move with their prescribed body velocity before the solve,
R^{n+1} = R^n + dt U_p, and the constraint J v^{n+1} = V holds at the new
positions.  The fluid starts at rest.
"""
import numpy as np

from . import constrained, ib
from .grid import axis_of, shift


def advection(v, h):
    d = v.shape[0]
    out = np.zeros_like(v)
    for a in range(d):
        axa = axis_of(a, d)
        acc = np.zeros_like(v[a])
        for b in range(d):
            axb = axis_of(b, d)
            if b == a:
                vb = v[a]
            else:
                vb = 0.25 * (v[b] + shift(v[b], 1, axb) + shift(v[b], -1, axa)
                             + shift(shift(v[b], -1, axa), 1, axb))
            acc += vb * (shift(v[a], 1, axb) - shift(v[a], -1, axb)) / (2.0 * h)
        out[a] = acc
    return out


def rhs(v_n, N_n, N_nm1, rho, dt, first):
    if first:
        return (rho / dt) * v_n - rho * N_n
    return (rho / dt) * v_n - rho * (1.5 * N_n - 0.5 * N_nm1)


def run(prob, nsteps, **kw):
    """Exact constrained solves along the trajectory; returns the list of Solutions."""
    d, n, h = prob.dim, prob.n, prob.h
    v = np.zeros((d,) + (n,) * d)
    N_prev = None
    R = prob.R.copy()
    centres = prob.centres.copy()
    out = []
    b = ib.body_of(prob.offsets)
    for step in range(nsteps):
        N_n = advection(v, h)
        g = rhs(v, N_n, N_prev, prob.rho, prob.dt, first=(step == 0))
        R = np.mod(R + prob.dt * prob.U[b], prob.L)
        centres = np.mod(centres + prob.dt * prob.U, prob.L)
        sysm = constrained.System.from_problem(prob, R=R)
        V = ib.marker_velocities(R, prob.offsets, centres, prob.U, prob.Omega, prob.L)
        sol = constrained.solve(sysm, g, None, -V, prob.offsets, centres, **kw)
        out.append(sol)
        N_prev = N_n
        v = sol.v
    return out
