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

The semi-Lagrangian alternative (``advection_sl``) transports v along
x - dt u(x) with multilinear interpolation, which is stable at any cell
Reynolds number (a convex combination of lattice values), where the centred
form with AB2 grows without bound once the viscous damping per step is weak
(Re = 100 on the 128^3 workload).

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


def face_velocity(v, a):
    """Velocity at the a-faces: v^a itself and, for b != a, the average of
    the four b-faces around each a-face (vbar^b of the advective form)."""
    d = v.shape[0]
    axa = axis_of(a, d)
    out = []
    for b in range(d):
        if b == a:
            out.append(v[a])
        else:
            axb = axis_of(b, d)
            out.append(0.25 * (v[b] + shift(v[b], 1, axb) + shift(v[b], -1, axa)
                               + shift(shift(v[b], -1, axa), 1, axb)))
    return out


def interp_lattice(q, s, fold=None):
    """Multilinear interpolation of the lattice values q at the fractional
    lattice coordinates s (one array per axis of q, each of q's shape).
    fold(ax, j) maps integer indices j along axis ax to (index, sign) arrays;
    None wraps periodically."""
    nd = q.ndim
    lo = [np.floor(x).astype(np.int64) for x in s]
    fr = [x - np.floor(x) for x in s]
    acc = np.zeros(q.shape)
    for corner in range(2 ** nd):
        w = np.ones(q.shape)
        sign = np.ones(q.shape)
        gi = []
        for ax in range(nd):
            o = (corner >> ax) & 1
            w = w * (fr[ax] if o else 1.0 - fr[ax])
            j = lo[ax] + o
            if fold is None:
                gi.append(np.mod(j, q.shape[ax]))
            else:
                jj, sg = fold(ax, j)
                gi.append(jj)
                sign = sign * sg
        acc += w * sign * q[tuple(gi)]
    return acc


def departure_values(v, h, dt):
    """Semi-Lagrangian transport (a reading: the paper cites its upwind
    advection scheme instead of giving it): v^a at the departure point
    x - dt u(x) of every a-face x, with u from ``face_velocity``, interpolated
    multilinearly on the a-face lattice.  In lattice units the departure point
    of face c is c - dt u / h along each axis."""
    d = v.shape[0]
    out = np.zeros_like(v)
    idx = np.indices(v.shape[1:]).astype(np.float64)
    for a in range(d):
        u = face_velocity(v, a)
        s = [idx[ax] - dt * u[d - 1 - ax] / h for ax in range(d)]
        out[a] = interp_lattice(v[a], s)
    return out


def advection_sl(v, h, dt):
    """The advection term of the semi-Lagrangian step, N = (v - v_departure)/dt,
    so that g = (rho/dt) v - rho N = (rho/dt) v_departure."""
    return (v - departure_values(v, h, dt)) / dt


def rhs(v_n, N_n, N_nm1, rho, dt, first):
    if first:
        return (rho / dt) * v_n - rho * N_n
    return (rho / dt) * v_n - rho * (1.5 * N_n - 0.5 * N_nm1)


def run(prob, nsteps, scheme="centred", v0=None, **kw):
    """Exact constrained solves along the trajectory; returns the list of
    Solutions.  scheme: "centred" (advective form, AB2) or "sl"
    (semi-Lagrangian transport, g = (rho/dt) v_departure).  v0: velocity at
    t = 0 ([d, n..]; default: the fluid at rest)."""
    d, n, h = prob.dim, prob.n, prob.h
    v = np.zeros((d,) + (n,) * d) if v0 is None else np.array(v0, dtype=np.float64)
    N_prev = None
    R = prob.R.copy()
    centres = prob.centres.copy()
    out = []
    b = ib.body_of(prob.offsets)
    for step in range(nsteps):
        if scheme == "sl":
            N_n = advection_sl(v, h, prob.dt)
            g = rhs(v, N_n, None, prob.rho, prob.dt, first=True)
        else:
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
