"""Steady Stokes flow between two concentric spheres (Sec. 7.3 and its
appendix): the analytic reference for the concentric-shells accuracy study.

TEST INFRASTRUCTURE ONLY (see the package header).

An inner sphere of radius a is at rest, the outer spherical cavity of radius
b > a translates with velocity V along the unit axis e, viscosity mu.  The
appendix prints coefficients for this flow, but as printed here they do not
meet the no-slip conditions (the tangential velocity on the inner sphere and
both components on the outer one come out wrong), so the oracle uses the
boundary value problem itself: Stokes' axisymmetric stream function
psi = sin^2(theta) f(r) with

    f(r) = A / r + B r + C r^2 + D r^4,
    u_r = 2 cos(theta) f / r^2,   u_theta = -sin(theta) f' / r,

(theta measured from e), the general solution of E^4 psi = 0 with this
angular form, and the four conditions f(a) = f'(a) = 0 (no slip on the inner
sphere) and f(b) = V b^2 / 2, f'(b) = V b (rigid translation of the cavity),
solved as a 4 x 4 linear system.  The pressure is
p = mu cos(theta) (2 B / r^2 + 20 D r) + constant, and the force the fluid
exerts on the inner sphere is -8 pi mu B e (B, the Stokeslet coefficient, is
negative here: the moving cavity drags the sphere along e); the paper's drag
law, that force = 6 pi mu a V K e with K = (1 - l^5) / alpha,
alpha = 1 - 9/4 l + 5/2 l^3 - 9/4 l^5 + l^6, l = a / b, is one of the pins.
The sphere's markers apply the opposite force to the fluid (the sign of
Lambda).
"""
import math

import numpy as np


def coefficients(a, b, V=1.0):
    """(A, B, C, D) of f(r) for inner radius a at rest and cavity b moving with V."""
    M = np.array([[1.0 / a, a, a * a, a ** 4],
                  [-1.0 / a ** 2, 1.0, 2.0 * a, 4.0 * a ** 3],
                  [1.0 / b, b, b * b, b ** 4],
                  [-1.0 / b ** 2, 1.0, 2.0 * b, 4.0 * b ** 3]])
    return np.linalg.solve(M, np.array([0.0, 0.0, V * b * b / 2.0, V * b]))


def drag_factor(lam):
    """K(l) of the paper's drag law force = 6 pi mu a V K."""
    alpha = 1.0 - 2.25 * lam + 2.5 * lam ** 3 - 2.25 * lam ** 5 + lam ** 6
    return (1.0 - lam ** 5) / alpha


def inner_force(a, b, V=1.0, mu=1.0):
    """Force of the fluid on the inner sphere along e: -8 pi mu B."""
    return -8.0 * math.pi * mu * coefficients(a, b, V)[1]


def lambda_from_drag(force, a, V=1.0, mu=1.0):
    """l = a / b from the drag on the inner sphere (K increases with l), by bisection."""
    target = force / (6.0 * math.pi * mu * a * V)
    lo, hi = 1e-6, 0.9
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if drag_factor(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _polar(X, centre, e, L):
    d = np.asarray(X, dtype=np.float64) - np.asarray(centre, dtype=np.float64)
    if L is not None:
        d = d - L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(axis=-1))
    rs = np.where(r > 0, r, 1.0)
    ct = (d @ e) / rs
    return d, r, rs, ct


def velocity(X, centre, a, b, V=1.0, e=(1.0, 0.0, 0.0), L=None):
    """Velocity at points X [..., 3]: 0 inside the inner sphere, the analytic
    flow between the spheres, V e outside the cavity (its rigid motion).
    L: periodic box side for minimum-image displacements (None: none)."""
    e = np.asarray(e, dtype=np.float64)
    e = e / np.linalg.norm(e)
    A, B, C, D = coefficients(a, b, V)
    d, r, rs, ct = _polar(X, centre, e, L)
    f = A / rs + B * rs + C * rs * rs + D * rs ** 4
    fp = -A / rs ** 2 + B + 2.0 * C * rs + 4.0 * D * rs ** 3
    er = d / rs[..., None]
    # u = u_r e_r + u_theta e_theta with sin(theta) e_theta = cos(theta) e_r - e
    ur = 2.0 * ct * f / rs ** 2
    u = ur[..., None] * er - (fp / rs)[..., None] * (ct[..., None] * er - e)
    u = np.where((r < a)[..., None], 0.0, u)
    u = np.where((r > b)[..., None], V * e, u)
    return u


def pressure(X, centre, a, b, V=1.0, mu=1.0, e=(1.0, 0.0, 0.0), L=None):
    """Pressure between the spheres, mu cos(theta) (2 B / r^2 + 20 D r) (gauge:
    no constant); NaN outside the annulus a <= r <= b."""
    e = np.asarray(e, dtype=np.float64)
    e = e / np.linalg.norm(e)
    A, B, C, D = coefficients(a, b, V)
    d, r, rs, ct = _polar(X, centre, e, L)
    p = mu * ct * (2.0 * B / rs ** 2 + 20.0 * D * rs)
    return np.where((r >= a) & (r <= b), p, np.nan)


def flow_errors(u, p, n, h, centre, a, b, V=1.0, mu=1.0, e=(1.0, 0.0, 0.0), frame=0.0):
    """Normalised error norms of a MAC solution (u [3][n][n][n] on the faces,
    the alpha-face of cell c at the cell centre minus h/2 along alpha, layout
    [k][j][i]; p [n][n][n] at cell centres) against the analytic flow with
    radii a < b.  Velocity: every face inside the cavity (r < b, the inner
    sphere's interior included, where the flow is at rest), all three
    components; pressure: cell centres in the annulus a <= r <= b, compared up
    to a constant (the mean difference over the annulus is removed).  Each
    norm is normalised by the same norm of the analytic field over the same
    points: L1 = sum|d| / sum|v|, L2 = sqrt(sum d^2 / sum v^2),
    Linf = max|d| / max|v|.  frame: velocity (along e) of the frame the
    solution is computed in (frame = V: the cavity at rest and the sphere
    moving with -V e); the solution is shifted by +frame e into the frame of
    the analytic flow (cavity moving with V e), so the norms are those of
    that flow, as the paper reports them."""
    L = n * h
    idx = (np.arange(n) + 0.5) * h
    zc, yc, xc = np.meshgrid(idx, idx, idx, indexing="ij")
    centres_xyz = np.stack([xc, yc, zc], axis=-1)
    du, vu = [], []
    for al in range(3):
        X = centres_xyz.copy()
        X[..., al] -= 0.5 * h
        d = X - np.asarray(centre)
        d -= L * np.round(d / L)
        r = np.sqrt((d ** 2).sum(axis=-1))
        inside = r < b
        ue = velocity(X[inside], centre, a, b, V, e, L)[:, al]
        du.append(u[al][inside] + frame * np.asarray(e)[al] / np.linalg.norm(e) - ue)
        vu.append(ue)
    du = np.concatenate(du)
    vu = np.concatenate(vu)
    d = centres_xyz - np.asarray(centre)
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(axis=-1))
    ann = (r >= a) & (r <= b)
    pe = pressure(centres_xyz[ann], centre, a, b, V, mu, e, L)
    dp = p[ann] - pe
    dp -= dp.mean()

    def norms(dv, v):
        return {"L1": float(np.abs(dv).sum() / np.abs(v).sum()),
                "L2": float(np.sqrt((dv ** 2).sum() / (v ** 2).sum())),
                "Linf": float(np.abs(dv).max() / np.abs(v).max())}
    return {"v": norms(du, vu), "p": norms(dp, pe), "faces": int(du.size), "cells": int(ann.sum())}
