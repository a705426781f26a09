"""MAC (staggered) grid operators on a periodic box, Sec. 3.2.

Layout: a scalar field has shape (n,)*d with axes ordered (z, y, x) in 3D and
(y, x) in 2D, so x is the fastest index.  A face-centred vector field has shape
(d, n, ..., n); component alpha (0 = x, 1 = y, 2 = z) lives on array axis
d-1-alpha of its own slab.  Cell centres sit at (i+1/2)h; the alpha-face with
index c sits half a cell below the centre of cell c along alpha.

Operators (plain definitions, periodic wrap):
    (G pi)^alpha_c = (pi_c - pi_{c-e_alpha}) / h
    (D v)_c       = sum_alpha (v^alpha_{c+e_alpha} - v^alpha_c) / h      (D = -G^T)
    (L x)_c       = sum_beta (x_{c+e_beta} - 2 x_c + x_{c-e_beta})     (dimensionless)
    A v           = (rho/dt) v - eta h^-2 L v                           (eq. A_def, kappa = 1)
Steady Stokes is rho/dt = 0.
"""
import numpy as np


def axis_of(alpha: int, d: int) -> int:
    return d - 1 - alpha


def shift(x, offset: int, axis: int):
    """Return y with y_c = x_{c + offset e_axis} (periodic)."""
    return np.roll(x, -offset, axis=axis)


def lap(x):
    """Dimensionless Laplacian of a scalar field (every axis of x is a grid axis)."""
    out = -2.0 * x.ndim * x
    for ax in range(x.ndim):
        out = out + shift(x, 1, ax) + shift(x, -1, ax)
    return out


def grad(p, h):
    d = p.ndim
    return np.stack([(p - shift(p, -1, axis_of(a, d))) / h for a in range(d)])


def div(v, h):
    d = v.shape[0]
    out = np.zeros(v.shape[1:])
    for a in range(d):
        ax = axis_of(a, d)
        out += (shift(v[a], 1, ax) - v[a]) / h
    return out


def helmholtz(v, c0, eta, h):
    """A v = c0 v - eta h^-2 L v, applied to every component (c0 = rho/dt, 0 when steady)."""
    return np.stack([c0 * v[a] - eta / (h * h) * lap(v[a]) for a in range(v.shape[0])])


def stokes_apply(v, p, c0, eta, h):
    """Unconstrained Stokes operator [[A, G], [-D, 0]] applied to (v, p)."""
    return helmholtz(v, c0, eta, h) + grad(p, h), -div(v, h)
