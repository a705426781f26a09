"""One geometric-multigrid V-cycle for (c0 - c1 L) x = b on a periodic grid.

Sec. 5.2 approximates A^-1 (vector Helmholtz, one cycle per velocity component)
and L_p^-1 (scalar Poisson) by a single V-cycle each (eq. P1_practical), and
leaves the cycle's internals to the cited multigrid solvers.  The cycle used
here is the documented reading of that passage; every grid (cell-centred
pressure or one face-centred velocity component) is a periodic lattice of n^d
points with the same dimensionless Laplacian L.

    level grid     n, n/2, ..., down to n_c = 4 points per side (or n if smaller)
    coarse op      (c0 - (c1/4) L) on the next level (rediscretised, spacing 2h)
    smoother       red-black Gauss-Seidel, red (even i+j+k) first; nu_pre sweeps
                   from a zero initial guess, nu_post sweeps after correction
    restriction    average of the 2^d fine points of each coarse point
    prolongation   cell-centred multilinear: weights 3/4, 1/4 per axis
    coarsest       nu_coarse red-black sweeps from zero
    singular case  (c0 == 0, steady periodic): b loses its mean on the finest and
                   coarsest levels and x loses its mean on output (the restricted
                   inverse of Sec. 5.1)
"""
import numpy as np

from .grid import lap, shift

COARSEST = 4


def parity(shape):
    idx = np.indices(shape)
    return idx.sum(axis=0) % 2


def apply_op(x, c0, c1):
    return c0 * x - c1 * lap(x)


def rb_sweep(x, b, c0, c1, color_mask):
    d = x.ndim
    nb = np.zeros_like(x)
    for ax in range(d):
        nb += shift(x, 1, ax) + shift(x, -1, ax)
    new = (b + c1 * nb) / (c0 + 2.0 * d * c1)
    return np.where(color_mask, new, x)


def smooth(x, b, c0, c1, sweeps):
    par = parity(x.shape)
    red = par == 0
    black = par == 1
    for _ in range(sweeps):
        x = rb_sweep(x, b, c0, c1, red)
        x = rb_sweep(x, b, c0, c1, black)
    return x


def restrict(r):
    d = r.ndim
    n = r.shape[0]
    shp = []
    for _ in range(d):
        shp += [n // 2, 2]
    return r.reshape(shp).mean(axis=tuple(range(1, 2 * d, 2)))


def prolong(e):
    """Multilinear cell-centred prolongation of a coarse field to the next finer level."""
    out = e
    for ax in range(e.ndim):
        lo = 0.75 * out + 0.25 * np.roll(out, 1, axis=ax)   # even children: neighbour below
        hi = 0.75 * out + 0.25 * np.roll(out, -1, axis=ax)  # odd children: neighbour above
        st = np.stack([lo, hi], axis=ax + 1)
        shp = list(out.shape)
        shp[ax] *= 2
        out = st.reshape(shp)
    return out


def vcycle(b, c0, c1, nu_pre=2, nu_post=2, nu_coarse=4, _top=True):
    b = np.asarray(b, dtype=np.float64)
    singular = c0 == 0.0
    n = b.shape[0]
    if singular and _top:
        b = b - b.mean()
    if n <= COARSEST:
        if singular:
            b = b - b.mean()
        x = smooth(np.zeros_like(b), b, c0, c1, nu_coarse)
    else:
        x = smooth(np.zeros_like(b), b, c0, c1, nu_pre)
        r = b - apply_op(x, c0, c1)
        e = vcycle(restrict(r), c0, c1 / 4.0, nu_pre, nu_post, nu_coarse, _top=False)
        x = x + prolong(e)
        x = smooth(x, b, c0, c1, nu_post)
    if singular and _top:
        x = x - x.mean()
    return x
