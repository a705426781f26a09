"""Peskin's four-point kernel phi(r), r in units of h.

Sec. 3.1 writes the regularised delta as a tensor product
delta_a(r) = h^-d prod_alpha phi(r_alpha / h).  The four-point phi is the one
from Peskin's review (cited in Sec. 4.1 for a ~ 1.25 h):

    phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8     for |r| <= 1
    phi(r) = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8   for 1 <= |r| <= 2
    phi(r) = 0                                           otherwise

It is the unique function supported on |r| < 2 that satisfies the even/odd
partition of unity, the zero first moment and sum phi^2 = 3/8; the tests check
those defining conditions rather than the formula.
"""
import numpy as np

SUPPORT = 4  # grid points per dimension with a nonzero weight


def phi(r):
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    inner = r <= 1.0
    outer = (r > 1.0) & (r < 2.0)
    ri = r[inner]
    out[inner] = (3.0 - 2.0 * ri + np.sqrt(1.0 + 4.0 * ri - 4.0 * ri * ri)) / 8.0
    ro = r[outer]
    out[outer] = (5.0 - 2.0 * ro - np.sqrt(np.maximum(0.0, -7.0 + 12.0 * ro - 4.0 * ro * ro))) / 8.0
    return out
