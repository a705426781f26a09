"""Interpolation J, spreading S and rigid-body kinematics, Secs. 2, 3.1 and 3.4.

    (J v)^alpha_i = sum_k v^alpha_k prod_beta phi((R_i^beta - x_k^{alpha,beta}) / h)
    (S L)^alpha_k = h^-d sum_i L^alpha_i prod_beta phi((R_i^beta - x_k^{alpha,beta}) / h)

x_k^{alpha,beta} is the beta coordinate of the alpha-face k: (k_beta + 1/2) h when
beta != alpha and k_beta h when beta == alpha.  Displacements use the periodic
minimum image.  The sums run over the support of phi (4 points per dimension);
every other term is zero.

Periodic steady Stokes replaces S by S' = S - vol^-1 1 1^T (eq. constrained_periodic):
the total marker force is removed again as a uniform force density.

Rigid marker velocities: V_i = U_p + Omega_p x (R_i - X_p), with Omega x r =
Omega (-r_y, r_x) in 2D.  Body force and torque: F_p = sum_i L_i,
T_p = sum_i (R_i - X_p) x L_i (Sec. 2; drag F = sum L, Sec. 7.3).
"""
import itertools

import numpy as np

from . import kernel


def taps_1d(pos, n, h, staggered):
    """Indices [N,4] and weights [N,4] of the 4 grid points near pos along one axis.

    staggered: the grid points of this axis sit at j*h (faces normal to the axis)
    instead of (j + 1/2) h (cell centres).
    """
    s = pos / h - (0.0 if staggered else 0.5)
    base = np.floor(s).astype(np.int64) - 1
    j = base[:, None] + np.arange(4)[None, :]
    w = kernel.phi(s[:, None] - j)
    return np.mod(j, n), w


def weights(R, n, h, alpha):
    """Flat grid indices [N, 4^d] and weights [N, 4^d] of marker taps on the alpha-faces."""
    N, d = R.shape
    idx1, w1 = [], []
    for beta in range(d):
        i, w = taps_1d(R[:, beta], n, h, staggered=(beta == alpha))
        idx1.append(i)
        w1.append(w)
    flat = np.zeros((N, 4 ** d), dtype=np.int64)
    wt = np.ones((N, 4 ** d))
    for t, combo in enumerate(itertools.product(range(4), repeat=d)):
        # combo[beta] is the tap along axis beta; flat index over array axes (z, y, x)
        f = np.zeros(N, dtype=np.int64)
        for beta in reversed(range(d)):
            f = f * n + idx1[beta][:, combo[beta]]
        flat[:, t] = f
        for beta in range(d):
            wt[:, t] *= w1[beta][:, combo[beta]]
    return flat, wt


def all_weights(R, n, h):
    """weights() for every component alpha (reused when R does not change)."""
    return [weights(R, n, h, a) for a in range(R.shape[1])]


def interp(v, R, h, W=None):
    """J v: [d, n..] face field -> [N, d] marker values."""
    d = v.shape[0]
    n = v.shape[1]
    W = W or all_weights(R, n, h)
    out = np.zeros((R.shape[0], d))
    for a in range(d):
        flat, wt = W[a]
        out[:, a] = (v[a].reshape(-1)[flat] * wt).sum(axis=1)
    return out


def spread(lam, R, n, h, W=None):
    """S Lambda: [N, d] marker forces -> [d, n..] face force density."""
    N, d = R.shape
    W = W or all_weights(R, n, h)
    out = np.zeros((d,) + (n,) * d)
    for a in range(d):
        flat, wt = W[a]
        acc = np.zeros(n ** d)
        np.add.at(acc, flat.reshape(-1), (wt * lam[:, a:a + 1]).reshape(-1))
        out[a] = acc.reshape((n,) * d)
    return out / h ** d


def spread_periodic_steady(lam, R, n, h, W=None):
    """S' Lambda = S Lambda - vol^-1 sum_i Lambda_i (uniform per component)."""
    d = R.shape[1]
    vol = (n * h) ** d
    out = spread(lam, R, n, h, W)
    tot = lam.sum(axis=0)
    for a in range(d):
        out[a] -= tot[a] / vol
    return out


def min_image(dr, L):
    return dr - L * np.round(dr / L)


def body_of(offsets):
    nb = len(offsets) - 1
    return np.repeat(np.arange(nb), np.diff(offsets))


def cross(omega, r):
    """Omega x r; omega has 1 component in 2D, 3 in 3D."""
    if r.shape[1] == 2:
        return np.stack([-omega[:, 0] * r[:, 1], omega[:, 0] * r[:, 0]], axis=1)
    return np.cross(omega, r)


def marker_velocities(R, offsets, centres, U, Omega, L):
    b = body_of(offsets)
    r = min_image(R - centres[b], L)
    return U[b] + cross(Omega[b], r)


def body_force_torque(lam, R, offsets, centres, L):
    nb = len(offsets) - 1
    d = R.shape[1]
    b = body_of(offsets)
    r = min_image(R - centres[b], L)
    F = np.zeros((nb, d))
    np.add.at(F, b, lam)
    if d == 2:
        tq = r[:, 0] * lam[:, 1] - r[:, 1] * lam[:, 0]
        T = np.zeros((nb, 1))
        np.add.at(T[:, 0], b, tq)
    else:
        T = np.zeros((nb, 3))
        np.add.at(T, b, np.cross(r, lam))
    return F, T
