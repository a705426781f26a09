"""Exact periodic Stokes solve by discrete Fourier transform, Sec. 3.3.

For a periodic box the MAC operators are circulant and commute
(eq. L_inv_periodic), so the unconstrained system eq. Stokes_saddle,

    A v + G pi = f,     -D v = hp,

is diagonal in Fourier space.  With theta_beta = 2 pi k_beta / n and numpy's
forward transform u_hat(k) = sum_j u_j exp(-i theta.j):

    G_hat_alpha = (1 - exp(-i theta_alpha)) / h
    D_hat_alpha = (exp(i theta_alpha) - 1) / h
    D_hat . G_hat = -sigma / h^2,  sigma = 4 sum_beta sin^2(theta_beta / 2)
    A_hat = rho/dt + eta sigma / h^2

and for k != 0:  pi_hat = (A_hat hp_hat + D_hat . f_hat) / (D_hat . G_hat),
                 v_hat  = (f_hat - G_hat pi_hat) / A_hat.
At k = 0 the pressure mean is set to zero; the velocity mean is f_hat(0)/A_hat(0)
when A is invertible and zero for steady Stokes (the restricted inverse of
Sec. 5.1, acting on mean-zero data and returning mean-zero data).

The transforms are SciPy's (pocketfft); they run on as many threads as the
caller's ``scipy.fft.set_workers`` context gives (one by default).
"""
import numpy as np
import scipy.fft as sfft


def _symbols(n, d, h):
    """theta arrays broadcastable to the rfftn output shape of a (n,)*d field."""
    th = []
    for ax in range(d):
        if ax == d - 1:
            k = np.arange(n // 2 + 1)
        else:
            k = np.fft.fftfreq(n, 1.0 / n)
        shape = [1] * d
        shape[ax] = len(k)
        th.append((2.0 * np.pi * k / n).reshape(shape))
    return th  # indexed by array axis


def solve(f, hp, c0, eta, h, d):
    """Solve the periodic unconstrained Stokes system.

    f:  [..., d, n..] momentum right-hand side (leading batch axes allowed)
    hp: [..., n..] continuity right-hand side, or None for zero
    Returns (v, pi) with the same shapes.
    """
    nd = f.ndim
    n = f.shape[-1]
    gaxes = tuple(range(nd - d, nd))
    cax = nd - d - 1
    th = _symbols(n, d, h)
    # component alpha varies along array axis d-1-alpha
    Gh = [(1.0 - np.exp(-1j * th[d - 1 - a])) / h for a in range(d)]
    Dh = [(np.exp(1j * th[d - 1 - a]) - 1.0) / h for a in range(d)]
    sigma = sum(4.0 * np.sin(t / 2.0) ** 2 for t in th)
    Ah = c0 + eta * sigma / (h * h)
    DG = -sigma / (h * h)
    zero = DG == 0.0
    DG_safe = np.where(zero, 1.0, DG)

    fh = sfft.rfftn(f, axes=gaxes)
    num = 0.0
    for a in range(d):
        num = num + Dh[a] * np.take(fh, a, axis=cax)
    if hp is not None:
        num = num + Ah * sfft.rfftn(hp, axes=tuple(range(hp.ndim - d, hp.ndim)))
    ph = np.where(zero, 0.0, num / DG_safe)
    singular = Ah == 0.0
    A_safe = np.where(singular, 1.0, Ah)
    vh = np.stack([np.where(singular, 0.0, (np.take(fh, a, axis=cax) - Gh[a] * ph) / A_safe)
                   for a in range(d)], axis=cax)
    shape = f.shape[-d:]
    v = sfft.irfftn(vh, s=shape, axes=gaxes)
    p = sfft.irfftn(ph, s=shape, axes=tuple(range(ph.ndim - d, ph.ndim)))
    return v, p


def helmholtz_solve(b, c0, c1):
    """Exact periodic solve of (c0 - c1 L) x = b for a scalar field (restricted when c0 == 0)."""
    d = b.ndim
    n = b.shape[-1]
    th = _symbols(n, d, 1.0)
    sigma = sum(4.0 * np.sin(t / 2.0) ** 2 for t in th)
    sym = c0 + c1 * sigma
    bh = sfft.rfftn(b)
    xh = np.where(sym == 0.0, 0.0, bh / np.where(sym == 0.0, 1.0, sym))
    return sfft.irfftn(xh, s=b.shape, axes=tuple(range(d)))
