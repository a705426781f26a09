"""Periodic drag formulas used to pin the oracle (Secs. 7.3 and 7.5).

3D, simple cubic array of spheres with cell length l (eq. drag_periodic):
    F / (eta V) = 6 pi R_h / (1 - 2.8373 (R_h/l) + 4.19 (R_h/l)^3 - 27.4 (R_h/l)^6)
2D, square array of disks (eq. drag_periodic_2D), phi = pi R_h^2 / l^2:
    F / (eta V) = 4 pi / (-ln sqrt(phi) - 0.738 + phi - 0.887 phi^2 + 2.038 phi^3)
Both are inverted for the hydrodynamic radius R_h by bisection.
"""
import math


def drag3d(rh, l):
    x = rh / l
    return 6.0 * math.pi * rh / (1.0 - 2.8373 * x + 4.19 * x ** 3 - 27.4 * x ** 6)


def drag2d(rh, l):
    phi = math.pi * rh * rh / (l * l)
    return 4.0 * math.pi / (-math.log(math.sqrt(phi)) - 0.738 + phi - 0.887 * phi ** 2 + 2.038 * phi ** 3)


def _invert(fun, target, lo, hi):
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fun(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def radius3d(drag_over_eta_v, l):
    """R_h from F/(eta V) for a cubic array (drag is increasing in R_h for R_h < 0.3 l)."""
    return _invert(lambda r: drag3d(r, l), drag_over_eta_v, 1e-9 * l, 0.3 * l)


def radius2d(drag_over_eta_v, l):
    return _invert(lambda r: drag2d(r, l), drag_over_eta_v, 1e-9 * l, 0.3 * l)
