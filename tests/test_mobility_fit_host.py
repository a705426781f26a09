"""Host logic of the fitted approximate mobility (Sec. 4.2 procedure,
Appendix A forms): the fitting routines recover the forms from data the forms
themselves generate, the self-mobility function has the limits the paper
states, and the compiled table is well formed."""
import math
import os
import re

import numpy as np
import pytest

from paper_1505_07865_amd import mobility_fit as mf


def test_phi0_limits():
    ah = 1.25
    z = (0.2, 0.3, 40.0)
    # inviscid: phi0(0) = 2 h^3 / (3 V_m), V_m = (8/3)^3 h^3 for the four-point kernel
    assert abs(mf.phi0(0.0, z, ah) - 2.0 / (3.0 * (8.0 / 3.0) ** 3)) < 1e-15
    # Stokes: phi0 beta -> 1 / (6 pi a/h)
    b = 1e14                           # the sqrt(beta) terms fall off as beta^-1/2
    assert abs(mf.phi0(b, z, ah) * b * 6.0 * math.pi * ah - 1.0) < 1e-6


def test_fit_steady_recovers_forms():
    ah = 1.2543
    b_true = np.array([0.0, 0.1188, 0.6485, 0.4377, -0.1236, 10.52, 0.2277])
    fx = mf.ft_steady(0.8, ah, b_true)
    b_true[0] = (0.8 / fx - 0.75 * ah) / 0.64
    rng = np.random.default_rng(0)
    x = rng.uniform(1.0, 12.0, 3000)
    h, eta, L = 1.0 / 64, 1.0, 1.0
    s = mf.SHIFT_3D / (6.0 * math.pi * eta * L)
    r = x * h
    perp = mf.ft_steady(x, ah, b_true) / (8.0 * math.pi * eta * r) - s
    g = mf.gt_steady(x, b_true) / (8.0 * math.pi * eta * r)
    self_mean = 1.0 / (6.0 * math.pi * eta * ah * h) - s
    ah_fit, b = mf.fit_steady(x, perp + g, perp, self_mean, eta, h, L)
    assert abs(ah_fit - ah) < 1e-12
    xs = np.linspace(0.0, 15.0, 400)
    assert np.allclose(mf.ft_steady(xs, ah_fit, b), mf.ft_steady(xs, ah, b_true), rtol=1e-4, atol=1e-6)
    assert np.allclose(mf.gt_steady(xs, b), mf.gt_steady(xs, b_true), rtol=1e-4, atol=1e-6)


def test_fit_beta_recovers_forms():
    beta, h = 0.25, 1.0 / 64
    eta = beta * h * h
    ph = 0.0243
    a_true = np.array([1.2, 0.8, 0.5, 1.1, 0.9, 0.3, 1.4, 0.02, 0.7, 0.6])
    b_true = np.array([1.3, 0.9, 0.6, 0.4, 0.3, 1.1])
    rng = np.random.default_rng(1)
    x = rng.uniform(1.0, 12.0, 3000)
    pre = beta / (eta * h)
    perp = -pre * mf.ft_beta(x, beta, ph, a_true) / (4.0 * math.pi * x ** 3)
    g = pre * 3.0 * mf.gt_beta(x, beta, ph, b_true) / (4.0 * math.pi * x ** 3)
    a, b = mf.fit_beta(x, perp + g, perp, beta, eta, h, ph)
    xs = np.linspace(1.0, 12.0, 200)
    ft_t, ft = mf.ft_beta(xs, beta, ph, a_true), mf.ft_beta(xs, beta, ph, a)
    gt_t, gt = mf.gt_beta(xs, beta, ph, b_true), mf.gt_beta(xs, beta, ph, b)
    assert np.max(np.abs(ft - ft_t)) < 1e-3 * np.max(np.abs(ft_t))
    assert np.max(np.abs(gt - gt_t)) < 1e-3 * np.max(np.abs(gt_t))


def test_pair_stats_of_a_known_tensor():
    """pair_stats reads f and g back from blocks f I + g r r^T."""
    rng = np.random.default_rng(2)
    R = rng.uniform(0.3, 0.7, (6, 3))
    N = len(R)
    M = np.zeros((3 * N, 3 * N))
    for i in range(N):
        M[3 * i:3 * i + 3, 3 * i:3 * i + 3] = 2.0 * np.eye(3)
        for j in range(N):
            if i != j:
                d = R[i] - R[j]
                r = np.linalg.norm(d)
                M[3 * i:3 * i + 3, 3 * j:3 * j + 3] = (1.0 / r) * np.eye(3) + (0.5 / r) * np.outer(d, d) / r ** 2
    r, par, perp, self_ = mf.pair_stats(M, R, 10.0)
    assert np.allclose(perp, 1.0 / r) and np.allclose(par, 1.5 / r) and np.allclose(self_, 2.0)


def test_compiled_table_is_well_formed():
    text = open(mf.TABLE).read()
    rows = int(re.search(r"kFitRows = (\d+);", text).group(1))
    if rows == 0:
        pytest.skip("no fitted table generated")
    betas = [float(v) for v in re.search(r"kFitBeta\[\d+\] = \{([^}]*)\}", text).group(1).split(",")]
    assert len(betas) == rows and betas == sorted(betas)
    ah = float(re.search(r"kFitAh = ([^;]+);", text).group(1))
    assert 1.15 < ah < 1.35            # the four-point marker radius near 1.25 h
    z = [float(v) for v in re.search(r"kFitZ\[3\] = \{([^}]*)\}", text).group(1).split(",")]
    ph = mf.phi0(np.array(betas), z, ah)
    assert np.all(np.diff(ph) < 0)     # the self mobility per unit beta falls with beta
    nums = [float(v) for v in re.findall(r"[-+]?\d+\.?\d*(?:[eE][-+]?\d+)?", text.split("kFitA", 1)[1])]
    assert all(np.isfinite(nums))

    def arr(pattern, cols):
        body = re.search(pattern + r"\s*=\s*\{(.*?)\};", text, re.S).group(1)
        vals = [float(v) for v in re.findall(r"[-+]?(?:\d+\.?\d*|\.\d+)(?:[eE][-+]?\d+)?", body)]
        return np.array(vals).reshape(rows, cols)

    A, B = arr(r"kFitA\[\d+\]\[10\]", 10), arr(r"kFitB\[\d+\]\[6\]", 6)
    # every row within the fit's bounds: no denominator changes sign at any
    # distance (rows in between blend two such functions)
    assert np.all(A >= np.array(mf.LB_A) - 1e-12) and np.all(A <= np.array(mf.UB_A) + 1e-12)
    assert np.all(B >= np.array(mf.LB_B) - 1e-12) and np.all(B <= np.array(mf.UB_B) + 1e-12)
    xs = np.linspace(0.1, 100.0, 2000)
    for k, beta in enumerate(betas):
        ph = float(mf.phi0(beta, z, ah))
        with np.errstate(over="ignore"):
            assert np.all(np.isfinite(mf.ft_beta(xs, beta, ph, A[k]))) and np.all(np.isfinite(mf.gt_beta(xs, beta, ph, B[k])))


def test_2d_fits_recover_forms():
    """Appendix B's forms: the 2D fits recover known coefficients, and
    phi0_2d starts at the inviscid value h^2 / (2 V_m)."""
    c_true = np.array([0.5, 0.3, 0.8, 0.6, 0.9, 0.2, 0.7, 0.4, 0.3])
    x = np.geomspace(1.0, 60.0, 200)
    f = mf.ft2_steady(x, c_true)
    g = mf.gt2_steady(x, c_true)
    eta, h, L, self_mean = 1.0, 1.0 / 256, 1.0, 0.3
    perp = self_mean - f / (4.0 * math.pi * eta)
    par = perp + g / (4.0 * math.pi * eta)
    ah, c = mf.fit_steady_2d(x, par, perp, self_mean, eta, h, L)
    assert abs(ah - L / (3.708 * math.exp(4.0 * math.pi * eta * self_mean)) / h) < 1e-12
    assert np.allclose(mf.ft2_steady(x, c), f, atol=1e-9) and np.allclose(mf.gt2_steady(x, c), g, atol=1e-9)
    beta = 0.5
    ct = np.array([1.0, 0.5, 0.7, 0.9, 1.2, 0.4, 0.3, 0.8, 0.5, 0.6, 0.2, 1.1, 0.9])
    ft = mf.ft2_beta(x, beta, ct)
    gt = mf.gt2_beta(x, beta, ct)
    perp = -ft / (2.0 * math.pi * x ** 2 * h ** 2)
    par = perp + gt / (math.pi * x ** 2 * h ** 2)
    cc = mf.fit_beta_2d(x, par, perp, beta, h)
    assert np.abs(mf.ft2_beta(x, beta, cc) - ft).max() < 1e-6 * np.abs(ft).max()
    assert np.abs(mf.gt2_beta(x, beta, cc) - gt).max() < 1e-6 * np.abs(gt).max()
    assert abs(mf.phi0_2d(1e-12, [0.1, 1.0, 1.0, 1.0]) - 1.0 / (2.0 * (8.0 / 3.0) ** 2)) < 1e-12


def test_compiled_2d_table_is_well_formed():
    text = open(mf.TABLE_2D).read()
    rows = int(re.search(r"kFit2Rows = (\d+);", text).group(1))
    if rows == 0:
        pytest.skip("no 2D fitted table generated")

    def arr(pattern):
        body = re.search(pattern + r"\s*=\s*\{(.*?)\};", text, re.S).group(1)
        return np.array([float(v) for v in re.findall(r"[-+]?(?:\d+\.?\d*|\.\d+)(?:[eE][-+]?\d+)?", body)])

    betas = arr(r"kFit2Beta\[\d+\]")
    assert len(betas) == rows and np.all(np.diff(betas) > 0)
    ah = float(re.search(r"kFit2Ah = ([^;]+);", text).group(1))
    assert 0.9 < ah < 1.2                      # the four-point marker radius in 2D, about 1.04 h
    z = arr(r"kFit2Z\[4\]")
    assert mf.phi0_2d_positive(z)
    st = arr(r"kFit2Steady\[9\]")
    assert np.all(st >= np.array(mf.LB_2S) - 1e-12) and np.all(st <= np.array(mf.UB_2S) + 1e-12)
    R = arr(r"kFit2Row\[\d+\]\[13\]").reshape(rows, 13)
    assert np.all(R >= np.array(mf.LB_2B) - 1e-12) and np.all(R <= np.array(mf.UB_2B) + 1e-12)
    xs = np.linspace(0.1, 200.0, 2000)
    assert np.all(np.isfinite(mf.ft2_steady(xs, st))) and np.all(np.isfinite(mf.gt2_steady(xs, st)))
    for k, beta in enumerate(betas):
        with np.errstate(over="ignore"):
            assert np.all(np.isfinite(mf.ft2_beta(xs, beta, R[k]))) and np.all(np.isfinite(mf.gt2_beta(xs, beta, R[k])))
