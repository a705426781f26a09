"""Fitted approximate mobility M~ of Sec. 4.2 (forms of Appendix A) for the
four-point kernel, from pair mobilities measured with this library's solver.

    python -m paper_1505_07865_amd.mobility_fit [--pairs P.npz [--measure-only | --fit-only]]

The measurement needs the GPU; --fit-only refits saved pair data on the host.

Procedure (Sec. 4.2): N markers placed at random in a cube of side l/8 inside
a periodic box of side l (here a second cloud in a cube of side l/4 as well,
for pairs at larger distances); the mobility M = J L^-1 S of the cloud is measured
and, for every pair (i, j), the parallel and perpendicular mobilities
    mu_par  = r^T M_ij r  = f(r) + g(r),      mu_perp = f(r)
give samples of f and g; the diagonal blocks give the self mobility f(0).
Here M is measured with constrained solves of the library: prescribing the
velocity e_k of one marker component (all other markers at rest) returns
Lambda = M^-1 e_k, column k of M^-1 (FGMRES to 2e-9 in fp64: the forces
spread by one marker put about 1e5 into the fluid rows of a unit
right-hand side, which leaves a rounding floor near 1e-10); M is its
inverse.  Markers are kept at least 1.05 h apart (closer
markers are refused as overlapping bodies), so the pair data start at r = h.

Fitted forms (Appendix A):
  steady Stokes, x = r/h, periodic shift s = 2.84 / (6 pi eta l):
    ft(x) = 8 pi eta r (f + s) = x / (3a/4h + b0 x^2)                x < 0.8
                               = b1 x e^{-b2 x} + (b3 x^2 + x^4) / (1 + b4 x^2 + x^4)
    gt(x) = 8 pi eta r g       = x^3 / (b5 + b6 x^2 + x^3)
    a from the measured self mobility f(0) = 1/(6 pi eta a) - s; b0 so that
    the two branches of ft meet at x = 0.8 (no pair is closer than h).
  finite viscous CFL number beta = eta dt / (rho h^2):
    phi0(beta) = eta h f(0) / beta = (1 + z1 sqrt(beta) + z2 beta)
                                     / (z0 + z3 beta + 6 pi (a/h) z2 beta^2),
    z0 = 3 V_m / (2 h^3) fixed by the inviscid self mobility (the paper's
    printed z0 is the reciprocal, which would contradict its own inviscid
    limit); per tabulated beta
    f(r) = -(beta/(eta h)) ft_b(x) / (4 pi x^3),  g(r) = (beta/(eta h)) 3 gt_b(x) / (4 pi x^3),
    ft_b = phi0 (-4 pi x^3 + a4 [x^5 - x^7 e^{-a3 x/sqrt(beta)} / (2 beta)])
           / (1 + a0 x + a1 x^2 + a2 x^3 + a4 phi0 x^5)
           + (a5 x^4 e^{-a6 x} + a7 x^4) / (1 + a8 x^3 + a9 x^5),
    gt_b = phi0 b5 [x^5 + x^7 e^{-b0 x/sqrt(beta)} / (6 beta)]
           / (1 + b1 x + b2 x^2 + b3 x^3 + b4 x^4 + b5 phi0 x^5).
    The inviscid end of the table is beta = 0.01 (the solver needs eta > 0);
    smaller beta use that row, larger than the last row the steady fit; in
    between, the library blends the two rows' fitted functions linearly in
    beta (Appendix A interpolates the coefficients, which for independently
    fitted rational forms is not a blend of the functions).

The table is written to csrc/mobility_fit_4pt.inc and compiled into the
library; params.mobility = IBR_MOB_FITTED selects it.
"""
import math
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "mobility_fit_4pt.inc")

# the paper's table (its inviscid row measured at 0.01), with rows added between
# its decades: the fitted functions change too much over a decade of beta for
# a linear blend between two rows
BETAS = (0.01, 0.1, 0.25, 0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0, 500.0, 1000.0)
VM_OVER_H3 = (8.0 / 3.0) ** 3          # four-point marker volume: squared weights sum to 3/8 per dimension
Z0 = 1.5 * VM_OVER_H3                  # phi0(0) = 2 h^3 / (3 V_m) = 1 / z0
SHIFT_3D = 2.84


# ---------------------------------------------------------------- fitted forms
def ft_steady(x, ah, b):
    b0, b1, b2, b3, b4 = b[:5]
    x = np.asarray(x, dtype=np.float64)
    near = x / (0.75 * ah + b0 * x * x)
    far = b1 * x * np.exp(-b2 * x) + (b3 * x ** 2 + x ** 4) / (1.0 + b4 * x ** 2 + x ** 4)
    return np.where(x < 0.8, near, far)


def gt_steady(x, b):
    b5, b6 = b[5], b[6]
    x = np.asarray(x, dtype=np.float64)
    return x ** 3 / (b5 + b6 * x ** 2 + x ** 3)


def phi0(beta, z, ah):
    z1, z2, z3 = z
    beta = np.asarray(beta, dtype=np.float64)
    return (1.0 + z1 * np.sqrt(beta) + z2 * beta) / (Z0 + z3 * beta + 6.0 * math.pi * ah * z2 * beta ** 2)


def ft_beta(x, beta, ph, a):
    a0, a1, a2, a3, a4, a5, a6, a7, a8, a9 = a
    x = np.asarray(x, dtype=np.float64)
    num = -4.0 * math.pi * x ** 3 + a4 * (x ** 5 - x ** 7 * np.exp(-a3 * x / math.sqrt(beta)) / (2.0 * beta))
    den = 1.0 + a0 * x + a1 * x ** 2 + a2 * x ** 3 + a4 * ph * x ** 5
    return ph * num / den + (a5 * x ** 4 * np.exp(-a6 * x) + a7 * x ** 4) / (1.0 + a8 * x ** 3 + a9 * x ** 5)


def gt_beta(x, beta, ph, b):
    b0, b1, b2, b3, b4, b5 = b
    x = np.asarray(x, dtype=np.float64)
    num = ph * b5 * (x ** 5 + x ** 7 * np.exp(-b0 * x / math.sqrt(beta)) / (6.0 * beta))
    return num / (1.0 + b1 * x + b2 * x ** 2 + b3 * x ** 3 + b4 * x ** 4 + b5 * ph * x ** 5)


# ---------------------------------------------------------------- fits
def fit_steady(x, par, perp, self_mean, eta, h, L):
    """(a/h, b0..b6) from steady pair data (x = r/h, mu_par, mu_perp) and the
    mean self mobility."""
    from scipy.optimize import least_squares
    s = SHIFT_3D / (6.0 * math.pi * eta * L)
    ah = 1.0 / (6.0 * math.pi * eta * (self_mean + s)) / h
    r = x * h
    ft = 8.0 * math.pi * eta * r * (perp + s)
    gt = 8.0 * math.pi * eta * r * (par - perp)
    far = x >= 0.8
    # bounds: the bump b1 x e^{-b2 x} decays (b2 > 0) and no denominator
    # vanishes (1 + b4 x^2 + x^4 > 0 needs b4 > -2; b5, b6 >= 0)
    rf = least_squares(lambda p: ft_steady(x[far], ah, np.r_[0.0, p]) - ft[far], [0.1, 0.5, 0.5, 0.0],
                       bounds=([-10.0, 1e-3, -10.0, -1.9], [10.0, 10.0, 10.0, 100.0]))
    rg = least_squares(lambda p: gt_steady(x, np.r_[np.zeros(5), p]) - gt, [1.0, 1.0],
                       bounds=([0.0, 0.0], [1e3, 1e3]))
    b1, b2, b3, b4 = rf.x
    # b0 from continuity of ft at x = 0.8
    fx = ft_steady(0.8, ah, [0.0, b1, b2, b3, b4])
    b0 = (0.8 / fx - 0.75 * ah) / 0.64
    return ah, np.array([b0, b1, b2, b3, b4, rg.x[0], rg.x[1]])


def fit_phi0(betas, phis, ah):
    from scipy.optimize import least_squares
    betas = np.asarray(betas)
    phis = np.asarray(phis)
    r = least_squares(lambda z: (phi0(betas, z, ah) - phis) / phis, [0.0, 0.3, 40.0])
    return r.x


# Bounds of the finite-beta coefficients: every denominator coefficient is
# non-negative (no pole at any distance), the decay rates a3, a6, b0 and the
# far-field weights a4, b5 positive, and all magnitudes below 1e3 (the
# rational forms are otherwise free to scale numerator and denominator
# together without bound).
LB_A = [0.0, 0.0, 0.0, 1e-3, 1e-6, -1e3, 1e-3, -1e3, 0.0, 0.0]
UB_A = [1e3, 1e3, 1e3, 1e2, 1e3, 1e3, 1e2, 1e3, 1e3, 1e3]
LB_B = [1e-3, 0.0, 0.0, 0.0, 0.0, 1e-6]
UB_B = [1e2, 1e3, 1e3, 1e3, 1e3, 1e3]


def fit_beta(x, par, perp, beta, eta, h, ph, prev=None):
    """(a0..a9, b0..b5) for one beta from pair data, within the bounds
    above; prev, the parameters of a neighbouring beta, is tried as a second
    starting point (the better fit is kept)."""
    from scipy.optimize import least_squares
    pre = beta / (eta * h)
    ft = -perp * 4.0 * math.pi * x ** 3 / pre
    gt = (par - perp) * 4.0 * math.pi * x ** 3 / (3.0 * pre)

    def best(fun, starts, lb, ub):
        with np.errstate(over="ignore", invalid="ignore"):
            fits = [least_squares(fun, np.clip(p0, lb, ub), bounds=(lb, ub), max_nfev=20000) for p0 in starts]
        return min(fits, key=lambda r: r.cost).x

    sa = [np.array([1, 1, 1, 1, 1, 0, 1, 0, 1, 1.0])]
    sb = [np.ones(6)]
    if prev is not None:
        sa.append(np.asarray(prev[0], dtype=np.float64))
        sb.append(np.asarray(prev[1], dtype=np.float64))
    a = best(lambda p: (ft_beta(x, beta, ph, p) - ft) / (np.abs(ft) + 0.05), sa, LB_A, UB_A)
    b = best(lambda p: (gt_beta(x, beta, ph, p) - gt) / (np.abs(gt) + 0.05), sb, LB_B, UB_B)
    return a, b


def pair_stats(M, R, L):
    """Pair data of a measured mobility M (dN x dN, markers R [N][d]):
    distances r, mu_par, mu_perp for every pair i < j, self mobilities."""
    N, d = R.shape
    i, j = np.triu_indices(N, 1)
    dr = R[i] - R[j]
    dr -= L * np.round(dr / L)
    r = np.linalg.norm(dr, axis=1)
    rh = dr / r[:, None]
    B = M.reshape(N, d, N, d)[i, :, j, :]
    par = np.einsum("pa,pab,pb->p", rh, B, rh)
    perp = (np.trace(B, axis1=1, axis2=2) - par) / (d - 1)
    self_ = np.array([np.trace(M[d * k:d * k + d, d * k:d * k + d]) / d for k in range(N)])
    return r, par, perp, self_


def cloud(seed, N, L, h, min_dist=1.05, side=0.125, dim=3):
    """N random markers in a cube (square) of side side * L at the box
    centre, at least min_dist h apart."""
    rng = np.random.default_rng(seed)
    c = np.full(dim, L / 2)
    R = []
    while len(R) < N:
        p = c + rng.uniform(-0.5 * side * L, 0.5 * side * L, dim)
        if all(np.linalg.norm(p - q) >= min_dist * h for q in R):
            R.append(p)
    return np.array(R)


# ---------------------------------------------------------------- measurement (GPU)
def measure(R, n, h, rho, eta, dt):
    """M of the marker cloud R from dN constrained solves.  For the columns of
    marker k, marker k is one body and the other N - 1 markers a second one
    at rest: the second body's block of the approximate mobility then covers
    their interactions, which keeps FGMRES short (with one body per marker
    the preconditioner sees only self mobilities and needs thousands of
    iterations)."""
    from . import ibr
    N, d = R.shape
    nrot = 3 if d == 3 else 1
    s = ibr.Solver(dim=d, n=n, h=h, rho=rho, eta=eta, dt=dt, rtol=2e-9, max_iters=2000, restart=200,
                   precision=ibr.FP64, graphs=0, mobility=ibr.MOB_ANALYTIC)
    Minv = np.zeros((d * N, d * N))
    t0 = time.perf_counter()
    for k in range(N):
        order = np.r_[np.delete(np.arange(N), k), k]
        Rk = R[order]
        s.set_bodies(Rk, np.array([0, N - 1, N]), np.vstack([Rk[:-1].mean(axis=0), Rk[-1]]))
        for a in range(d):
            U = np.zeros((2, d))
            U[1, a] = 1.0
            s.set_velocities(U, np.zeros((2, nrot)))
            s.solve()
            col = np.zeros((N, d))
            col[order] = s.solution().lam
            Minv[:, d * k + a] = col.reshape(-1)
        if (k + 1) % 20 == 0:
            print("  %d / %d markers, %.1f s" % (k + 1, N, time.perf_counter() - t0), flush=True)
    s.close()
    Minv = 0.5 * (Minv + Minv.T)
    return np.linalg.inv(Minv)


def write_table(path, ah, bst, z, rows):
    def fmt(v):
        return ", ".join("%.17g" % x for x in v)
    lines = ["// Fitted approximate mobility of the four-point kernel (forms of the",
             "// paper's Appendix A, Sec. 4.2 fitting procedure); generated by",
             "// paper_1505_07865_amd/mobility_fit.py from pair mobilities measured with",
             "// this library's solver (64^3, two clouds of 120 markers):",
             "//   python -m paper_1505_07865_amd.mobility_fit --measure-only --pairs P.npz   (GPU)",
             "//   python -m paper_1505_07865_amd.mobility_fit --fit-only --pairs P.npz[,Q.npz]",
             "// Do not edit.",
             "constexpr int kFitRows = %d;" % len(rows),
             "constexpr double kFitAh = %.17g;" % ah,
             "constexpr double kFitSteady[7] = {%s};" % fmt(bst),
             "constexpr double kFitZ[3] = {%s};" % fmt(z),
             "constexpr double kFitBeta[%d] = {%s};" % (len(rows), fmt([r[0] for r in rows])),
             "constexpr double kFitA[%d][10] = {%s};" % (len(rows), ", ".join("{%s}" % fmt(r[1]) for r in rows)),
             "constexpr double kFitB[%d][6] = {%s};" % (len(rows), ", ".join("{%s}" % fmt(r[2]) for r in rows))]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def measure_clouds(clouds, n, h, rho, eta, dt, L):
    """Pair data (x = r/h, mu_par, mu_perp) and self mobilities of several
    clouds, concatenated."""
    parts = [pair_stats(measure(R, n, h, rho, eta, dt), R, L) for R in clouds]
    return tuple(np.concatenate([p[k] for p in parts]) for k in range(4))


def measure_all(n=64, N=120, seed=0, betas=BETAS, steady=True):
    """Pair data of two clouds of N markers, steady and at the given betas:
    one cloud in a cube of side l/8 (the paper's, dense pairs from h to
    14 h) and one of side l/4 (pairs out to about 27 h).  Returns
    {key: (x, mu_par, mu_perp, self)} with key "steady" or the beta."""
    h = 1.0 / n
    L = n * h
    clouds = [cloud(seed, N, L, h), cloud(seed + 1, N, L, h, side=0.25)]
    data = {}
    if steady:
        print("steady: 2 clouds of %d markers" % N, flush=True)
        r, par, perp, self_ = measure_clouds(clouds, n, h, 0.0, 1.0, 0.0, L)
        data["steady"] = (r / h, par, perp, self_)
    for beta in betas:
        # rho = 1, dt = 1: eta = beta h^2
        print("beta %g" % beta, flush=True)
        r, par, perp, self_ = measure_clouds(clouds, n, h, 1.0, beta * h * h, 1.0, L)
        data[beta] = (r / h, par, perp, self_)
    return data


def save_pairs(path, data, n):
    np.savez(path, n=n, **{("steady" if k == "steady" else "beta%r" % k): np.stack(v[:3]) for k, v in data.items()},
             **{("self_steady" if k == "steady" else "self_beta%r" % k): v[3] for k, v in data.items()})


def load_pairs(paths, betas=BETAS):
    """Pair data from one or more files written by save_pairs (comma-separated
    paths; later files add keys)."""
    data, n = {}, None
    for path in paths.split(","):
        z = np.load(path)
        n = int(z["n"])
        if "steady" in z.files:
            data["steady"] = tuple(z["steady"]) + (z["self_steady"],)
        for beta in betas:
            if "beta%r" % beta in z.files:
                data[beta] = tuple(z["beta%r" % beta]) + (z["self_beta%r" % beta],)
    missing = [b for b in ("steady",) + tuple(betas) if b not in data]
    if missing:
        raise ValueError("pair data missing for %s" % missing)
    return data, n


def binned(x, par, perp, xmax, nbins=160):
    """Pair data averaged in bins of x (uniform in log x from the closest pair
    to xmax): the fitted functions are smooth, and the averages carry the
    data's trend without its scatter at a hundredth of the cost.  Returns the
    bins' mean x, mu_par, mu_perp and their pair counts."""
    k = x <= xmax
    x, par, perp = x[k], par[k], perp[k]
    edges = np.geomspace(x.min() * (1 - 1e-9), xmax * (1 + 1e-9), nbins + 1)
    idx = np.clip(np.searchsorted(edges, x) - 1, 0, nbins - 1)
    cnt = np.bincount(idx, minlength=nbins).astype(np.float64)
    keep = cnt > 0
    mean = lambda v: (np.bincount(idx, weights=v, minlength=nbins)[keep] / cnt[keep])
    return mean(x), mean(par), mean(perp), cnt[keep]


def fit_all(data, n, xmax=16.0):
    """The table from measured pair data.  Pairs farther than xmax h (a
    quarter of the 64^3 box) are left out: there the box's periodic images
    change the pair mobility by more than the constant shift accounts for."""
    h = 1.0 / n
    L = n * h
    x, par, perp, self_ = data["steady"]
    xb, pb, qb, _ = binned(x, par, perp, xmax)
    ah, bst = fit_steady(xb, pb, qb, self_.mean(), 1.0, h, L)
    print("  steady: a/h %.4f  b %s" % (ah, np.array2string(bst, precision=4)), flush=True)
    # a periodic box with inertia has a mean mode: a force F on one marker moves
    # the whole fluid with F dt / (rho l^3), which adds dt / (rho l^3) to f
    # (self term included) whatever the distance; it belongs to the box, not
    # to the kernel, so it leaves the data here (the library adds it back for
    # periodic boxes; rho = dt = 1)
    mean_mode = 1.0 / L ** 3
    phis = [(data[b][3].mean() - mean_mode) * h ** 3 for b in BETAS]   # eta h f(0) / beta with rho = dt = 1
    z = fit_phi0(BETAS, phis, ah)
    print("  phi0: z %s" % np.array2string(z, precision=4), flush=True)
    rows = []
    prev = None
    for beta in BETAS[::-1]:
        x, par, perp, _ = data[beta]
        xb, pb, qb, _ = binned(x, par - mean_mode, perp - mean_mode, xmax)
        t0 = time.perf_counter()
        a, b = fit_beta(xb, pb, qb, beta, beta * h * h, h, float(phi0(beta, z, ah)), prev)
        print("  beta %g fitted (%.1f s)" % (beta, time.perf_counter() - t0), flush=True)
        rows.insert(0, (beta, a, b))
        prev = (a, b)
    return ah, bst, z, rows


# ---------------------------------------------------------------- two dimensions (Appendix B)
# The paper's 2D table is beta in {0, 0.1, 0.25, 0.5, 1, 5, 10}; the inviscid row
# is measured at 0.01 and a row at 2 is added; above 10 the steady fit applies.
BETAS_2D = (0.01, 0.1, 0.25, 0.5, 1.0, 2.0, 5.0, 10.0)
CV_2D = (8.0 / 3.0) ** 2               # four-point marker area V_m / h^2
Z0_2D = 1.0 / (2.0 * CV_2D)            # phi0(0) = eta f_0(0) / beta = h^2 / (2 V_m)
HASIMOTO_2D = 3.708                    # f(0) = ln(l / (3.708 a)) / (4 pi eta), periodic square
TABLE_2D = os.path.join(HERE, "csrc", "mobility_fit_4pt_2d.inc")


def ft2_steady(x, c):
    """-(4 pi eta)(f(r) - f(0)), coefficients a0..a4 = c[0:5]."""
    a0, a1, a2, a3, a4 = c[:5]
    x = np.asarray(x, dtype=np.float64)
    lx = np.log(np.maximum(x, 1e-300))
    return (a0 * x ** 2 + a1 * x ** 3 + a2 * x ** 3 * lx) / (1.0 + a3 * x + a4 * x ** 2 + a2 * x ** 3)


def gt2_steady(x, c):
    """(4 pi eta) g(r), coefficients b0..b3 = c[5:9]."""
    b0, b1, b2, b3 = c[5:9]
    x = np.asarray(x, dtype=np.float64)
    return (b0 * x ** 2 + b1 * x ** 3) / (1.0 + b2 * x + b3 * x ** 2 + b1 * x ** 3)


def phi0_2d(beta, z):
    """eta f(0) / beta, z = (z1, z2, z3, z4)."""
    z1, z2, z3, z4 = z
    beta = np.asarray(beta, dtype=np.float64)
    return (Z0_2D + z1 * beta ** 3 * np.log(beta)) / (1.0 + z2 * beta + z3 * beta ** 2 + z4 * beta ** 4)


def ft2_beta(x, beta, c):
    """f~ with f(r) = -(beta / (2 pi eta x^2)) f~; c = (a0, a1, a2, a3, p1, b1, b2, ...)."""
    a0, a1, a2, a3, p1, b1, b2 = c[:7]
    x = np.asarray(x, dtype=np.float64)
    lx = np.log(np.maximum(x, 1e-300))
    vis = x ** 3 * lx / (beta * (a0 + 2.0 * x)) * np.exp(-p1 * x / math.sqrt(beta))
    return vis + (a1 * x ** 2 + a2 * x ** 3 + a3 * x ** 4) / (1.0 + b1 * x ** 2 + b2 * x ** 3 + a3 * x ** 4)


def gt2_beta(x, beta, c):
    """g~ with g(r) = (beta / (pi eta x^2)) g~; c[7:13] = (c0, c1, c2, c3, p2, p3)."""
    c0, c1, c2, c3, p2, p3 = c[7:13]
    x = np.asarray(x, dtype=np.float64)
    vis = x ** 3 / (beta * (c0 + 4.0 * x)) * np.exp(-p2 * x / math.sqrt(beta))
    return vis + x ** 3 / (np.exp(-p3 * x) * (c1 + c2 * x + c3 * x ** 2) + x ** 3)


# bounds: every denominator positive at every distance; decay rates positive
LB_2S = [-1e3, -1e3, 1e-6, 0.0, 0.0, -1e3, 1e-6, 0.0, 0.0]
UB_2S = [1e3, 1e3, 1e3, 1e3, 1e3, 1e3, 1e3, 1e3, 1e3]
LB_2B = [0.0, -1e3, -1e3, 1e-6, 1e-3, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1e-3, 1e-3]
UB_2B = [1e3, 1e3, 1e3, 1e3, 1e2, 1e3, 1e3, 1e3, 1e3, 1e3, 1e3, 1e2, 1e2]
LB_Z2 = [-1.0, -1e3, -1e3, 0.0]
UB_Z2 = [1.0, 1e3, 1e3, 1e3]


def fit_steady_2d(x, par, perp, self_mean, eta, h, L):
    """(a/h, a0..a4, b0..b3) from steady 2D pair data."""
    from scipy.optimize import least_squares
    ah = L / (HASIMOTO_2D * math.exp(4.0 * math.pi * eta * self_mean)) / h
    ft = -4.0 * math.pi * eta * (perp - self_mean)
    gt = 4.0 * math.pi * eta * (par - perp)
    w = 1.0 / (np.abs(ft) + 0.05)
    rf = least_squares(lambda q: (ft2_steady(x, np.r_[q, np.zeros(4)]) - ft) * w, [1.0, 1.0, 1.0, 1.0, 1.0],
                       bounds=(LB_2S[:5], UB_2S[:5]))
    wg = 1.0 / (np.abs(gt) + 0.05)
    rg = least_squares(lambda q: (gt2_steady(x, np.r_[np.zeros(5), q]) - gt) * wg, [1.0, 1.0, 1.0, 1.0],
                       bounds=(LB_2S[5:], UB_2S[5:]))
    return ah, np.r_[rf.x, rg.x]


def phi0_2d_positive(z, lo=1e-4, hi=1e5):
    """Numerator and denominator of phi0_2d positive over beta in [lo, hi]."""
    b = np.geomspace(lo, hi, 4000)
    num = Z0_2D + z[0] * b ** 3 * np.log(b)
    den = 1.0 + z[1] * b + z[2] * b ** 2 + z[3] * b ** 4
    return bool(np.all(num > 0) and np.all(den > 0))


def fit_phi0_2d(betas, phis):
    """z1..z4 from the self mobilities; several starts, the best fit whose
    numerator and denominator stay positive (a sign change would put a pole
    or a negative self mobility at some beta)."""
    from scipy.optimize import least_squares
    betas = np.asarray(betas)
    phis = np.asarray(phis)
    fits = []
    for z0 in ([0.01, 1.0, 1.0, 0.01], [0.001, 1.3, -0.3, 0.01], [0.05, 2.0, 0.0, 0.1]):
        r = least_squares(lambda z: (phi0_2d(betas, z) - phis) / phis, np.clip(z0, LB_Z2, UB_Z2),
                          bounds=(LB_Z2, UB_Z2))
        if phi0_2d_positive(r.x):
            fits.append(r)
    if not fits:
        raise RuntimeError("no 2D phi0 fit keeps its numerator and denominator positive")
    return min(fits, key=lambda r: r.cost).x


def fit_beta_2d(x, par, perp, beta, h, prev=None):
    """The 13 coefficients of one 2D row from pair data (rho = dt = 1, the
    box's mean mode removed)."""
    from scipy.optimize import least_squares
    ft = -2.0 * math.pi * x ** 2 * h ** 2 * perp
    gt = math.pi * x ** 2 * h ** 2 * (par - perp)

    def best(fun, starts, lb, ub):
        with np.errstate(over="ignore", invalid="ignore"):
            fits = [least_squares(fun, np.clip(p0, lb, ub), bounds=(lb, ub), max_nfev=20000) for p0 in starts]
        return min(fits, key=lambda r: r.cost).x

    sa = [np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])]
    sb = [np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0])]
    if prev is not None:
        sa.append(np.asarray(prev[:7]))
        sb.append(np.asarray(prev[7:]))
    a = best(lambda q: (ft2_beta(x, beta, np.r_[q, np.zeros(6)]) - ft) / (np.abs(ft) + 0.05), sa, LB_2B[:7],
             UB_2B[:7])
    b = best(lambda q: (gt2_beta(x, beta, np.r_[np.zeros(7), q]) - gt) / (np.abs(gt) + 0.05), sb, LB_2B[7:],
             UB_2B[7:])
    return np.r_[a, b]


def measure_all_2d(n=256, N=120, seed=0, betas=BETAS_2D, steady=True):
    """2D pair data: two clouds of N markers in squares of side l/8 and l/4."""
    h = 1.0 / n
    L = n * h
    clouds = [cloud(seed, N, L, h, dim=2), cloud(seed + 1, N, L, h, side=0.25, dim=2)]
    data = {}
    if steady:
        print("2D steady: 2 clouds of %d markers" % N, flush=True)
        r, par, perp, self_ = measure_clouds(clouds, n, h, 0.0, 1.0, 0.0, L)
        data["steady"] = (r / h, par, perp, self_)
    for beta in betas:
        print("2D beta %g" % beta, flush=True)
        r, par, perp, self_ = measure_clouds(clouds, n, h, 1.0, beta * h * h, 1.0, L)
        data[beta] = (r / h, par, perp, self_)
    return data


def fit_all_2d(data, n, xmax=None):
    """The 2D table from measured pair data (pairs within a quarter of the box)."""
    h = 1.0 / n
    L = n * h
    xmax = xmax or n / 4.0
    x, par, perp, self_ = data["steady"]
    xb, pb, qb, _ = binned(x, par, perp, xmax)
    ah, cst = fit_steady_2d(xb, pb, qb, self_.mean(), 1.0, h, L)
    print("  2D steady: a/h %.4f  c %s" % (ah, np.array2string(cst, precision=4)), flush=True)
    mean_mode = 1.0 / L ** 2             # dt / (rho l^2) with rho = dt = 1
    phis = [(data[b][3].mean() - mean_mode) * h ** 2 for b in BETAS_2D]   # eta f(0) / beta
    z = fit_phi0_2d(BETAS_2D, phis)
    print("  2D phi0: z %s" % np.array2string(z, precision=4), flush=True)
    rows = []
    prev = None
    for beta in BETAS_2D[::-1]:
        x, par, perp, _ = data[beta]
        xb, pb, qb, _ = binned(x, par - mean_mode, perp - mean_mode, xmax)
        t0 = time.perf_counter()
        c = fit_beta_2d(xb, pb, qb, beta, h, prev)
        print("  2D beta %g fitted (%.1f s)" % (beta, time.perf_counter() - t0), flush=True)
        rows.insert(0, (beta, c))
        prev = c
    return ah, cst, z, rows


def write_table_2d(path, ah, cst, z, rows):
    def fmt(v):
        return ", ".join("%.17g" % x for x in v)
    lines = ["// Fitted approximate mobility of the four-point kernel in two dimensions",
             "// (forms of the paper's Appendix B, Sec. 4.2 fitting procedure); generated",
             "// by paper_1505_07865_amd/mobility_fit.py from pair mobilities measured with",
             "// this library's solver (256^2, two clouds of 120 markers):",
             "//   python -m paper_1505_07865_amd.mobility_fit --dim 2 --measure-only --pairs P.npz   (GPU)",
             "//   python -m paper_1505_07865_amd.mobility_fit --dim 2 --fit-only --pairs P.npz",
             "// Do not edit.",
             "constexpr int kFit2Rows = %d;" % len(rows),
             "constexpr double kFit2Ah = %.17g;" % ah,
             "constexpr double kFit2Steady[9] = {%s};" % fmt(cst),
             "constexpr double kFit2Z[4] = {%s};" % fmt(z),
             "constexpr double kFit2Beta[%d] = {%s};" % (len(rows), fmt([r[0] for r in rows])),
             "constexpr double kFit2Row[%d][13] = {%s};" % (len(rows), ", ".join("{%s}" % fmt(r[1]) for r in rows))]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(n=64, N=120, seed=0, out=TABLE, pairs=None, measure_only=False, fit_only=False, betas=BETAS,
         steady=True, dim=3):
    if fit_only:
        data, n = load_pairs(pairs, BETAS if dim == 3 else BETAS_2D)
    else:
        data = measure_all(n, N, seed, betas, steady) if dim == 3 else measure_all_2d(n, N, seed, betas, steady)
        if pairs:
            save_pairs(pairs, data, n)
            print("wrote", pairs, flush=True)
        if measure_only:
            return
    if dim == 3:
        ah, bst, z, rows = fit_all(data, n)
        write_table(out, ah, bst, z, rows)
    else:
        ah, cst, z, rows = fit_all_2d(data, n)
        write_table_2d(out, ah, cst, z, rows)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=3, choices=(2, 3))
    ap.add_argument("--out", default=None, help="table file to write (default: the library's table)")
    ap.add_argument("--markers", type=int, default=120)
    ap.add_argument("--n", type=int, default=None, help="grid (default 64 in 3D, 256 in 2D)")
    ap.add_argument("--pairs", default=None, help="pair data file (.npz) to write after measuring, or to fit")
    ap.add_argument("--measure-only", action="store_true", help="measure and write --pairs, no fit")
    ap.add_argument("--fit-only", action="store_true",
                    help="fit the pair data in --pairs (comma-separated files; no GPU)")
    ap.add_argument("--betas", default=None, help="measure: comma-separated subset of the table's betas")
    ap.add_argument("--no-steady", action="store_true", help="measure: skip the steady data")
    a = ap.parse_args()
    table = BETAS if a.dim == 3 else BETAS_2D
    betas = table if a.betas is None else tuple(float(b) for b in a.betas.split(","))
    main(n=a.n or (64 if a.dim == 3 else 256), N=a.markers, out=a.out or (TABLE if a.dim == 3 else TABLE_2D),
         pairs=a.pairs, measure_only=a.measure_only, fit_only=a.fit_only, betas=betas, steady=not a.no_steady,
         dim=a.dim)
