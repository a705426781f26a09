"""No-slip walls at both ends of the last axis: the slit channel of Sec. 7
(flow between two parallel walls, periodic along the others), with the
boundary treatment of the appendix on physical boundary conditions.

TEST INFRASTRUCTURE ONLY (see the package header).

Geometry.  Periodic along every axis but the last one (z in 3D, y in 2D),
which is array axis 0 of a scalar slab (axes are ordered (z, y, x) / (y, x)).
No-slip walls sit at z = 0 and z = L = n h.  Storage is that of the periodic
box:
  * tangential components (alpha < d-1) and the pressure live at cell centres
    along z, (k + 1/2) h, k = 0..n-1: all n values are unknowns;
  * the normal component lives on faces z = k h, k = 0..n-1; face 0 lies on
    the wall (face n is the other wall) and holds 0: it is not an unknown.

Extension E (the appendix fills ghost values by a mirror image with a sign):
  * tangential velocity (no slip, homogeneous Dirichlet): the ghost cell at
    -1-m mirrors cell m with the sign reversed, the ghost at n+m mirrors n-1-m;
  * normal velocity: ghost face -m mirrors face m with the sign reversed,
    ghost n+m mirrors n-m; the wall faces 0 and n are 0;
  * pressure inside the preconditioner's Poisson problem (homogeneous
    Neumann): the ghost mirrors the interior value with the sign kept.  The
    appendix's text gives the Neumann mirror a minus sign too; that cannot be
    a Neumann condition (it is the Dirichlet one), so the sign kept is the
    reading taken here.
The fluid operators use the same E: the Laplacian of a tangential component
next to a wall sees the reversed mirror value, the normal component's rows at
the wall faces are not equations (the operator returns 0 there), the
gradient vanishes on the wall faces, and the divergence uses the wall faces'
zero flux.  Interpolation is J = J0 E and spreading S = E^T S0 (standard
kernel weights on the extended lattice, ghost taps folded back with the
mirror's sign; taps on the wall faces are dropped), so the two stay adjoint
and an interpolated tangential velocity vanishes on the wall.

With walls the velocity block has no null space (Dirichlet along z), so
steady Stokes needs no mean constraint: S is used as is (no S'), and only the
pressure keeps its constant mode (fixed by a zero mean).

``solve`` is the exact solution operator of the wall-bounded MAC Stokes
system: a Fourier transform along the periodic axes leaves, for every
wavevector, a small dense system along z, assembled here from the stencils
and solved by LAPACK (the pressure gauge by a bordered row).  ``vcycle`` is
the multigrid V-cycle of the preconditioner with the walls' boundary rules;
the paper leaves the cycle to the cited solvers, so its transfers are a
reading: cell-centred for the tangential components and the pressure,
vertex-centred along z for the normal component (whose values sit on the
walls' lattice planes).
"""
import itertools
import math
from dataclasses import dataclass

import numpy as np

from . import constrained, ib, kernel

CELL_DIR = "cell_dir"   # tangential velocity: mirror with the sign reversed
FACE_DIR = "face_dir"   # normal velocity: wall faces pinned to zero
CELL_NEU = "cell_neu"   # pressure: mirror with the sign kept


def kinds(d):
    """Boundary kind of each velocity component along z."""
    return [CELL_DIR] * (d - 1) + [FACE_DIR]


# ---------------------------------------------------------------- extension E along z
def extend(j, n, kind):
    """(interior index, sign) that ghost or interior index j stands for along
    z, or (None, 0) for a wall face (value 0)."""
    if kind == FACE_DIR:
        if j == 0 or j == n:
            return None, 0
        if j < 0:
            return -j, -1
        if j > n:
            return 2 * n - j, -1
        return j, 1
    sgn = -1 if kind == CELL_DIR else 1
    if j < 0:
        return -1 - j, sgn
    if j >= n:
        return 2 * n - 1 - j, sgn
    return j, 1


def znbr(x, off, kind):
    """y with y_k = (E x)_{k + off} along array axis 0 (off = +-1)."""
    n = x.shape[0]
    y = np.empty_like(x)
    for k in range(n):
        j, s = extend(k + off, n, kind)
        y[k] = 0.0 if j is None else s * x[j]
    return y


def pnbr(x, off, ax):
    """Periodic neighbour along array axis ax >= 1."""
    return np.roll(x, -off, axis=ax)


def lap(x, kind):
    """Dimensionless Laplacian with the walls' extension along z; the rows of
    the normal component's wall faces are 0."""
    out = (znbr(x, 1, kind) - x) + (znbr(x, -1, kind) - x)
    for ax in range(1, x.ndim):
        out = out + (pnbr(x, 1, ax) - x) + (pnbr(x, -1, ax) - x)
    if kind == FACE_DIR:
        out[0] = 0.0
    return out


def grad(p, h):
    """G pi on the faces; zero on the wall faces."""
    d = p.ndim
    out = []
    for a in range(d):
        ax = d - 1 - a
        if ax == 0:
            g = np.zeros_like(p)
            g[1:] = (p[1:] - p[:-1]) / h
        else:
            g = (p - pnbr(p, -1, ax)) / h
        out.append(g)
    return np.stack(out)


def div(v, h):
    """D v at cell centres; the wall faces carry no flux."""
    d = v.shape[0]
    out = np.zeros(v.shape[1:])
    for a in range(d):
        ax = d - 1 - a
        if ax == 0:
            up = np.zeros_like(v[a])
            up[:-1] = v[a][1:]
            lo = v[a].copy()
            lo[0] = 0.0
            out += (up - lo) / h
        else:
            out += (pnbr(v[a], 1, ax) - v[a]) / h
    return out


def stokes_apply(v, p, c0, eta, h):
    """[[A, G], [-D, 0]] (v, pi) with the walls; A = c0 - eta h^-2 L per component."""
    d = v.shape[0]
    ks = kinds(d)
    mv = np.stack([c0 * v[a] - eta / (h * h) * lap(v[a], ks[a]) for a in range(d)]) + grad(p, h)
    mv[d - 1][0] = 0.0
    return mv, -div(v, h)


# ---------------------------------------------------------------- J = J0 E, S = E^T S0
def taps_1d(pos, n, h, staggered, wall):
    """Indices [N, 4] and weights [N, 4] of the taps along one axis; along the
    wall axis the taps beyond a wall fold back with the mirror's sign and the
    taps on wall faces get weight 0 (index 0, harmless)."""
    s = pos / h - (0.0 if staggered else 0.5)
    base = np.floor(s).astype(np.int64) - 1
    j = base[:, None] + np.arange(4)[None, :]
    w = kernel.phi(s[:, None] - j)
    if not wall:
        return np.mod(j, n), w
    kind = FACE_DIR if staggered else CELL_DIR
    idx = np.zeros_like(j)
    wt = np.zeros_like(w)
    for m in range(j.shape[0]):
        for t in range(4):
            q, sg = extend(int(j[m, t]), n, kind)
            if q is not None:
                idx[m, t] = q
                wt[m, t] = sg * w[m, t]
    return idx, wt


def weights(R, n, h, alpha):
    N, d = R.shape
    idx1, w1 = [], []
    for beta in range(d):
        i, w = taps_1d(R[:, beta], n, h, staggered=(beta == alpha), wall=(beta == d - 1))
        idx1.append(i)
        w1.append(w)
    flat = np.zeros((N, 4 ** d), dtype=np.int64)
    wt = np.ones((N, 4 ** d))
    for t, combo in enumerate(itertools.product(range(4), repeat=d)):
        f = np.zeros(N, dtype=np.int64)
        for beta in reversed(range(d)):
            f = f * n + idx1[beta][:, combo[beta]]
        flat[:, t] = f
        for beta in range(d):
            wt[:, t] *= w1[beta][:, combo[beta]]
    return flat, wt


def all_weights(R, n, h):
    return [weights(R, n, h, a) for a in range(R.shape[1])]


def check_inside(R, L):
    """Markers must lie strictly between the walls."""
    z = np.asarray(R)[:, -1]
    if not (np.all(z > 0.0) and np.all(z < L)):
        raise ValueError("markers must lie strictly between the walls")


# ---------------------------------------------------------------- exact solve
def _mode_matrices(n, d, h, c0, eta):
    """Dense z-systems of every Fourier mode of the periodic axes, inverted.

    Unknowns per mode: the d-1 tangential components (n cells each), the
    normal component on faces 1..n-1, the pressure (n cells), and one border
    unknown for the pressure gauge (zero mean); the rows are the momentum
    equations, continuity, and the gauge row."""
    nt = d - 1
    size = nt * n + (n - 1) + n
    per = [np.fft.fftfreq(n, 1.0 / n)] * (d - 2) + [np.arange(n // 2 + 1)]
    # Laplacian along z
    Lc = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    Lc[0, 0] -= 1.0
    Lc[-1, -1] -= 1.0
    Lf = -2.0 * np.eye(n - 1) + np.eye(n - 1, k=1) + np.eye(n - 1, k=-1)
    # normal derivative pieces: Gz (faces 1..n-1 <- cells), Dz (cells <- faces 1..n-1)
    Gz = np.zeros((n - 1, n))
    for f in range(1, n):
        Gz[f - 1, f] = 1.0 / h
        Gz[f - 1, f - 1] = -1.0 / h
    Dz = np.zeros((n, n - 1))
    for c in range(n):
        if c + 1 <= n - 1:
            Dz[c, c] += 1.0 / h       # face c+1 is column c
        if c >= 1:
            Dz[c, c - 1] -= 1.0 / h   # face c is column c-1
    grids = np.meshgrid(*per, indexing="ij")
    shape = grids[0].shape
    inv = np.zeros(shape + (size + 1, size + 1), dtype=np.complex128)
    for idx in np.ndindex(*shape):
        th = [2.0 * np.pi * g[idx] / n for g in grids]   # per periodic array axis 1..d-1
        sig = sum(2.0 * np.cos(t) - 2.0 for t in th)
        K = np.zeros((size + 1, size + 1), dtype=np.complex128)
        po = nt * n + (n - 1)
        for a in range(nt):
            # component a varies along array axis d-1-a, i.e. periodic axis index d-2-a
            t = th[d - 2 - a]
            Ga = (1.0 - np.exp(-1j * t)) / h
            Da = (np.exp(1j * t) - 1.0) / h
            r = slice(a * n, (a + 1) * n)
            K[r, r] = c0 * np.eye(n) - eta / (h * h) * (Lc + sig * np.eye(n))
            K[r, po:po + n] = Ga * np.eye(n)
            K[po:po + n, r] = -Da * np.eye(n)
        zf = slice(nt * n, nt * n + n - 1)
        K[zf, zf] = c0 * np.eye(n - 1) - eta / (h * h) * (Lf + sig * np.eye(n - 1))
        K[zf, po:po + n] = Gz
        K[po:po + n, zf] = -Dz
        # gauge: the border unknown enters every continuity row; the last row fixes the mean
        if all(g[idx] == 0 for g in grids):
            K[po:po + n, size] = 1.0
            K[size, po:po + n] = 1.0
        else:
            K[size, size] = 1.0
        inv[idx] = np.linalg.inv(K)
    return inv


_CACHE = {}


def solve(f, hp, c0, eta, h, d):
    """Exact wall-bounded Stokes solve: A v + G pi = f, -D v = hp, mean pi = 0.

    f [..., d, n..] (the normal component's wall-face values are ignored), hp
    [..., n..] or None.  Returns (v, pi); v is 0 on the wall faces."""
    n = f.shape[-1]
    key = (n, d, h, c0, eta)
    if key not in _CACHE:
        _CACHE.clear()
        _CACHE[key] = _mode_matrices(n, d, h, c0, eta)
    inv = _CACHE[key]
    lead = f.shape[:-(d + 1)]
    fr = f.reshape((-1, d) + (n,) * d)
    hr = np.zeros((fr.shape[0],) + (n,) * d) if hp is None else np.asarray(hp).reshape((-1,) + (n,) * d)
    pax = tuple(range(2, d + 1))          # periodic axes of a [batch, z, ...] slab
    nt = d - 1
    size = nt * n + (n - 1) + n
    vs, ps = [], []
    for b in range(fr.shape[0]):
        comps = [np.fft.rfftn(fr[b, a][None], axes=pax)[0] for a in range(d)]
        hh = np.fft.rfftn(hr[b][None], axes=pax)[0]
        mshape = comps[0].shape[1:]
        rhs = np.zeros(mshape + (size + 1,), dtype=np.complex128)
        for a in range(nt):
            rhs[..., a * n:(a + 1) * n] = np.moveaxis(comps[a], 0, -1)
        rhs[..., nt * n:nt * n + n - 1] = np.moveaxis(comps[d - 1][1:], 0, -1)
        rhs[..., nt * n + n - 1:size] = np.moveaxis(hh, 0, -1)
        sol = np.einsum("...ij,...j->...i", inv, rhs)
        out = []
        full = [n] + [n] * (d - 1)
        for a in range(nt):
            out.append(np.fft.irfftn(np.moveaxis(sol[..., a * n:(a + 1) * n], -1, 0)[None], s=full[1:], axes=pax)[0])
        zn = np.zeros((n,) + mshape, dtype=np.complex128)
        zn[1:] = np.moveaxis(sol[..., nt * n:nt * n + n - 1], -1, 0)
        out.append(np.fft.irfftn(zn[None], s=full[1:], axes=pax)[0])
        pp = np.fft.irfftn(np.moveaxis(sol[..., nt * n + n - 1:size], -1, 0)[None], s=full[1:], axes=pax)[0]
        vs.append(np.stack(out))
        ps.append(pp)
    v = np.stack(vs).reshape(lead + (d,) + (n,) * d)
    p = np.stack(ps).reshape(lead + (n,) * d)
    return v, p


# ---------------------------------------------------------------- constrained system
class System(constrained.System):
    """The constrained system of eq. constrained_Stokes with the walls:
    S = E^T S0 (no S', no velocity mean), J = J0 E, exact wall-bounded
    Stokes solves."""

    def __init__(self, dim, n, h, c0, eta, R):
        self.d = dim
        self.n = n
        self.h = h
        self.c0 = c0
        self.eta = eta
        self.R = np.asarray(R, dtype=np.float64)
        check_inside(self.R, n * h)
        self.steady = c0 == 0.0
        self.W = all_weights(self.R, n, h)

    def spread(self, lam):
        return ib.spread(lam, self.R, self.n, self.h, self.W)

    def stokes(self, f, hp=None):
        return solve(f, hp, self.c0, self.eta, self.h, self.d)


def solve_problem(prob, g=None, hp=None, **kw):
    """Exact solution of a prescribed-motion problem between the walls."""
    c0 = 0.0 if prob.steady else prob.rho / prob.dt
    sysm = System(prob.dim, prob.n, prob.h, c0, prob.eta, prob.R)
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    return constrained.solve(sysm, g, hp, -V, prob.offsets, prob.centres, **kw)


def residual(sysm, v, p, lam, g, hp, W):
    """Blocks of b - K x of the wall-bounded system."""
    d, n = sysm.d, sysm.n
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    if hp is None:
        hp = np.zeros((n,) * d)
    rm, rc = stokes_apply(v, p, sysm.c0, sysm.eta, sysm.h)
    rm = g - (rm - sysm.spread(lam))
    rm[d - 1][0] = 0.0
    rc = hp - rc
    rl = W + sysm.interp(v)
    return rm, rc, rl


# ---------------------------------------------------------------- V-cycle with the walls
def _diag(shape, c0, c1, kind):
    """Diagonal of (c0 - c1 L) per cell: the mirror value of a boundary cell
    is the cell itself, with the sign of the mirror."""
    d = len(shape)
    dg = np.full(shape, c0 + 2.0 * d * c1)
    if kind != FACE_DIR:
        s = 1.0 if kind == CELL_DIR else -1.0
        dg[0] += s * c1
        dg[-1] += s * c1
    return dg


def _nbr_sum(x, kind):
    """Sum of the neighbours that are other unknowns (a boundary cell's mirror
    image is itself and sits in the diagonal instead)."""
    up = np.roll(x, -1, axis=0)
    dn = np.roll(x, 1, axis=0)
    if kind != FACE_DIR:
        up[-1] = 0.0
        dn[0] = 0.0
    s = up + dn
    for ax in range(1, x.ndim):
        s = s + pnbr(x, 1, ax) + pnbr(x, -1, ax)
    return s


def apply_op(x, c0, c1, kind):
    out = _diag(x.shape, c0, c1, kind) * x - c1 * _nbr_sum(x, kind)
    if kind == FACE_DIR:
        out[0] = 0.0
    return out


def smooth(x, b, c0, c1, kind, sweeps):
    par = np.indices(x.shape).sum(axis=0) % 2
    dg = _diag(x.shape, c0, c1, kind)
    for _ in range(sweeps):
        for colour in (0, 1):
            new = (b + c1 * _nbr_sum(x, kind)) / dg
            x = np.where(par == colour, new, x)
            if kind == FACE_DIR:
                x[0] = 0.0
    return x


def _pair_mean(x, ax):
    """Average of the 2 fine points of each coarse point along axis ax."""
    shp = list(x.shape)
    shp[ax] //= 2
    shp.insert(ax + 1, 2)
    return x.reshape(shp).mean(axis=ax + 1)


def restrict(r, kind):
    """Cell kinds: average of the 2^d children.  Normal component: its faces
    are vertex-centred along z (coarse face K on fine face 2K), so z takes
    full weighting 1/4, 1/2, 1/4 of fine faces 2K-1, 2K, 2K+1 (the coarse wall
    face stays 0); the periodic axes average their 2 children."""
    out = r
    for ax in range(1, r.ndim):
        out = _pair_mean(out, ax)
    if kind != FACE_DIR:
        return _pair_mean(out, 0)
    n = r.shape[0]
    rz = np.zeros((n // 2,) + out.shape[1:])
    for K in range(1, n // 2):
        rz[K] = 0.25 * out[2 * K - 1] + 0.5 * out[2 * K] + 0.25 * out[2 * K + 1]
    return rz


def _prolong_periodic_axis(x, ax):
    """Cell-centred linear interpolation (3/4, 1/4) along a periodic axis."""
    lo = 0.75 * x + 0.25 * np.roll(x, 1, axis=ax)
    hi = 0.75 * x + 0.25 * np.roll(x, -1, axis=ax)
    st = np.stack([lo, hi], axis=ax + 1)
    shp = list(x.shape)
    shp[ax] *= 2
    return st.reshape(shp)


def prolong(e, kind):
    """Multilinear prolongation.  Along z: cell kinds interpolate 3/4, 1/4
    with the mirror value of the boundary cell beyond a wall; the normal
    component copies coarse face K onto fine face 2K and averages coarse
    faces K and K+1 onto fine face 2K+1 (the wall face K = n/2 is 0), and its
    fine wall faces get no correction.  The periodic axes are cell-centred."""
    out = e
    if kind == FACE_DIR:
        nc = out.shape[0]
        f = np.zeros((2 * nc,) + out.shape[1:])
        f[0::2] = out
        up = np.roll(out, -1, axis=0)
        up[-1] = 0.0
        f[1::2] = 0.5 * (out + up)
        out = f
    else:
        s = -1.0 if kind == CELL_DIR else 1.0
        below = np.roll(out, 1, axis=0)
        above = np.roll(out, -1, axis=0)
        below[0] = s * out[0]
        above[-1] = s * out[-1]
        st = np.stack([0.75 * out + 0.25 * below, 0.75 * out + 0.25 * above], axis=1)
        shp = list(out.shape)
        shp[0] *= 2
        out = st.reshape(shp)
    for ax in range(1, e.ndim):
        out = _prolong_periodic_axis(out, ax)
    if kind == FACE_DIR:
        out[0] = 0.0
    return out


def vcycle(b, c0, c1, kind, nu_pre=2, nu_post=2, nu_coarse=4, _top=True):
    """One V-cycle for (c0 - c1 L) x = b with the walls' rules for `kind`;
    the Neumann problem with c0 = 0 is singular and loses its mean like the
    periodic one."""
    b = np.asarray(b, dtype=np.float64).copy()
    if kind == FACE_DIR:
        b[0] = 0.0
    singular = c0 == 0.0 and kind == CELL_NEU
    n = b.shape[0]
    if singular and _top:
        b = b - b.mean()
    if n <= 4:
        if singular:
            b = b - b.mean()
        x = smooth(np.zeros_like(b), b, c0, c1, kind, nu_coarse)
    else:
        x = smooth(np.zeros_like(b), b, c0, c1, kind, nu_pre)
        r = b - apply_op(x, c0, c1, kind)
        e = vcycle(restrict(r, kind), c0, c1 / 4.0, kind, nu_pre, nu_post, nu_coarse, _top=False)
        x = x + prolong(e, kind)
        x = smooth(x, b, c0, c1, kind, nu_post)
    if singular and _top:
        x = x - x.mean()
    return x


@dataclass
class MG:
    nu_pre: int = 2
    nu_post: int = 2
    nu_coarse: int = 4


def ps_inv(g, hp, c0, eta, h, mg=None):
    """Projection preconditioner P_S^-1 (eq. P1_practical) with the walls:
    one V-cycle per velocity component, the divergence, one Neumann V-cycle
    for the pressure, the gradient correction (zero on the wall faces)."""
    mg = mg or MG()
    d = g.shape[0]
    ks = kinds(d)
    v = np.stack([vcycle(g[a], c0, eta / (h * h), ks[a], mg.nu_pre, mg.nu_post, mg.nu_coarse) for a in range(d)])
    q = -div(v, h) - (0.0 if hp is None else hp)
    phi = vcycle(q, 0.0, -1.0, CELL_NEU, mg.nu_pre, mg.nu_post, mg.nu_coarse)
    gp = grad(phi, 1.0)
    v = v + h * gp
    pi = -c0 * h * h * phi + eta * q
    return v, pi


# ---------------------------------------------------------------- Faxen's slit mobility
# Series of Sec. 7 (eq. Faxen_slit) for a sphere of hydrodynamic radius R
# translating parallel to the walls of an infinite slit of width d, at the
# midplane (H = d/2) and at the quarter plane (H = d/4), H the distance to the
# nearer wall: mobility = (6 pi eta R)^-1 (1 + c1 x + c3 x^3 + c4 x^4 + c5 x^5),
# x = R / H.
FAXEN = {"half": (-1.004, 0.418, 0.21, -0.169), "quarter": (-0.6526, 0.1475, -0.131, -0.0644)}


def faxen_mobility(R, H, where, eta=1.0):
    c1, c3, c4, c5 = FAXEN[where]
    x = R / H
    return (1.0 + c1 * x + c3 * x ** 3 + c4 * x ** 4 + c5 * x ** 5) / (6.0 * math.pi * eta * R)


def radius_from_slit_drag(F, V, H, where, eta=1.0):
    """Effective radius R_L for which Faxen's series gives drag F at speed V
    (the drag F / V = 1 / mobility grows with R; bisection)."""
    lo, hi = 1e-9 * H, 0.6 * H
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 1.0 / faxen_mobility(mid, H, where, eta) < F / V:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------- unsteady steps between the walls
def advection(v, h):
    """The centred advective form of ``navier.advection`` with the walls'
    extension: a tangential component's neighbour across a wall is its mirror
    image with the sign reversed, the normal component's wall faces hold 0
    (so the averaged normal velocity and its differences need no ghost), and
    the normal component's rows on the wall faces are 0 (not equations)."""
    d = v.shape[0]
    ks = kinds(d)
    out = np.zeros_like(v)
    for a in range(d):
        axa = d - 1 - a
        acc = np.zeros_like(v[a])

        def nb(x, off, ax, kind):
            return znbr(x, off, kind) if ax == 0 else pnbr(x, off, ax)

        for b in range(d):
            axb = d - 1 - b
            if b == a:
                vb = v[a]
            else:
                # v^b at c, c + e_b, c - e_a, c - e_a + e_b; along the wall axis these
                # stay inside the lattice or land on a wall face (value 0)
                vm = nb(v[b], -1, axa, ks[b])
                vb = 0.25 * (v[b] + nb(v[b], 1, axb, ks[b]) + vm + nb(vm, 1, axb, ks[b]))
            acc += vb * (nb(v[a], 1, axb, ks[a]) - nb(v[a], -1, axb, ks[a])) / (2.0 * h)
        out[a] = acc
    out[d - 1][0] = 0.0
    return out


def face_velocity(v, a):
    """``navier.face_velocity`` with the walls' extension: the averaged
    components read their neighbours across a wall through E."""
    d = v.shape[0]
    ks = kinds(d)
    axa = d - 1 - a

    def nb(x, off, ax, kind):
        return znbr(x, off, kind) if ax == 0 else pnbr(x, off, ax)

    out = []
    for b in range(d):
        if b == a:
            out.append(v[a])
        else:
            axb = d - 1 - b
            vm = nb(v[b], -1, axa, ks[b])
            out.append(0.25 * (v[b] + nb(v[b], 1, axb, ks[b]) + vm + nb(vm, 1, axb, ks[b])))
    return out


def _fold_along_z(kind, n):
    """Index map of E for any integer z index (repeated mirroring has period
    2n); periodic wrap along the other axes."""
    def fold(ax, j):
        if ax != 0:
            return np.mod(j, n), np.ones(j.shape)
        jm = np.mod(j, 2 * n)
        if kind == FACE_DIR:
            idx = np.where(jm <= n, jm, 2 * n - jm)
            sgn = np.where(jm < n, 1.0, -1.0)
            sgn = np.where((jm == 0) | (jm == n), 0.0, sgn)
            return np.where(idx == n, 0, idx), sgn
        idx = np.where(jm < n, jm, 2 * n - 1 - jm)
        sgn = np.where(jm < n, 1.0, -1.0 if kind == CELL_DIR else 1.0)
        return idx, sgn
    return fold


def departure_values(v, h, dt):
    """``navier.departure_values`` between the walls: the face velocity with
    the wall rules, and the interpolation reading the lattice through E along
    z (a departure point beyond a wall reads the mirror image)."""
    from . import navier
    d, n = v.shape[0], v.shape[1]
    ks = kinds(d)
    out = np.zeros_like(v)
    idx = np.indices(v.shape[1:]).astype(np.float64)
    for a in range(d):
        u = face_velocity(v, a)
        sl = [idx[ax] - dt * u[d - 1 - ax] / h for ax in range(d)]
        out[a] = navier.interp_lattice(v[a], sl, _fold_along_z(ks[a], n))
    out[d - 1][0] = 0.0
    return out


def advection_sl(v, h, dt):
    """N = (v - v_departure)/dt between the walls; the normal component's
    wall rows are 0."""
    N = (v - departure_values(v, h, dt)) / dt
    N[v.shape[0] - 1][0] = 0.0
    return N


def run(prob, nsteps, scheme="centred", **kw):
    """Exact constrained solves along a trajectory between the walls (the
    steps of ``navier.run``: AB2 advection or semi-Lagrangian transport,
    backward Euler viscosity, bodies translated before each solve)."""
    from . import navier
    d, n, h = prob.dim, prob.n, prob.h
    v = np.zeros((d,) + (n,) * d)
    N_prev = None
    R = prob.R.copy()
    centres = prob.centres.copy()
    out = []
    b = ib.body_of(prob.offsets)
    c0 = prob.rho / prob.dt
    for step in range(nsteps):
        if scheme == "sl":
            N_n = advection_sl(v, h, prob.dt)
            g = navier.rhs(v, N_n, None, prob.rho, prob.dt, first=True)
        else:
            N_n = advection(v, h)
            g = navier.rhs(v, N_n, N_prev, prob.rho, prob.dt, first=(step == 0))
        g[d - 1][0] = 0.0
        R = R + prob.dt * prob.U[b]
        centres = centres + prob.dt * prob.U
        sysm = System(d, n, h, c0, prob.eta, R)
        V = ib.marker_velocities(R, prob.offsets, centres, prob.U, prob.Omega, prob.L)
        sol = constrained.solve(sysm, g, None, -V, prob.offsets, centres, **kw)
        out.append(sol)
        N_prev = N_n
        v = sol.v
    return out
