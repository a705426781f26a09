"""No-slip walls on any set of axes, up to every side of the box: the
non-periodic domain of Sec. 7.1 (a sphere moving through a box with no-slip
conditions on all sides) and the walled box of Sec. 7.3, with the boundary
treatment of the appendix on physical boundary conditions.

TEST INFRASTRUCTURE ONLY (see the package header).

``walls`` is a tuple of d booleans: walls[alpha] puts no-slip walls at both
ends of axis alpha (coordinate alpha, array axis d-1-alpha of a field, whose
axes are ordered (z, y, x) / (y, x)).  At least one axis carries walls.  Along
a walled axis each field follows the rules of the slit channel
(``oracle.walls``, whose module text gives them in full):
  * velocity component alpha along its own walled axis: faces k h, face 0 on
    the wall holds 0 and is not an unknown (the other wall is face n);
  * velocity component alpha along another walled axis: cell-centred, the
    ghost mirrors the interior with the sign reversed (homogeneous Dirichlet);
  * pressure: cell-centred, mirror with the sign kept (homogeneous Neumann,
    the Poisson problem of P_S^-1).
Along an axis without walls everything is periodic.  J = J0 E and S = E^T S0
fold the kernel's taps back through the same mirrors on every walled axis.
With any wall the velocity block has no null space: S is used as is (no S')
and only the pressure's constant mode is fixed (zero mean).

The exact solve assembles the whole MAC system of eq. Stokes_saddle as a
sparse matrix from one-dimensional difference matrices (Kronecker products
over the axes), borders it by the pressure gauge (a multiplier in every
continuity row, a zero-mean row) and factors it by sparse LU (SuperLU through
SciPy).  ``stokes_apply`` states the same operator a second way, as stencils
on the mirror-extended fields; the tests check one against the other.  The
V-cycle and P_S^-1 carry the slit channel's transfers to every walled axis:
cell-centred averaging and 3/4-1/4 interpolation for cell-centred kinds,
vertex-centred full weighting and copy/average interpolation for the normal
component along its own axis.
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import constrained, ib, kernel

PER = "per"             # no wall along this axis: periodic
CELL_DIR = "cell_dir"   # tangential velocity: mirror with the sign reversed
FACE_DIR = "face_dir"   # normal velocity along its own axis: wall faces pinned to 0
CELL_NEU = "cell_neu"   # pressure: mirror with the sign kept


def normalise(walls, d):
    w = tuple(bool(x) for x in walls)
    if len(w) != d or not any(w):
        raise ValueError("walls must name d axes, at least one of them walled")
    return w


def field_kinds(d, walls, field):
    """Kind of a field along each ARRAY axis; field = velocity component
    0..d-1, or "p" for the pressure."""
    out = []
    for ax in range(d):
        beta = d - 1 - ax
        if not walls[beta]:
            out.append(PER)
        elif field == "p":
            out.append(CELL_NEU)
        else:
            out.append(FACE_DIR if beta == field else CELL_DIR)
    return out


# ---------------------------------------------------------------- extension E along one axis
def extend(j, n, kind):
    """(interior index, sign) that index j stands for along one axis, or
    (None, 0) for a wall face (value 0)."""
    if kind == PER:
        return j % n, 1
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


def nbr(x, off, ax, kind):
    """y with y_k = (E x)_{k + off} along array axis ax (off = +-1)."""
    n = x.shape[ax]
    idx = np.zeros(n, dtype=np.int64)
    sgn = np.zeros(n)
    for k in range(n):
        j, s = extend(k + off, n, kind)
        if j is not None:
            idx[k], sgn[k] = j, s
    shape = [1] * x.ndim
    shape[ax] = n
    return np.take(x, idx, axis=ax) * sgn.reshape(shape)


def wall_mask(n, d, walls, a):
    """Boolean mask of component a's wall faces (index 0 along its own axis
    when that axis is walled)."""
    m = np.zeros((n,) * d, dtype=bool)
    if walls[a]:
        sl = [slice(None)] * d
        sl[d - 1 - a] = 0
        m[tuple(sl)] = True
    return m


# ---------------------------------------------------------------- operators as stencils
def lap(x, kinds):
    """Dimensionless Laplacian on the mirror-extended field; rows of wall
    faces are 0."""
    out = np.zeros_like(x)
    for ax in range(x.ndim):
        out = out + (nbr(x, 1, ax, kinds[ax]) - x) + (nbr(x, -1, ax, kinds[ax]) - x)
    for ax in range(x.ndim):
        if kinds[ax] == FACE_DIR:
            sl = [slice(None)] * x.ndim
            sl[ax] = 0
            out[tuple(sl)] = 0.0
    return out


def grad(p, h, walls):
    """G pi on the faces; zero on the wall faces."""
    d = p.ndim
    out = []
    for a in range(d):
        ax = d - 1 - a
        g = (p - np.roll(p, 1, axis=ax)) / h
        if walls[a]:
            sl = [slice(None)] * d
            sl[ax] = 0
            g[tuple(sl)] = 0.0
        out.append(g)
    return np.stack(out)


def div(v, h, walls):
    """D v at cell centres; wall faces carry no flux."""
    d = v.shape[0]
    out = np.zeros(v.shape[1:])
    for a in range(d):
        ax = d - 1 - a
        lo = v[a].copy()
        up = np.roll(v[a], -1, axis=ax)
        if walls[a]:
            sl0 = [slice(None)] * d
            sl0[ax] = 0
            lo[tuple(sl0)] = 0.0          # face 0 is the wall
            sln = [slice(None)] * d
            sln[ax] = -1
            up[tuple(sln)] = 0.0          # face n is the other wall
        out += (up - lo) / h
    return out


def stokes_apply(v, p, c0, eta, h, walls):
    """[[A, G], [-D, 0]] (v, pi) with the walls; A = c0 - eta h^-2 L per
    component; the rows of the wall faces are 0."""
    d = v.shape[0]
    n = v.shape[-1]
    mv = np.stack([c0 * v[a] - eta / (h * h) * lap(v[a], field_kinds(d, walls, a)) for a in range(d)])
    mv = mv + grad(p, h, walls)
    for a in range(d):
        mv[a][wall_mask(n, d, walls, a)] = 0.0
    return mv, -div(v, h, walls)


# ---------------------------------------------------------------- operators as sparse matrices
def _lap1(n, kind):
    """1D second difference of one kind (n x n)."""
    L = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    if kind == PER:
        L[0, -1] += 1.0
        L[-1, 0] += 1.0
    elif kind == CELL_DIR:
        L[0, 0] -= 1.0
        L[-1, -1] -= 1.0
    elif kind == CELL_NEU:
        L[0, 0] += 1.0
        L[-1, -1] += 1.0
    else:                       # FACE_DIR: face 0 is the wall (no unknown), face n too
        L[0, :] = 0.0
        L[:, 0] = 0.0
    return L


def _grad1(n, walled):
    """Cell -> face difference along one axis: face j reads cells j and j-1."""
    G = np.eye(n) - np.eye(n, k=-1)
    if walled:
        G[0, :] = 0.0
    else:
        G[0, -1] = -1.0
    return G


def _div1(n, walled):
    """Face -> cell difference along one axis: cell j reads faces j+1 and j."""
    D = np.eye(n, k=1) - np.eye(n)
    if walled:
        D[:, 0] = 0.0             # face 0 is the wall; face n (beyond the last row) too
    else:
        D[-1, 0] = 1.0
    return D


def _along(M, ax, d, n):
    """The matrix acting with M along array axis ax of a C-ordered field."""
    out = sp.identity(1, format="csr")
    for k in range(d):
        out = sp.kron(out, sp.csr_matrix(M) if k == ax else sp.identity(n, format="csr"), format="csr")
    return out


def operator_blocks(n, d, h, c0, eta, walls):
    """A_a (with identity rows on the wall faces), G_a, D_a as sparse matrices."""
    C = n ** d
    A, G, D = [], [], []
    for a in range(d):
        ks = field_kinds(d, walls, a)
        La = sp.csr_matrix((C, C))
        for ax in range(d):
            La = La + _along(_lap1(n, ks[ax]), ax, d, n)
        Aa = (c0 * sp.identity(C) - (eta / (h * h)) * La).tolil()
        wm = np.flatnonzero(wall_mask(n, d, walls, a).reshape(-1))
        for r in wm:
            Aa[r, :] = 0.0
            Aa[:, r] = 0.0
            Aa[r, r] = 1.0
        A.append(Aa.tocsr())
        ax = d - 1 - a
        G.append(_along(_grad1(n, walls[a]), ax, d, n) / h)
        D.append(_along(_div1(n, walls[a]), ax, d, n) / h)
    return A, G, D


def assemble(n, d, h, c0, eta, walls):
    """The bordered sparse system [[A, G, 0], [-D, 0, 1], [0, 1^T, 0]]."""
    A, G, D = operator_blocks(n, d, h, c0, eta, walls)
    C = n ** d
    rows = []
    for a in range(d):
        rows.append([A[a] if b == a else None for b in range(d)] + [G[a], None])
    rows.append([-D[b] for b in range(d)] + [None, sp.csr_matrix(np.ones((C, 1)))])
    rows.append([None] * d + [sp.csr_matrix(np.ones((1, C))), None])
    return sp.bmat(rows, format="csc")


_LU = {}


def solve(f, hp, c0, eta, h, d, walls):
    """Exact walled Stokes solve: A v + G pi = f, -D v = hp, mean pi = 0.

    f [..., d, n..] (wall-face entries ignored), hp [..., n..] or None.
    Returns (v, pi); v is 0 on the wall faces."""
    walls = normalise(walls, d)
    n = f.shape[-1]
    key = (n, d, h, c0, eta, walls)
    if key not in _LU:
        _LU.clear()
        _LU[key] = spla.splu(assemble(n, d, h, c0, eta, walls))
    lu = _LU[key]
    C = n ** d
    lead = f.shape[:-(d + 1)]
    fr = np.asarray(f, dtype=np.float64).reshape((-1, d, C)).copy()
    for a in range(d):
        fr[:, a, wall_mask(n, d, walls, a).reshape(-1)] = 0.0
    hr = np.zeros((fr.shape[0], C)) if hp is None else np.asarray(hp, dtype=np.float64).reshape((-1, C))
    rhs = np.concatenate([fr.reshape(fr.shape[0], d * C), hr, np.zeros((fr.shape[0], 1))], axis=1)
    sol = lu.solve(rhs.T.copy()).T
    v = sol[:, :d * C].reshape(lead + (d,) + (n,) * d)
    p = sol[:, d * C:(d + 1) * C].reshape(lead + (n,) * d)
    return v, p


# ---------------------------------------------------------------- J = J0 E, S = E^T S0
def taps_1d(pos, n, h, kind):
    """Indices [N, 4] and weights [N, 4] of the taps along one axis, folded
    through the extension of that axis (taps on wall faces get weight 0)."""
    s = pos / h - (0.0 if kind == FACE_DIR else 0.5)
    base = np.floor(s).astype(np.int64) - 1
    j = base[:, None] + np.arange(4)[None, :]
    w = kernel.phi(s[:, None] - j)
    idx = np.zeros_like(j)
    wt = np.zeros_like(w)
    for m in range(j.shape[0]):
        for t in range(4):
            q, sg = extend(int(j[m, t]), n, kind)
            if q is not None:
                idx[m, t] = q
                wt[m, t] = sg * w[m, t]
    return idx, wt


def _taps_kind(alpha, beta, walls):
    if not walls[beta]:
        return PER
    return FACE_DIR if beta == alpha else CELL_DIR


def weights(R, n, h, alpha, walls):
    N, d = R.shape
    idx1, w1 = [], []
    for beta in range(d):
        kind = _taps_kind(alpha, beta, walls)
        if kind == PER:
            i, w = ib.taps_1d(R[:, beta], n, h, staggered=(beta == alpha))
        else:
            i, w = taps_1d(R[:, beta], n, h, kind)
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


def all_weights(R, n, h, walls):
    return [weights(R, n, h, a, walls) for a in range(R.shape[1])]


def check_inside(R, L, walls):
    """Markers must lie strictly inside the walls of every walled axis."""
    R = np.asarray(R)
    for beta, w in enumerate(walls):
        if w and not (np.all(R[:, beta] > 0.0) and np.all(R[:, beta] < L)):
            raise ValueError("markers must lie strictly between the walls")


# ---------------------------------------------------------------- constrained system
class System(constrained.System):
    """eq. constrained_Stokes with the walls: S = E^T S0 (no S', no velocity
    mean), J = J0 E, exact walled Stokes solves."""

    def __init__(self, dim, n, h, c0, eta, R, walls):
        self.d = dim
        self.n = n
        self.h = h
        self.c0 = c0
        self.eta = eta
        self.walls = normalise(walls, dim)
        self.R = np.asarray(R, dtype=np.float64)
        check_inside(self.R, n * h, self.walls)
        self.steady = c0 == 0.0
        self.W = all_weights(self.R, n, h, self.walls)

    def spread(self, lam):
        return ib.spread(lam, self.R, self.n, self.h, self.W)

    def stokes(self, f, hp=None):
        return solve(f, hp, self.c0, self.eta, self.h, self.d, self.walls)


def all_walls(d):
    return (True,) * d


def solve_problem(prob, walls=None, g=None, hp=None, **kw):
    """Exact solution of a prescribed-motion problem in the walled box
    (walls on every side unless given)."""
    walls = all_walls(prob.dim) if walls is None else walls
    c0 = 0.0 if prob.steady else prob.rho / prob.dt
    sysm = System(prob.dim, prob.n, prob.h, c0, prob.eta, prob.R, walls)
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    return constrained.solve(sysm, g, hp, -V, prob.offsets, prob.centres, **kw)


def residual(sysm, v, p, lam, g, hp, W):
    """Blocks of b - K x of the walled system."""
    d, n = sysm.d, sysm.n
    if g is None:
        g = np.zeros((d,) + (n,) * d)
    if hp is None:
        hp = np.zeros((n,) * d)
    rm, rc = stokes_apply(v, p, sysm.c0, sysm.eta, sysm.h, sysm.walls)
    rm = g - (rm - sysm.spread(lam))
    for a in range(d):
        rm[a][wall_mask(n, d, sysm.walls, a)] = 0.0
    return rm, hp - rc, W + sysm.interp(v)


# ---------------------------------------------------------------- V-cycle with the walls
def _diag(shape, c0, c1, kinds):
    """Diagonal of (c0 - c1 L): a boundary cell's mirror image is the cell
    itself and joins the diagonal with the mirror's sign."""
    d = len(shape)
    dg = np.full(shape, c0 + 2.0 * d * c1)
    for ax, kind in enumerate(kinds):
        if kind in (CELL_DIR, CELL_NEU):
            s = 1.0 if kind == CELL_DIR else -1.0
            for end in (0, -1):
                sl = [slice(None)] * d
                sl[ax] = end
                dg[tuple(sl)] += s * c1
    return dg


def _nbr_sum(x, kinds):
    """Sum of the neighbours that are other unknowns."""
    s = np.zeros_like(x)
    d = x.ndim
    for ax, kind in enumerate(kinds):
        up = np.roll(x, -1, axis=ax)
        dn = np.roll(x, 1, axis=ax)
        if kind != PER:
            # beyond the last cell: its own mirror (diagonal) or the wall face (0);
            # before the first: its own mirror (diagonal), or for faces the
            # wall face's row, which is not an equation
            sl = [slice(None)] * d
            sl[ax] = -1
            up[tuple(sl)] = 0.0
            sl[ax] = 0
            dn[tuple(sl)] = 0.0
        s = s + up + dn
    return s


def _pin(x, kinds):
    for ax, kind in enumerate(kinds):
        if kind == FACE_DIR:
            sl = [slice(None)] * x.ndim
            sl[ax] = 0
            x[tuple(sl)] = 0.0
    return x


def apply_op(x, c0, c1, kinds):
    return _pin(_diag(x.shape, c0, c1, kinds) * x - c1 * _nbr_sum(x, kinds), kinds)


def smooth(x, b, c0, c1, kinds, sweeps):
    par = np.indices(x.shape).sum(axis=0) % 2
    dg = _diag(x.shape, c0, c1, kinds)
    for _ in range(sweeps):
        for colour in (0, 1):
            new = (b + c1 * _nbr_sum(x, kinds)) / dg
            x = _pin(np.where(par == colour, new, x), kinds)
    return x


def restrict(r, kinds):
    """Per axis: cell-centred kinds average their 2 children; the normal
    component along its own axis takes full weighting 1/4, 1/2, 1/4 of fine
    faces 2K-1, 2K, 2K+1 (the coarse wall face K = 0 stays 0)."""
    out = r
    for ax, kind in enumerate(kinds):
        n = out.shape[ax]
        if kind != FACE_DIR:
            shp = list(out.shape)
            shp[ax] //= 2
            shp.insert(ax + 1, 2)
            out = out.reshape(shp).mean(axis=ax + 1)
        else:
            o = np.moveaxis(out, ax, 0)
            rz = np.zeros((n // 2,) + o.shape[1:])
            for K in range(1, n // 2):
                rz[K] = 0.25 * o[2 * K - 1] + 0.5 * o[2 * K] + 0.25 * o[2 * K + 1]
            out = np.moveaxis(rz, 0, ax)
    return out


def prolong(e, kinds):
    """Per axis: cell-centred kinds interpolate 3/4, 1/4 (periodic neighbour,
    or the mirror value of the boundary cell beyond a wall); the normal
    component along its own axis copies coarse face K onto fine face 2K and
    averages faces K and K+1 onto 2K+1 (the wall face n/2 is 0).  Fine wall
    faces get no correction."""
    out = e
    for ax, kind in enumerate(kinds):
        o = np.moveaxis(out, ax, 0)
        nc = o.shape[0]
        if kind == FACE_DIR:
            f = np.zeros((2 * nc,) + o.shape[1:])
            f[0::2] = o
            up = np.roll(o, -1, axis=0)
            up[-1] = 0.0
            f[1::2] = 0.5 * (o + up)
        else:
            below = np.roll(o, 1, axis=0)
            above = np.roll(o, -1, axis=0)
            if kind != PER:
                s = -1.0 if kind == CELL_DIR else 1.0
                below[0] = s * o[0]
                above[-1] = s * o[-1]
            f = np.stack([0.75 * o + 0.25 * below, 0.75 * o + 0.25 * above], axis=1)
            f = f.reshape((2 * nc,) + o.shape[1:])
        out = np.moveaxis(f, 0, ax)
    return _pin(out, kinds)


def vcycle(b, c0, c1, kinds, nu_pre=2, nu_post=2, nu_coarse=4, _top=True):
    """One V-cycle for (c0 - c1 L) x = b with the given kinds per array
    axis; the problem is singular (and loses its mean like the periodic one)
    when c0 = 0 and no axis is Dirichlet."""
    b = _pin(np.asarray(b, dtype=np.float64).copy(), kinds)
    singular = c0 == 0.0 and all(k in (PER, CELL_NEU) for k in kinds)
    n = b.shape[0]
    if singular and _top:
        b = b - b.mean()
    if n <= 4:
        if singular:
            b = b - b.mean()
        x = smooth(np.zeros_like(b), b, c0, c1, kinds, nu_coarse)
    else:
        x = smooth(np.zeros_like(b), b, c0, c1, kinds, nu_pre)
        r = b - apply_op(x, c0, c1, kinds)
        e = vcycle(restrict(r, kinds), c0, c1 / 4.0, kinds, nu_pre, nu_post, nu_coarse, _top=False)
        x = x + prolong(e, kinds)
        x = smooth(x, b, c0, c1, kinds, nu_post)
    if singular and _top:
        x = x - x.mean()
    return x


def ps_inv(g, hp, c0, eta, h, walls, nu_pre=2, nu_post=2, nu_coarse=4):
    """Projection preconditioner P_S^-1 (eq. P1_practical) with the walls:
    one V-cycle per velocity component, the divergence, one V-cycle of the
    pressure's Neumann problem, the gradient correction (zero on wall faces)."""
    d = g.shape[0]
    walls = normalise(walls, d)
    v = np.stack([vcycle(g[a], c0, eta / (h * h), field_kinds(d, walls, a), nu_pre, nu_post, nu_coarse)
                  for a in range(d)])
    q = -div(v, h, walls) - (0.0 if hp is None else hp)
    phi = vcycle(q, 0.0, -1.0, field_kinds(d, walls, "p"), nu_pre, nu_post, nu_coarse)
    v = v + h * grad(phi, 1.0, walls)
    pi = -c0 * h * h * phi + eta * q
    return v, pi


# ---------------------------------------------------------------- unsteady steps in the box
def advection(v, h, walls):
    """The centred advective form of ``navier.advection`` with the walls'
    extension on every walled axis: a tangential component's neighbour across
    a wall is its mirror image with the sign reversed; the normal components'
    wall faces hold 0 (so the averaged normal velocities and their own
    differences need no ghost); the normal components' rows on their wall
    faces are 0."""
    d = v.shape[0]
    n = v.shape[-1]
    out = np.zeros_like(v)
    for a in range(d):
        ka = field_kinds(d, walls, a)
        axa = d - 1 - a
        acc = np.zeros_like(v[a])
        for b in range(d):
            axb = d - 1 - b
            if b == a:
                vb = v[a]
            else:
                kb = field_kinds(d, walls, b)
                # v^b at c, c + e_b, c - e_a, c - e_a + e_b
                vm = nbr(v[b], -1, axa, kb[axa])
                vb = 0.25 * (v[b] + nbr(v[b], 1, axb, kb[axb]) + vm + nbr(vm, 1, axb, kb[axb]))
            acc += vb * (nbr(v[a], 1, axb, ka[axb]) - nbr(v[a], -1, axb, ka[axb])) / (2.0 * h)
        acc[wall_mask(n, d, walls, a)] = 0.0
        out[a] = acc
    return out


def face_velocity(v, a, walls):
    """``navier.face_velocity`` with the walls' extension."""
    d = v.shape[0]
    axa = d - 1 - a
    out = []
    for b in range(d):
        if b == a:
            out.append(v[a])
        else:
            kb = field_kinds(d, walls, b)
            axb = d - 1 - b
            vm = nbr(v[b], -1, axa, kb[axa])
            out.append(0.25 * (v[b] + nbr(v[b], 1, axb, kb[axb]) + vm + nbr(vm, 1, axb, kb[axb])))
    return out


def _fold(kinds, n):
    """Index map of E along each array axis for any integer index (repeated
    mirroring has period 2n; periodic axes wrap)."""
    def fold(ax, j):
        kind = kinds[ax]
        if kind == PER:
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


def advection_sl(v, h, dt, walls):
    """N = (v - v_departure) / dt in the box: the departure point of each face
    from its face velocity (wall rules), the interpolation reading the lattice
    through E on every walled axis; the wall rows are 0."""
    from . import navier
    d, n = v.shape[0], v.shape[-1]
    vd = np.zeros_like(v)
    idx = np.indices(v.shape[1:]).astype(np.float64)
    for a in range(d):
        u = face_velocity(v, a, walls)
        sl = [idx[ax] - dt * u[d - 1 - ax] / h for ax in range(d)]
        vd[a] = navier.interp_lattice(v[a], sl, _fold(field_kinds(d, walls, a), n))
    N = (v - vd) / dt
    for a in range(d):
        N[a][wall_mask(n, d, walls, a)] = 0.0
    return N


def run(prob, nsteps, walls=None, scheme="centred", **kw):
    """Exact constrained solves along a trajectory in the box (the steps of
    ``navier.run``: AB2 advection or semi-Lagrangian transport, backward
    Euler viscosity, bodies translated before each solve)."""
    from . import navier
    d, n, h = prob.dim, prob.n, prob.h
    walls = all_walls(d) if walls is None else normalise(walls, d)
    v = np.zeros((d,) + (n,) * d)
    N_prev = None
    R = prob.R.copy()
    centres = prob.centres.copy()
    out = []
    b = ib.body_of(prob.offsets)
    c0 = prob.rho / prob.dt
    for step in range(nsteps):
        if scheme == "sl":
            N_n = advection_sl(v, h, prob.dt, walls)
            g = navier.rhs(v, N_n, None, prob.rho, prob.dt, first=True)
        else:
            N_n = advection(v, h, walls)
            g = navier.rhs(v, N_n, N_prev, prob.rho, prob.dt, first=(step == 0))
        for a in range(d):
            g[a][wall_mask(n, d, walls, a)] = 0.0
        R = R + prob.dt * prob.U[b]
        centres = centres + prob.dt * prob.U
        sysm = System(d, n, h, c0, prob.eta, R, walls)
        V = ib.marker_velocities(R, prob.offsets, centres, prob.U, prob.Omega, prob.L)
        sol = constrained.solve(sysm, g, None, -V, prob.offsets, centres, **kw)
        out.append(sol)
        N_prev = N_n
        v = sol.v
    return out


# ---------------------------------------------------------------- moving walls
# Walls with a prescribed velocity (inhomogeneous Dirichlet data; Sec. 7.3's
# box moves with the cavity, the appendix on physical boundaries gives the
# mirror rule).  wall_vel[beta] = (U_lo, U_hi): the velocity vectors of the
# walls at coordinate 0 and at l along walled axis beta.  Along beta a
# component tangential to the wall has ghost values 2 U - v (the mirror
# image about the wall value); the normal component's wall faces hold
# U . e_beta, and its ghost faces are 2 U - v as well.  Written here on an
# explicitly padded lattice (two ghost layers per side along every axis,
# periodic axes wrapped), independently of the folded taps above.
PAD = 2


def padded(v, walls, wall_vel):
    """Velocity components on the padded lattice: v [d, n..] (the normal
    components' wall faces ignored).  Returns [d] arrays of shape (n+2 PAD,)*d,
    index j + PAD for lattice index j (face n, the high wall, included)."""
    d, n = v.shape[0], v.shape[-1]
    out = []
    for a in range(d):
        x = np.asarray(v[a], dtype=np.float64)
        for ax in range(d):
            beta = d - 1 - ax
            x = np.moveaxis(x, ax, 0)
            if not walls[beta]:
                y = np.concatenate([x[-PAD:], x, x[:PAD]], axis=0)
            else:
                lo, hi = (np.asarray(wall_vel[beta][0])[a], np.asarray(wall_vel[beta][1])[a]) \
                    if wall_vel is not None and wall_vel.get(beta) is not None else (0.0, 0.0)
                y = np.zeros((n + 2 * PAD,) + x.shape[1:])
                y[PAD:PAD + n] = x
                if beta == a:
                    # faces: 0 and n on the walls, ghosts mirror about the wall values
                    y[PAD] = lo
                    y[PAD + n] = hi
                    for m in range(1, PAD + 1):
                        y[PAD - m] = 2.0 * lo - y[PAD + m]
                    for m in range(1, PAD):
                        y[PAD + n + m] = 2.0 * hi - y[PAD + n - m]
                else:
                    for m in range(PAD):
                        y[PAD - 1 - m] = 2.0 * lo - x[m]
                        y[PAD + n + m] = 2.0 * hi - x[n - 1 - m]
            x = np.moveaxis(y, 0, ax)
        out.append(x)
    return out


def stokes_apply_padded(v, p, c0, eta, h, walls, wall_vel):
    """[[A, G], [-D, 0]] (v, pi) evaluated on the padded lattice with the
    walls' data; rows of the normal components' wall faces are 0."""
    d, n = v.shape[0], v.shape[-1]
    V = padded(v, walls, wall_vel)
    inner = tuple([slice(PAD, PAD + n)] * d)
    mv = np.zeros_like(np.asarray(v, dtype=np.float64))
    div = np.zeros((n,) * d)
    for a in range(d):
        x = V[a]
        lap = np.zeros((n,) * d)
        c = x[inner]
        for ax in range(d):
            up = [slice(PAD, PAD + n)] * d
            dn = [slice(PAD, PAD + n)] * d
            up[ax] = slice(PAD + 1, PAD + n + 1)
            dn[ax] = slice(PAD - 1, PAD + n - 1)
            lap += (x[tuple(up)] - c) + (x[tuple(dn)] - c)
        ax = d - 1 - a
        up = [slice(PAD, PAD + n)] * d
        up[ax] = slice(PAD + 1, PAD + n + 1)
        div += (x[tuple(up)] - c) / h
        mv[a] = c0 * c - eta / (h * h) * lap
    mv = mv + grad(p, h, walls)
    for a in range(d):
        mv[a][wall_mask(n, d, walls, a)] = 0.0
    return mv, -div


def interp_padded(v, R, h, walls, wall_vel):
    """J v with the walls' data: the standard kernel taps on the padded
    lattice (no folding)."""
    d, n = v.shape[0], v.shape[-1]
    V = padded(v, walls, wall_vel)
    N = R.shape[0]
    out = np.zeros((N, d))
    for a in range(d):
        for m in range(N):
            taps = []
            for beta in range(d):
                s = R[m, beta] / h - (0.0 if beta == a else 0.5)
                base = int(np.floor(s)) - 1
                js = base + np.arange(4)
                ws = kernel.phi(s - js)
                if not walls[beta]:
                    js = np.mod(js, n)
                taps.append((js + PAD, ws))
            acc = 0.0
            for combo in itertools.product(range(4), repeat=d):
                idx = tuple(taps[d - 1 - ax][0][combo[d - 1 - ax]] for ax in range(d))
                w = 1.0
                for beta in range(d):
                    w *= taps[beta][1][combo[beta]]
                acc += w * V[a][idx]
            out[m, a] = acc
    return out


def solve_problem_moving(prob, wall_vel, walls=None, g=None, hp=None, **kw):
    """Exact solution with moving walls: the walls' data enter as the affine
    parts of the stencils and of J on the padded lattice (the homogeneous
    operator applied to zero interior values), moved to the right-hand side;
    the homogeneous constrained system is solved as in ``solve_problem``; the
    normal components' wall faces then take the wall values."""
    d, n, h = prob.dim, prob.n, prob.h
    walls = all_walls(d) if walls is None else normalise(walls, d)
    c0 = 0.0 if prob.steady else prob.rho / prob.dt
    zero = np.zeros((d,) + (n,) * d)
    am, ac = stokes_apply_padded(zero, np.zeros((n,) * d), c0, prob.eta, h, walls, wall_vel)
    ja = interp_padded(zero, prob.R, h, walls, wall_vel)
    g = (np.zeros((d,) + (n,) * d) if g is None else np.asarray(g, dtype=np.float64)) - am
    hp = (np.zeros((n,) * d) if hp is None else np.asarray(hp, dtype=np.float64)) - ac
    sysm = System(d, n, h, c0, prob.eta, prob.R, walls)
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    sol = constrained.solve(sysm, g, hp, -V + ja, prob.offsets, prob.centres, **kw)
    for beta in range(d):
        if walls[beta]:
            sl = [slice(None)] * d
            sl[d - 1 - beta] = 0
            lo = 0.0 if wall_vel is None or wall_vel.get(beta) is None else float(np.asarray(wall_vel[beta][0])[beta])
            sol.v[beta][tuple(sl)] = lo
    return sol
