"""Pins of the walled-box oracle (``oracle/box.py``): no-slip walls on any set
of axes, up to every side (Sec. 7.1's non-periodic domain, Sec. 7.3's box;
the appendix on physical boundary conditions).

* The sparse operator (Kronecker products of 1D difference matrices) equals
  the stencils on the mirror-extended fields, written separately.
* D = -G^T on the unknowns and A is symmetric (the appendix's extension keeps
  the discrete adjoints).
* Walls on the last axis only reproduce the slit-channel oracle (itself
  pinned by eigenvectors, closed forms and a dense solve): exact solve,
  V-cycle, P_S^-1, marker taps.
* The walls follow the axes: a permutation of the axes (with the walls)
  permutes the exact solution.
* A duct (walls on two axes) under a uniform force along the third has the
  discrete Poisson solution of the sine series (DST-II), a closed form.
* A gradient force is balanced by the pressure alone (v = 0, pi = phi).
* The V-cycle converges to the exact solution of its own operator.
* The constrained solve meets every row of the walled system, and J, S stay
  adjoint with the tangential velocity vanishing on a wall.
"""
import itertools

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import box, ib, walls


def _fields(rng, d, n, wl):
    v = rng.standard_normal((d,) + (n,) * d)
    for a in range(d):
        v[a][box.wall_mask(n, d, wl, a)] = 0.0
    p = rng.standard_normal((n,) * d)
    return v, p


MASKS2 = [(True, True), (True, False), (False, True)]
MASKS3 = [(True, True, True), (True, False, False), (False, True, True), (True, False, True)]


@pytest.mark.parametrize("d,wl", [(2, m) for m in MASKS2] + [(3, m) for m in MASKS3])
def test_sparse_operator_equals_stencils(d, wl):
    rng = np.random.default_rng(1)
    n = 8
    h, c0, eta = 1.0 / n, 3.0, 0.7
    v, p = _fields(rng, d, n, wl)
    mv, mc = box.stokes_apply(v, p, c0, eta, h, wl)
    K = box.assemble(n, d, h, c0, eta, wl)
    C = n ** d
    x = np.concatenate([v.reshape(-1), p.reshape(-1), [0.0]])
    y = K @ x
    ref = mv.copy()
    # the sparse rows of wall faces are identity rows (v = 0 there)
    for a in range(d):
        ref[a][box.wall_mask(n, d, wl, a)] = v[a][box.wall_mask(n, d, wl, a)]
    assert np.allclose(y[:d * C], ref.reshape(-1), rtol=0, atol=1e-11 * np.abs(ref).max())
    assert np.allclose(y[d * C:(d + 1) * C], mc.reshape(-1), rtol=0, atol=1e-11 * np.abs(mc).max())


@pytest.mark.parametrize("d,wl", [(2, (True, True)), (3, (True, True, True)), (3, (False, True, False))])
def test_adjoint_structure(d, wl):
    n = 8
    A, G, D = box.operator_blocks(n, d, 1.0 / n, 0.0, 1.0, wl)
    for a in range(d):
        keep = ~box.wall_mask(n, d, wl, a).reshape(-1)
        Ga = G[a].toarray()[keep]
        Da = D[a].toarray()[:, keep]
        assert np.array_equal(Da, -Ga.T)
        Aa = A[a].toarray()
        assert np.array_equal(Aa, Aa.T)
        # Dirichlet along a walled axis: A is positive definite even when steady
        assert np.linalg.eigvalsh(Aa[np.ix_(keep, keep)]).min() > 0


@pytest.mark.parametrize("d", [2, 3])
def test_last_axis_walls_reproduce_the_slit_channel(d):
    rng = np.random.default_rng(2)
    n = 8 if d == 3 else 16
    h = 1.0 / n
    wl = (False,) * (d - 1) + (True,)
    for c0 in (0.0, 5.0):
        f = rng.standard_normal((d,) + (n,) * d)
        hp = rng.standard_normal((n,) * d)
        hp -= hp.mean()
        vb, pb = box.solve(f, hp, c0, 0.8, h, d, wl)
        vs, ps = walls.solve(f, hp, c0, 0.8, h, d)
        scale = np.abs(vs).max()
        assert np.abs(vb - vs).max() < 1e-11 * scale
        assert np.abs(pb - ps).max() < 1e-11 * np.abs(ps).max()
        # P_S^-1 and the V-cycles
        vb, pb = box.ps_inv(f, hp, c0, 0.8, h, wl)
        vs, ps = walls.ps_inv(f, hp, c0, 0.8, h)
        assert np.abs(vb - vs).max() < 1e-12 * np.abs(vs).max()
        assert np.abs(pb - ps).max() < 1e-12 * np.abs(ps).max()
    # marker taps, every component
    R = rng.uniform(0.05, 0.95, (7, d))
    for a in range(d):
        fb, wb = box.weights(R, n, h, a, wl)
        fs, ws = walls.weights(R, n, h, a)
        assert np.array_equal(fb, fs) and np.array_equal(wb, ws)


def test_walls_follow_the_axes():
    """Swapping x and y (the components, the array axes and the walls) maps
    the exact solution onto itself."""
    rng = np.random.default_rng(3)
    d, n = 3, 8
    h = 1.0 / n
    wl = (True, False, True)
    sw = (False, True, True)           # walls after swapping x and y
    f = rng.standard_normal((d,) + (n,) * d)
    v, p = box.solve(f, None, 2.0, 1.0, h, d, wl)
    # array axes are (z, y, x): swap array axes 1 and 2, components 0 and 1
    fs = np.swapaxes(f[[1, 0, 2]], 2, 3)
    vs, ps = box.solve(fs, None, 2.0, 1.0, h, d, sw)
    assert np.abs(np.swapaxes(vs[[1, 0, 2]], 2, 3) - v).max() < 1e-12 * np.abs(v).max()
    assert np.abs(np.swapaxes(ps, 1, 2) - p).max() < 1e-12 * np.abs(p).max()


def test_duct_flow_is_the_sine_series():
    """Walls on y and z, periodic x, force f e_x: u solves -eta h^-2 L u = f
    on the cross-section with reversed mirrors; the DST-II diagonalises that
    Laplacian with eigenvalues -4 sin^2(pi k / 2n) per axis."""
    d, n = 3, 8
    h, eta = 1.0 / n, 0.6
    wl = (False, True, True)
    f = np.zeros((d,) + (n,) * d)
    f[0] = 1.0
    v, p = box.solve(f, None, 0.0, eta, h, d, wl)
    assert np.abs(v[1:]).max() < 1e-12 and np.abs(p).max() < 1e-10
    k = np.arange(1, n + 1)
    lam = 4.0 * np.sin(np.pi * k / (2 * n)) ** 2
    rhs = np.ones((n, n))                              # (z, y) cross-section
    coef = sfft.dstn(rhs, type=2) / (eta / h ** 2 * (lam[:, None] + lam[None, :]))
    u = sfft.idstn(coef, type=2)
    assert np.abs(v[0] - u[:, :, None]).max() < 1e-12 * u.max()
    # and a 2D channel: the 1D discrete Poiseuille profile
    n = 32
    h = 1.0 / n
    lam = 4.0 * np.sin(np.pi * np.arange(1, n + 1) / (2 * n)) ** 2
    v2, _ = box.solve(np.stack([np.ones((n, n)), np.zeros((n, n))]), None, 0.0, eta, h, 2, (False, True))
    u1 = sfft.idst(sfft.dst(np.ones(n), type=2) / (eta / h ** 2 * lam), type=2)
    assert np.abs(v2[0] - u1[:, None]).max() < 1e-12 * u1.max()


@pytest.mark.parametrize("d", [2, 3])
def test_gradient_force_is_hydrostatic(d):
    rng = np.random.default_rng(4)
    n = 8
    h = 1.0 / n
    wl = (True,) * d
    phi = rng.standard_normal((n,) * d)
    f = box.grad(phi, h, wl)
    for c0 in (0.0, 4.0):
        v, p = box.solve(f, None, c0, 1.3, h, d, wl)
        assert np.abs(v).max() < 1e-11 * np.abs(f).max() * h
        assert np.abs(p - (phi - phi.mean())).max() < 1e-11 * np.abs(phi).max()


@pytest.mark.parametrize("d,field,c0", [(3, 0, 0.0), (3, 2, 0.0), (3, "p", 0.0), (3, 1, 50.0), (2, 1, 0.0),
                                        (2, "p", 0.0)])
def test_vcycle_converges_to_exact(d, field, c0):
    rng = np.random.default_rng(5)
    n = 16 if d == 3 else 32
    wl = (True,) * d
    kinds = box.field_kinds(d, wl, field)
    c1 = 1.0
    b = rng.standard_normal((n,) * d)
    if field == "p" and c0 == 0.0:
        b -= b.mean()
    b = box._pin(b, kinds)
    # exact solution of the cycle's own operator on the unknowns
    C = n ** d
    Aop = np.zeros((C, C))
    for j in range(C):
        e = np.zeros(C)
        e[j] = 1.0
        Aop[:, j] = box.apply_op(e.reshape((n,) * d), c0, c1, kinds).reshape(-1)
    free = box._pin(np.ones((n,) * d), kinds).reshape(-1) != 0     # not a wall face
    A = Aop[np.ix_(free, free)]
    x = np.zeros(C)
    x[free] = np.linalg.lstsq(A, b.reshape(-1)[free], rcond=None)[0]
    if field == "p" and c0 == 0.0:
        x -= x.mean()
    xe = x.reshape((n,) * d)
    xk = np.zeros_like(b)
    errs = []
    for _ in range(8):
        r = b - box.apply_op(xk, c0, c1, kinds)
        xk = xk + box.vcycle(r, c0, c1, kinds)
        if field == "p" and c0 == 0.0:
            xk -= xk.mean()
        errs.append(np.abs(xk - xe).max())
    scale = np.abs(xe).max()
    # contraction per cycle while above rounding (a strongly diagonal problem
    # reaches it in a cycle or two)
    ratios = [errs[i + 1] / errs[i] for i in range(len(errs) - 1) if errs[i + 1] > 1e-12 * scale]
    assert all(q < 0.5 for q in ratios[1:]), errs
    assert errs[-1] < 1e-3 * scale


@pytest.mark.parametrize("d", [2, 3])
def test_constrained_solve_meets_the_system(d):
    rng = np.random.default_rng(6)
    n = 8 if d == 3 else 16
    h = 1.0 / n
    wl = (True,) * d
    R = rng.uniform(0.25, 0.75, (6, d))
    for c0 in (0.0, 10.0):
        sysm = box.System(d, n, h, c0, 1.0, R, wl)
        W = rng.standard_normal((6, d))
        sol = box.constrained.solve(sysm, None, None, W, np.array([0, 6]), R.mean(axis=0)[None, :])
        rm, rc, rl = box.residual(sysm, sol.v, sol.p, sol.lam, None, None, W)
        assert np.abs(rm).max() < 1e-9 * np.abs(sysm.spread(sol.lam)).max()
        assert np.abs(rc).max() < 1e-9 * np.abs(sol.v).max() / h
        assert np.abs(rl).max() < 1e-10 * np.abs(W).max()
    # adjointness and zero tangential velocity on a wall
    v = rng.standard_normal((d,) + (n,) * d)
    for a in range(d):
        v[a][box.wall_mask(n, d, wl, a)] = 0.0
    lam = rng.standard_normal((6, d))
    lhs = np.sum(sysm.interp(v) * lam)
    rhs = np.sum(v * sysm.spread(lam)) * h ** d
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    Rw = R.copy()
    Rw[:, 0] = 1e-12                          # on the x = 0 wall (inside by a hair)
    sw = box.System(d, n, h, c0, 1.0, Rw, wl)
    u = sw.interp(v)
    assert np.abs(u[:, 1:]).max() < 1e-9 * np.abs(v).max()   # tangential components vanish
    with pytest.raises(ValueError):
        box.System(d, n, h, c0, 1.0, R - 0.5, wl)


@pytest.mark.parametrize("d", [2, 3])
def test_advection_reproduces_the_slit_and_follows_the_axes(d):
    rng = np.random.default_rng(8)
    n = 8
    h, dt = 1.0 / n, 0.02
    wl = (False,) * (d - 1) + (True,)
    v = rng.standard_normal((d,) + (n,) * d)
    v[d - 1][0] = 0.0
    assert np.abs(box.advection(v, h, wl) - walls.advection(v, h)).max() < 1e-13 * np.abs(v).max() ** 2 / h
    assert np.abs(box.advection_sl(v, h, dt, wl) - walls.advection_sl(v, h, dt)).max() < 1e-12 / dt
    if d == 3:
        # walls on x and z; swapping x and y maps the terms onto themselves
        wa, wb = (True, False, True), (False, True, True)
        v = rng.standard_normal((d,) + (n,) * d)
        for a in range(d):
            v[a][box.wall_mask(n, d, wa, a)] = 0.0
        vs = np.swapaxes(v[[1, 0, 2]], 2, 3)
        for fa, fb in ((box.advection(v, h, wa), box.advection(vs, h, wb)),
                       (box.advection_sl(v, h, dt, wa), box.advection_sl(vs, h, dt, wb))):
            assert np.abs(np.swapaxes(fb[[1, 0, 2]], 2, 3) - fa).max() < 1e-12 * np.abs(fa).max()


def test_box_steps_reproduce_the_slit():
    """Two unsteady steps with walls on the last axis only equal the slit
    oracle's trajectory (the box's stepping adds nothing of its own)."""
    from synthetic import slit_problem
    prob = slit_problem(5, dim=2, n=16, nbodies=1, radius_h=3.0, wall_gap_h=2.0, rotate=False,
                        rho=1.0, dt=0.5 / 16, eta=0.05)
    a = box.run(prob, 2, walls=(False, True))
    b = walls.run(prob, 2)
    for sa, sb in zip(a, b):
        assert np.abs(sa.v - sb.v).max() < 1e-10 * np.abs(sb.v).max()
        assert np.abs(sa.F - sb.F).max() < 1e-10 * np.abs(sb.F).max()


# ---------------------------------------------------------------- moving walls
@pytest.mark.parametrize("d,wl", [(2, (True, True)), (3, (True, True, True)), (3, (False, False, True))])
def test_padded_lattice_matches_the_folded_operators(d, wl):
    """With the walls at rest the padded-lattice stencils and interpolation
    (written separately) equal the folded ones."""
    rng = np.random.default_rng(11)
    n = 8
    h = 1.0 / n
    v, p = _fields(rng, d, n, wl)
    mv, mc = box.stokes_apply(v, p, 2.0, 0.7, h, wl)
    pv, pc = box.stokes_apply_padded(v, p, 2.0, 0.7, h, wl, None)
    assert np.abs(pv - mv).max() < 1e-11 * np.abs(mv).max() and np.abs(pc - mc).max() < 1e-11 * np.abs(mc).max()
    R = rng.uniform(0.02, 0.98, (9, d))
    sysm = box.System(d, n, h, 0.0, 1.0, R, wl)
    assert np.abs(box.interp_padded(v, R, h, wl, None) - sysm.interp(v)).max() < 1e-13 * np.abs(v).max()


def _rigid_problem(d, n, R, U, rho=0.0, eta=1.0, dt=0.0):
    from synthetic.workloads import _assemble
    c = R.mean(axis=0)
    return _assemble(d, n, 1.0 / n, rho, eta, dt, [R], c[None, :], np.asarray(U, dtype=np.float64)[None, :],
                     np.zeros((1, 3 if d == 3 else 1)), [0.1], 0, "moving_walls")


@pytest.mark.parametrize("d", [2, 3])
def test_box_moving_with_a_body_carries_the_fluid(d):
    """Every wall and the body moving with the same U: the fluid moves with U
    everywhere, with no force on the body (steady and unsteady)."""
    from synthetic import fibonacci_sphere, disk_ring
    n = 8 if d == 3 else 16
    h = 1.0 / n
    U = np.array([0.7, -0.4, 0.3][:d])
    R = fibonacci_sphere(20, 2.0 * h, np.full(3, 0.5)) if d == 3 else disk_ring(12, 3.0 * h, np.full(2, 0.5))
    wv = {beta: (U, U) for beta in range(d)}
    for rho, dt in ((0.0, 0.0), (1.0, 0.05)):
        prob = _rigid_problem(d, n, R, U, rho=rho, dt=dt)
        # the uniform flow's own inertia term (rho / dt) U is the right-hand side
        g = None if rho == 0.0 else np.stack([np.full((n,) * d, (rho / dt) * U[a]) for a in range(d)])
        sol = box.solve_problem_moving(prob, wv, g=g)
        for a in range(d):
            assert np.abs(sol.v[a] - U[a]).max() < 1e-10
        assert np.abs(sol.lam).max() < 1e-8


def test_slit_couette_is_linear():
    """Slit channel (walls on y, 2D), the bottom wall at rest and the top one
    sliding with U: the discrete flow is the linear profile exactly; a marker
    moving with the local fluid velocity feels no force."""
    n = 16
    h = 1.0 / n
    U = 0.8
    wl = (False, True)
    wv = {1: (np.zeros(2), np.array([U, 0.0]))}
    c = np.array([0.5, 0.375])
    # one marker (a rigid body of several would not follow the shear)
    prob = _rigid_problem(2, n, c[None, :], [U * c[1], 0.0])
    sol = box.solve_problem_moving(prob, wv, walls=wl)
    y = (np.arange(n) + 0.5) * h
    assert np.abs(sol.v[0] - (U * y)[:, None]).max() < 1e-12
    assert np.abs(sol.v[1]).max() < 1e-12 and np.abs(sol.lam).max() < 1e-9


@pytest.mark.parametrize("d", [2, 3])
def test_moving_walls_equal_the_shifted_frame(d):
    """The box's walls moving with U around a body at rest equal, shifted by
    U, the box at rest around the body moving with -U (steady Stokes)."""
    from synthetic import box_problem
    prob = box_problem(4, dim=d, n=8 if d == 3 else 16, nbodies=1, radius_h=2.0 if d == 3 else 3.0,
                       wall_gap_h=1.0, rotate=False)
    U = np.array([0.6, -0.3, 0.2][:d])
    lab = _rigid_problem(d, prob.n, prob.R, np.zeros(d))
    wv = {beta: (U, U) for beta in range(d)}
    sl = box.solve_problem_moving(lab, wv)
    cav = _rigid_problem(d, prob.n, prob.R, -U)
    sc = box.solve_problem(cav)
    for a in range(d):
        assert np.abs(sl.v[a] - (sc.v[a] + U[a])).max() < 1e-10 * np.abs(U).max()
    assert np.abs(sl.lam - sc.lam).max() < 1e-9 * np.abs(sc.lam).max()
