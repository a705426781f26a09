"""GPU parity of free kinematics (bodies moving under applied force and torque)
against the oracle, through the C ABI.

* operator: the enlarged matrix (marker rows -J v + K U on free bodies, body
  rows K* Lambda, identity rows for prescribed bodies) applied to random
  vectors equals the oracle's constrained operator plus its rigid map K, to
  rounding (1e-12 relative);
* preconditioner: the per-body saddle step after the fluid solve equals the
  oracle's (1e-9, fp64);
* solves: fp64 at rtol 1e-10 matches the oracle's exact free-kinematics
  solution (v, pi, F, T and the free bodies' U, Omega within 1e-8 relative
  L2; Lambda within 1e-6 raw); mixed precision at rtol 1e-8 within 1e-6;
* state: ibr_step refuses free bodies, and clearing the free set gives back
  the prescribed-motion solve.
"""
import numpy as np
import pytest

from oracle import constrained, dense, free, precond
from synthetic import small_problem

pytestmark = pytest.mark.gpu

CASES = {
    "3d32_steady_mixedset": (dict(dim=3, n=32, nbodies=3, radius_h=3.0), [1, 0, 1]),
    "3d16_unsteady_one": (dict(dim=3, n=16, nbodies=1, radius_h=2.5, rho=1.0, dt=0.5 / 16, eta=0.05), [1]),
    "2d64_steady_all": (dict(dim=2, n=64, nbodies=2, radius_h=5.0), [1, 1]),
    "2d32_unsteady_mixedset": (dict(dim=2, n=32, nbodies=2, radius_h=4.0, rho=1.0, dt=0.5 / 32, eta=0.02), [0, 1]),
}


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _loads(prob, seed):
    rng = np.random.default_rng(seed)
    nr = 3 if prob.dim == 3 else 1
    return rng.uniform(-1, 1, (prob.nbodies, prob.dim)), rng.uniform(-1, 1, (prob.nbodies, nr))


@pytest.fixture(params=sorted(CASES))
def case(request):
    kw, mask = CASES[request.param]
    return small_problem(23, **kw), mask, request.param


def _body_block(prob, z):
    """Split the body block of the library's layout into [nb, d + rotations] rows."""
    d, nb = prob.dim, prob.nbodies
    nr = 3 if d == 3 else 1
    U = z[:nb * d].reshape(nb, d)
    Om = z[nb * d:nb * d + nb * nr].reshape(nb, nr)
    return np.concatenate([U, Om], axis=1)


def _solver(prob, mask, F, T, **kw):
    """The oracle's preconditioner uses the analytic approximate mobility."""
    from paper_1505_07865_amd import ibr
    kw.setdefault("mobility", ibr.MOB_ANALYTIC)
    s = ibr.from_problem(prob, **kw)
    s.set_free_bodies(mask, F, T)
    return s


def test_free_operator_matches_oracle(case):
    prob, mask, name = case
    print("case", name, flush=True)
    F, T = _loads(prob, 1)
    s = _solver(prob, mask, F, T)
    d, nb, N = prob.dim, prob.nbodies, prob.nmarkers
    nr = 3 if d == 3 else 1
    base = (d + 1) * prob.n ** d + d * N
    assert s.NV == base + nb * (d + nr)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(s.NV)
    y = s.apply_operator(x)
    sysm = constrained.System.from_problem(prob)
    ye = np.concatenate([dense.apply_operator(sysm, x[:base]), np.zeros(s.NV - base)])
    bodies = [b for b in range(nb) if mask[b]]
    K = free.rigid_matrix(prob.R, prob.offsets, prob.centres, prob.L, bodies)
    xb = _body_block(prob, x[base:])
    ye[(d + 1) * prob.n ** d:base] += K @ np.concatenate([xb[b] for b in bodies])
    lam = x[(d + 1) * prob.n ** d:base]
    yb = xb.copy()
    kt = K.T @ lam
    q = d + nr
    for j, b in enumerate(bodies):
        yb[b] = kt[j * q:(j + 1) * q]
    ye[base:base + nb * d] = yb[:, :d].reshape(-1)
    ye[base + nb * d:] = yb[:, d:].reshape(-1)
    assert np.abs(y - ye).max() <= 1e-12 * np.abs(ye).max()
    s.close()


def test_free_preconditioner_matches_oracle(case):
    from paper_1505_07865_amd import ibr
    prob, mask, name = case
    print("case", name, flush=True)
    F, T = _loads(prob, 2)
    s = _solver(prob, mask, F, T, pc=ibr.PC_LOWER, n_s=2)
    sysm = constrained.System.from_problem(prob)
    P = precond.for_problem(prob, sysm, ns=2, full=False, free=mask)
    d, n, N, nb = prob.dim, prob.n, prob.nmarkers, prob.nbodies
    nv, npr = d * n ** d, n ** d
    base = nv + npr + d * N
    rng = np.random.default_rng(9)
    r = np.concatenate([dense.apply_operator(sysm, rng.standard_normal(base)), rng.standard_normal(s.NV - base)])
    z = s.precondition(r)
    zv, zp, zl, zu = P.apply(r[:nv].reshape((d,) + (n,) * d), r[nv:nv + npr].reshape((n,) * d),
                             r[nv + npr:base].reshape(N, d), _body_block(prob, r[base:]))
    assert _rel(z[:nv].reshape(zv.shape), zv) < 1e-9
    gp = z[nv:nv + npr]
    assert _rel(gp - gp.mean(), (zp - zp.mean()).reshape(-1)) < 1e-9
    assert _rel(z[nv + npr:base].reshape(zl.shape), zl) < 1e-9
    assert _rel(_body_block(prob, z[base:]), zu) < 1e-9
    s.close()


def test_free_solve_fp64_matches_oracle(case):
    prob, mask, name = case
    print("case", name, flush=True)
    F, T = _loads(prob, 4)
    s = _solver(prob, mask, F, T, rtol=1e-10)
    info = s.solve()
    sol = s.solution()
    U, Om = s.velocities()
    s.close()
    ex, Uf, Of = free.solve_problem(prob, mask, F, T)
    print("iters", info["iters"], "rel residual %.2e" % info["rel_residual"], flush=True)
    assert info["rel_residual"] <= 1e-10
    assert _rel(sol.u, ex.v) < 1e-8
    assert _rel(sol.p, ex.p) < 1e-8
    assert _rel(sol.F, ex.F) < 1e-8
    assert _rel(sol.T, ex.T) < 1e-8
    assert _rel(sol.lam, ex.lam) < 1e-6
    fr = np.array(mask, dtype=bool)
    assert _rel(U[fr], Uf[fr]) < 1e-8
    assert _rel(Om[fr], Of[fr]) < 1e-8
    # prescribed bodies report their prescribed motion; free ones carry their load
    assert np.array_equal(U[~fr], prob.U[~fr]) and np.array_equal(Om[~fr], prob.Omega[~fr])
    assert np.abs(sol.F[fr] - F[fr]).max() <= 1e-8 * np.abs(F).max()


@pytest.mark.parametrize("name", ["3d32_steady_mixedset", "2d64_steady_all"])
def test_free_solve_mixed_precision(name):
    from paper_1505_07865_amd import ibr
    kw, mask = CASES[name]
    prob = small_problem(23, **kw)
    F, T = _loads(prob, 5)
    s = _solver(prob, mask, F, T, rtol=1e-8, precision=ibr.MIXED)
    info = s.solve()
    sol = s.solution()
    U, Om = s.velocities()
    s.close()
    ex, Uf, Of = free.solve_problem(prob, mask, F, T)
    assert info["rel_residual"] <= 1e-8
    fr = np.array(mask, dtype=bool)
    assert _rel(sol.u, ex.v) < 1e-6
    assert _rel(U[fr], Uf[fr]) < 1e-6
    assert _rel(Om[fr], Of[fr]) < 1e-6


def test_free_state_changes():
    from paper_1505_07865_amd import ibr
    kw, mask = CASES["3d16_unsteady_one"]
    prob = small_problem(23, **kw)
    F, T = _loads(prob, 6)
    s = _solver(prob, mask, F, T, rtol=1e-10)
    with pytest.raises(ibr.IbrError):
        s.step()
    s.solve()
    # a second load on the same bodies
    s.set_free_bodies(mask, 2.0 * F, 2.0 * T)
    s.solve()
    U2, Om2 = s.velocities()
    _, Uf, Of = free.solve_problem(prob, mask, 2.0 * F, 2.0 * T)
    assert _rel(U2, Uf) < 1e-8 and _rel(Om2, Of) < 1e-8
    # back to prescribed motion: the plain constrained solve
    s.set_free_bodies(None)
    assert s.NV == (prob.dim + 1) * prob.n ** prob.dim + prob.dim * prob.nmarkers
    s.solve()
    sol = s.solution()
    ex = constrained.solve_problem(prob)
    assert _rel(sol.u, ex.v) < 1e-8 and _rel(sol.F, ex.F) < 1e-8
    s.close()
