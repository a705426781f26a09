"""Pins of the free-kinematics oracle (bodies moving under applied loads).

* the Schur route of ``oracle.free`` equals the whole enlarged system
  assembled densely (stencils, marker velocities of unit rigid motions, body
  force/torque sums) and solved by LAPACK;
* the body resistance matrix built from prescribed-motion solves of
  ``oracle.constrained`` (an independently pinned path) is symmetric positive
  definite (Lorentz reciprocity holds for the discrete system), and the free
  solve under any load returns exactly its inverse applied to that load;
* prescribing the velocities the free solve returned gives back its fields,
  and the bodies then carry exactly their applied loads.
"""
import numpy as np
import pytest

from oracle import constrained, dense, free, ib
from synthetic import small_problem


def _loads(rng, nb, d):
    return rng.uniform(-1, 1, size=(nb, d)), rng.uniform(-1, 1, size=(nb, 3 if d == 3 else 1))


CASES = [
    dict(dim=2, n=16, radius_h=3.0, nbodies=2, gap_h=2.0),
    dict(dim=2, n=16, radius_h=3.0, nbodies=2, gap_h=2.0, rho=1.0, dt=0.02),
    dict(dim=3, n=8, radius_h=1.5),
    dict(dim=3, n=8, radius_h=1.5, rho=1.0, dt=0.05, eta=0.3),
]


def _fluid_rhs(prob, rng):
    d, n = prob.dim, prob.n
    g = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    hp -= hp.mean()
    if prob.steady:
        g -= g.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    return g, hp


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("fluid_rhs", [False, True])
def test_free_schur_equals_dense(case, fluid_rhs, rng):
    prob = small_problem(7, **case)
    nb = prob.nbodies
    mask = [1] * nb if nb == 1 else [1, 0]          # 2D: one free disk beside a prescribed one
    F, T = _loads(rng, nb, prob.dim)
    g, hp = _fluid_rhs(prob, rng) if fluid_rhs else (None, None)
    sysm = constrained.System.from_problem(prob)
    W = free.constraint_rhs(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L, mask)
    sol, Uf, Of = free.solve(sysm, g, hp, W, prob.offsets, prob.centres, mask, F, T)
    v, p, lam, Ud, Od = dense.solve_free(sysm, g, hp, W, prob.offsets, prob.centres, mask, F, T)
    p = p - p.mean()
    assert np.abs(sol.v - v).max() <= 1e-10 * np.abs(v).max()
    assert np.abs(sol.p - p).max() <= 1e-10 * np.abs(p).max()
    assert np.abs(sol.lam - lam).max() <= 1e-10 * np.abs(lam).max()
    assert np.abs(Uf - Ud).max() <= 1e-10 * np.abs(Ud).max()
    assert np.abs(Of - Od).max() <= 1e-10 * max(np.abs(Od).max(), 1e-300)
    # the free body hands its applied load to the fluid
    for b in range(nb):
        if mask[b]:
            assert np.allclose(sol.F[b], F[b], rtol=0, atol=1e-10 * np.abs(F).max())
            assert np.allclose(sol.T[b], T[b], rtol=0, atol=1e-10 * np.abs(T).max())


def _resistance(prob):
    """Columns: body forces and torques for a unit velocity of one rigid mode
    (all other bodies held at rest), from prescribed-motion solves."""
    d, nb = prob.dim, prob.nbodies
    nr = 3 if d == 3 else 1
    q = d + nr
    sysm = constrained.System.from_problem(prob)
    Rm = np.zeros((q * nb, q * nb))
    for p in range(nb):
        for k in range(q):
            U = np.zeros((nb, d))
            Om = np.zeros((nb, nr))
            if k < d:
                U[p, k] = 1.0
            else:
                Om[p, k - d] = 1.0
            V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, U, Om, prob.L)
            sol = constrained.solve(sysm, None, None, -V, prob.offsets, prob.centres)
            Rm[:, p * q + k] = np.concatenate([np.concatenate([sol.F[b], sol.T[b]]) for b in range(nb)])
    return Rm


@pytest.mark.parametrize("case", [dict(dim=2, n=32, radius_h=4.0, nbodies=2),
                                  dict(dim=3, n=16, radius_h=2.5)])
def test_free_velocities_are_inverse_resistance(case, rng):
    prob = small_problem(11, **case)
    nb, d = prob.nbodies, prob.dim
    Rm = _resistance(prob)
    assert np.abs(Rm - Rm.T).max() <= 1e-10 * np.abs(Rm).max()      # reciprocity
    assert np.linalg.eigvalsh(0.5 * (Rm + Rm.T)).min() > 0           # dissipation
    F, T = _loads(rng, nb, d)
    mask = [1] * nb
    sol, Uf, Of = free.solve_problem(prob, mask, F, T)
    f = np.concatenate([np.concatenate([F[b], T[b]]) for b in range(nb)])
    u = np.concatenate([np.concatenate([Uf[b], Of[b]]) for b in range(nb)])
    assert np.abs(Rm @ u - f).max() <= 1e-9 * np.abs(f).max()


@pytest.mark.parametrize("case", [dict(dim=2, n=32, radius_h=4.0, nbodies=3),
                                  dict(dim=3, n=16, radius_h=2.5, nbodies=2)])
def test_prescribing_free_velocities_round_trip(case, rng):
    prob = small_problem(13, **case)
    nb, d = prob.nbodies, prob.dim
    mask = [1, 0] + [1] * (nb - 2)
    F, T = _loads(rng, nb, d)
    sol, Uf, Of = free.solve_problem(prob, mask, F, T)
    U = np.where(np.array(mask)[:, None] == 1, Uf, prob.U)
    Om = np.where(np.array(mask)[:, None] == 1, Of, prob.Omega)
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, U, Om, prob.L)
    ref = constrained.solve(constrained.System.from_problem(prob), None, None, -V, prob.offsets, prob.centres)
    assert np.abs(ref.v - sol.v).max() <= 1e-10 * np.abs(sol.v).max()
    assert np.abs(ref.lam - sol.lam).max() <= 1e-9 * np.abs(sol.lam).max()
    for b in range(nb):
        if mask[b]:
            assert np.abs(ref.F[b] - F[b]).max() <= 1e-9 * np.abs(F).max()
            assert np.abs(ref.T[b] - T[b]).max() <= 1e-9 * np.abs(T).max()


def test_cg_route_equals_dense_route(rng):
    prob = small_problem(17, 3, 16, radius_h=2.5, nbodies=2)
    F, T = _loads(rng, 2, 3)
    a, Ua, Oa = free.solve_problem(prob, [1, 1], F, T)
    b, Ub, Ob = free.solve_problem(prob, [1, 1], F, T, dense_limit=0, tol=1e-13)
    assert np.abs(a.lam - b.lam).max() <= 1e-9 * np.abs(a.lam).max()
    assert np.abs(np.concatenate([Ua, Oa], 1) - np.concatenate([Ub, Ob], 1)).max() <= \
        1e-9 * np.abs(np.concatenate([Ua, Oa], 1)).max()


@pytest.mark.parametrize("case", [dict(dim=2, n=32, radius_h=4.0, nbodies=3),
                                  dict(dim=3, n=16, radius_h=2.5, nbodies=2)])
def test_preconditioner_body_step_solves_its_saddle_problem(case, rng):
    """The per-body step of the preconditioner with free bodies solves
    M~_p Lambda_p - K_p U_p = dU_p and K_p* Lambda_p = r_U,p exactly, and
    passes prescribed bodies' rows through."""
    from oracle import mobility, precond
    prob = small_problem(19, **case)
    nb, d = prob.nbodies, prob.dim
    mask = [1, 0] + [1] * (nb - 2)
    sysm = constrained.System.from_problem(prob)
    P = precond.for_problem(prob, sysm, ns=2, free=mask)
    rv = rng.standard_normal((d,) + (prob.n,) * d)
    rv -= rv.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    rp = rng.standard_normal((prob.n,) * d)
    rp -= rp.mean()
    rl = rng.standard_normal((prob.nmarkers, d))
    ru = rng.standard_normal((nb, d + (3 if d == 3 else 1)))
    v, p, lam, zu = P.apply(rv, rp, rl, ru)
    dU = -(sysm.interp(v) + rl)
    blocks, mp = mobility.blocks_for_problem(prob)
    f0 = mobility.self_term(mp)
    for b in range(nb):
        lo, hi = prob.offsets[b], prob.offsets[b + 1]
        if not mask[b]:
            assert np.array_equal(zu[b], ru[b])
            continue
        Kb = free.rigid_matrix(prob.R, prob.offsets, prob.centres, prob.L, [b])[lo * d:hi * d]
        Mb = blocks[b] + P.shifts[b] * f0 * np.eye(blocks[b].shape[0])    # the block M~ the factor is of
        res1 = Mb @ lam[lo:hi].reshape(-1) - Kb @ zu[b] - dU[lo:hi].reshape(-1)
        assert np.abs(res1).max() <= 1e-9 * np.abs(dU[lo:hi]).max()
        F, T = ib.body_force_torque(lam, prob.R, prob.offsets, prob.centres, prob.L)
        assert np.abs(np.concatenate([F[b], T[b]]) - ru[b]).max() <= 1e-10 * np.abs(ru[b]).max()
