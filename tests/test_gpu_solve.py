"""GPU solves against the oracle's exact solution of eq. constrained_Stokes.

Bars (Sec. 3 system, tolerances derived from the FGMRES stopping rule):
* fp64 at rtol 1e-10: v, pi, F, T within 1e-8 relative L2 of the exact solution;
  Lambda within 1e-8 after projecting out the near-null compression modes of
  the true mobility (Sec. 3.3), raw Lambda within 1e-6;
* mixed (fp32 preconditioner, fp64 outer) at rtol 1e-8: the true residual meets
  the tolerance, v, F, T are within 1e-8 of the exact solution, and on the
  64^3 sphere within 10x of the fp64 solve's error at the same rtol; the
  steady periodic gauge <v> = 0 (eq. constrained_periodic) holds to 1e-12 of
  max |v| in both precisions;
* every solve reports a recomputed fp64 residual below rtol.
"""
import numpy as np
import pytest

from oracle import constrained, ib, navier
from synthetic import config0_disk2d, config1_sphere3d, small_problem

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _lam_projected_error(prob, lam, ex_lam):
    """Lambda error outside the modes of the true mobility with tiny eigenvalues."""
    sysm = constrained.System.from_problem(prob)
    M = sysm.mobility_dense()
    w, Q = np.linalg.eigh(0.5 * (M + M.T))
    keep = w > 1e-4 * w.max()
    d = (lam - ex_lam).reshape(-1)
    dp = Q[:, keep] @ (Q[:, keep].T @ d)
    return np.linalg.norm(dp) / np.linalg.norm(ex_lam)


def _solve(prob, **kw):
    from paper_1505_07865_amd import ibr
    s = ibr.from_problem(prob, **kw)
    info = s.solve()
    sol = s.solution()
    s.close()
    return info, sol


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_disk2d_fp64(seed):
    prob = config0_disk2d(seed)
    print("disk2d seed", seed, flush=True)
    info, sol = _solve(prob, rtol=1e-10)
    ex = constrained.solve_problem(prob)
    assert info["rel_residual"] <= 1e-10
    assert _rel(sol.u, ex.v) < 1e-8
    assert _rel(sol.p, ex.p) < 1e-8
    assert _rel(sol.F, ex.F) < 1e-8
    assert _lam_projected_error(prob, sol.lam, ex.lam) < 1e-8
    assert _rel(sol.lam, ex.lam) < 1e-6


@pytest.mark.parametrize("kw", [dict(dim=3, n=32, nbodies=3, radius_h=3.0),
                                dict(dim=3, n=16, nbodies=1, radius_h=2.5, rho=1.0, dt=0.5 / 16, eta=0.05),
                                dict(dim=2, n=64, nbodies=2, radius_h=5.0, rho=1.0, dt=0.5 / 64, eta=0.01)])
def test_small_multibody_fp64(kw):
    prob = small_problem(13, **kw)
    print("small", kw, flush=True)
    info, sol = _solve(prob, rtol=1e-10)
    ex = constrained.solve_problem(prob)
    assert info["rel_residual"] <= 1e-10
    assert _rel(sol.u, ex.v) < 1e-8
    assert _rel(sol.p, ex.p) < 1e-8
    assert _rel(sol.F, ex.F) < 1e-8
    assert _rel(sol.T, ex.T) < 1e-8


_SPHERE_EXACT = {}


def _sphere_exact(seed):
    if seed not in _SPHERE_EXACT:
        _SPHERE_EXACT[seed] = constrained.solve_problem(config1_sphere3d(seed))
    return _SPHERE_EXACT[seed]


def _gauge(sol):
    return np.abs(sol.u.reshape(sol.u.shape[0], -1).mean(axis=1)).max() / np.abs(sol.u).max()


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sphere3d_config(precision, seed):
    from paper_1505_07865_amd import ibr
    prob = config1_sphere3d(seed)
    print("sphere3d 64^3", precision, "seed", seed, flush=True)
    rtol = 1e-10 if precision == "fp64" else 1e-8
    info, sol = _solve(prob, rtol=rtol, precision=ibr.FP64 if precision == "fp64" else ibr.MIXED)
    ex = _sphere_exact(seed)
    print("iters", info["iters"], "err v %.2e F %.2e T %.2e gauge %.1e" % (
        _rel(sol.u, ex.v), _rel(sol.F, ex.F), _rel(sol.T, ex.T), _gauge(sol)), flush=True)
    assert info["rel_residual"] <= rtol
    bar = 1e-8
    assert _rel(sol.u, ex.v) < bar
    assert _rel(sol.F, ex.F) < bar
    assert _rel(sol.T, ex.T) < bar
    assert _gauge(sol) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_sphere3d_mixed_error_near_fp64(seed):
    """At the same rtol (1e-8) the mixed solve's error against the oracle is
    within 10x of the fp64 solve's: the outer fp64 iteration wins back what
    the fp32 preconditioner loses, the null directions of the steady periodic
    operator included (their gauge is fixed in fp64)."""
    from paper_1505_07865_amd import ibr
    prob = config1_sphere3d(seed)
    ex = _sphere_exact(seed)
    errs = {}
    for name, prec in (("fp64", ibr.FP64), ("mixed", ibr.MIXED)):
        info, sol = _solve(prob, rtol=1e-8, precision=prec)
        assert info["rel_residual"] <= 1e-8
        errs[name] = max(_rel(sol.u, ex.v), _rel(sol.F, ex.F), _rel(sol.T, ex.T))
        print(name, "seed", seed, "iters", info["iters"], "err %.2e" % errs[name], flush=True)
    assert errs["mixed"] <= 10.0 * max(errs["fp64"], 1e-12), errs


def test_full_preconditioner_same_answer():
    from paper_1505_07865_amd import ibr
    prob = small_problem(3, 3, 32, nbodies=2, radius_h=3.0)
    i1, s1 = _solve(prob, rtol=1e-10, pc=ibr.PC_LOWER)
    i2, s2 = _solve(prob, rtol=1e-10, pc=ibr.PC_FULL, n_s=4)
    assert _rel(s1.u, s2.u) < 1e-8
    assert i2["ps_applications"] >= 2 * 4 * i2["iters"]


def test_unsteady_steps_match_oracle():
    from paper_1505_07865_amd import ibr
    prob = small_problem(17, 3, 16, nbodies=2, radius_h=2.0, rho=1.0, dt=0.5 / 16, eta=0.02, nsteps=3,
                         rotate=False)
    s = ibr.from_problem(prob, rtol=1e-11)
    ex = navier.run(prob, 3)
    for k in range(3):
        info = s.step()
        sol = s.solution()
        print("step", k, info["iters"], _rel(sol.u, ex[k].v), flush=True)
        assert info["rel_residual"] <= 1e-11
        assert _rel(sol.u, ex[k].v) < 1e-8
        assert _rel(sol.F, ex[k].F) < 1e-8
    R, X = s.markers()
    b = ib.body_of(prob.offsets)
    Re = np.mod(prob.R + 3 * prob.dt * prob.U[b], prob.L)
    assert np.abs(ib.min_image(R - Re, prob.L)).max() < 1e-12
    s.close()


def test_repeat_solve_bitwise_deterministic():
    prob = small_problem(2, 3, 16, nbodies=1, radius_h=3.0)
    _, a = _solve(prob, rtol=1e-10)
    _, b = _solve(prob, rtol=1e-10)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.lam, b.lam)


def test_edge_cases():
    from paper_1505_07865_amd import ibr
    # a single marker, sitting on the periodic boundary
    s = ibr.Solver(dim=3, n=16, h=1.0 / 16, rtol=1e-10)
    R = np.array([[0.0, 1.0 - 1e-15, 0.5]])
    s.set_bodies(R, [0, 1], R.copy())
    s.set_velocities([[1.0, 0.0, 0.0]], [[0.0, 0.0, 0.0]])
    info = s.solve()
    sol = s.solution()
    ex = constrained.solve(constrained.System(3, 16, 1.0 / 16, 0.0, 1.0, np.mod(R, 1.0)), None, None,
                           -np.array([[1.0, 0.0, 0.0]]), np.array([0, 1]), np.mod(R, 1.0))
    assert _rel(sol.u, ex.v) < 1e-8
    # zero velocities: zero solution, zero iterations
    s.set_velocities([[0.0, 0.0, 0.0]], [[0.0, 0.0, 0.0]])
    info = s.solve()
    assert info["iters"] == 0 and np.abs(s.solution().u).max() == 0.0
    # max_iters reached -> IBR_ENOCONV with the iterate kept
    s2 = ibr.Solver(dim=3, n=16, h=1.0 / 16, rtol=1e-14, max_iters=2)
    s2.set_bodies(R, [0, 1], R.copy())
    s2.set_velocities([[1.0, 0.0, 0.0]], [[0.0, 0.0, 0.0]])
    with pytest.raises(ibr.IbrError) as e:
        s2.solve()
    assert e.value.status == 3
    # invalid bodies are rejected
    with pytest.raises(ibr.IbrError) as e:
        s2.set_bodies(R, [0, 0], R.copy())
    assert e.value.status == 1
    with pytest.raises(ibr.IbrError) as e:
        s2.set_bodies(np.array([[np.nan, 0, 0]]), [0, 1], R.copy())
    assert e.value.status == 1
    # a time step translates the bodies: rotating bodies are refused
    s3 = ibr.Solver(dim=3, n=16, h=1.0 / 16, rho=1.0, dt=0.01, rtol=1e-10)
    s3.set_bodies(R, [0, 1], R.copy())
    s3.set_velocities([[1.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]])
    with pytest.raises(ibr.IbrError) as e:
        s3.step()
    assert e.value.status == 1
    s3.set_velocities([[1.0, 0.0, 0.0]], [[0.0, 0.0, 0.0]])
    assert s3.step()["rel_residual"] <= 1e-10
    s.close()
    s2.close()
    s3.close()


def test_graph_replay_matches_stream_launches():
    """Captured iteration graphs replayed across restarts and steps give the
    bitwise result of plain stream launches (the same kernels in the same order)."""
    from paper_1505_07865_amd import ibr
    prob = small_problem(23, 3, 32, nbodies=2, radius_h=3.0, rho=1.0, dt=0.5 / 32, eta=0.02, nsteps=3,
                         rotate=False)
    out = []
    for graphs in (1, 0):
        s = ibr.from_problem(prob, rtol=1e-10, restart=6, graphs=graphs)
        sols = []
        for _ in range(3):
            info = s.step()
            sols.append(s.solution())
            assert info["restarts"] >= 2      # graphs are replayed across restart cycles
        out.append(sols)
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a.u, b.u) and np.array_equal(a.lam, b.lam) and np.array_equal(a.p, b.p)


def test_device_pointer_rhs_and_solution():
    """ibr_set_rhs_dev / ibr_get_solution_dev (torch tensors on the GPU) give
    bitwise the host-pointer results; host memory is rejected."""
    import torch
    from paper_1505_07865_amd import ibr
    prob = small_problem(31, 3, 16, nbodies=2, radius_h=2.5)
    d, n = prob.dim, prob.n
    rng = np.random.default_rng(4)
    g = rng.standard_normal((d,) + (n,) * d)
    hp = rng.standard_normal((n,) * d)
    s = ibr.from_problem(prob, rtol=1e-10)
    s.set_rhs(g, hp)
    s.solve()
    a = s.solution()
    gd = torch.from_numpy(g).cuda()
    hd = torch.from_numpy(hp).cuda()
    s.set_rhs(None, None)
    s.set_rhs_dev(gd, hd)
    s.solve()
    u = torch.zeros((d,) + (n,) * d, dtype=torch.float64, device="cuda")
    p = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    lam = torch.zeros((prob.nmarkers, d), dtype=torch.float64, device="cuda")
    F = torch.zeros((prob.nbodies, d), dtype=torch.float64, device="cuda")
    T = torch.zeros((prob.nbodies, 3), dtype=torch.float64, device="cuda")
    s.solution_dev(u, p, lam, F, T)
    assert np.array_equal(u.cpu().numpy(), a.u) and np.array_equal(p.cpu().numpy(), a.p)
    assert np.array_equal(lam.cpu().numpy(), a.lam)
    assert np.array_equal(F.cpu().numpy(), a.F) and np.array_equal(T.cpu().numpy(), a.T)
    # the oracle's exact solution of the same system with this fluid forcing
    sysm = constrained.System.from_problem(prob)
    V = ib.marker_velocities(prob.R, prob.offsets, prob.centres, prob.U, prob.Omega, prob.L)
    gm = g - g.reshape(d, -1).mean(axis=1).reshape((d,) + (1,) * d)
    ex = constrained.solve(sysm, gm, hp - hp.mean(), -V, prob.offsets, prob.centres)
    assert _rel(a.u, ex.v) < 1e-8 and _rel(a.F, ex.F) < 1e-8
    with pytest.raises(ibr.IbrError) as e:
        s.set_rhs_dev(torch.zeros((d,) + (n,) * d, dtype=torch.float64), None)
    assert e.value.status == 1
    s.close()
    # the same solve on a caller's stream (a torch stream at default priority)
    side = torch.cuda.Stream()
    s2 = ibr.from_problem(prob, rtol=1e-10, stream=side.cuda_stream)
    s2.set_rhs_dev(gd, hd)
    s2.solve()
    b = s2.solution()
    assert np.array_equal(a.u, b.u) and np.array_equal(a.lam, b.lam)
    s2.close()


@pytest.mark.parametrize("filled,re", [(False, 0.0), (True, 0.0), (False, 10.0), (True, 10.0)])
@pytest.mark.parametrize("pc,ns", [("lower", 2), ("full", 8)])
def test_icosahedral_shell_matches_oracle(filled, re, pc, ns):
    """The solver-study geometry (162-marker icosahedral shell, empty or filled,
    steady or one Re = 10 step, 32^3): converged solutions equal the exact one
    for both preconditioners and any N_s."""
    from paper_1505_07865_amd import ibr
    from synthetic import shell_problem
    prob = shell_problem(5, 32, 2, filled=filled, re=re)
    print(prob.name, prob.nmarkers, pc, ns, flush=True)
    info, sol = _solve(prob, rtol=1e-10, pc=ibr.PC_FULL if pc == "full" else ibr.PC_LOWER, n_s=ns)
    ex = constrained.solve_problem(prob)
    assert info["rel_residual"] <= 1e-10
    assert _rel(sol.u, ex.v) < 1e-8 and _rel(sol.F, ex.F) < 1e-8
    # a translating shell (Omega = 0) feels almost no torque: measure the torque
    # error against the force's moment scale |F| R
    tscale = max(np.linalg.norm(ex.T), np.linalg.norm(ex.F) * prob.meta["radius_h"] * prob.h)
    assert np.linalg.norm(sol.T - ex.T) < 1e-8 * tscale
    per_iter = (2 if pc == "full" else 1) * ns
    assert info["ps_applications"] == per_iter * info["iters"]


@pytest.mark.parametrize("dim,n,walls", [(3, 8, 0), (2, 16, 0), (3, 8, 1), (2, 16, 1)])
def test_smallest_grids_match_oracle(dim, n, walls):
    """The smallest grids the library accepts (8^3, 16^2: the whole V-cycle in
    the one-workgroup tail, one spreading tile), periodic and between walls,
    solve to the oracle's exact answer."""
    from oracle import walls as owalls
    from synthetic import slit_problem
    from paper_1505_07865_amd import ibr
    if walls:
        prob = slit_problem(2, dim=dim, n=n, nbodies=1, radius_h=1.5 if dim == 3 else 2.5, wall_gap_h=0.5)
        ex = owalls.solve_problem(prob)
    else:
        prob = small_problem(2, dim, n, nbodies=1, radius_h=1.5 if dim == 3 else 2.5)
        ex = constrained.solve_problem(prob)
    print("smallest", dim, n, walls, prob.nmarkers, flush=True)
    s = ibr.from_problem(prob, rtol=1e-10)
    s.solve()
    sol = s.solution()
    s.close()
    assert _rel(sol.u, ex.v) < 1e-8 and _rel(sol.F, ex.F) < 1e-8
