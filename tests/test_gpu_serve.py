"""Serving: a request answered inside a concurrent mix (several workers,
resident contexts reused across grid sizes) is bitwise the answer of the same
request solved alone in a fresh context."""
import numpy as np
import pytest

from synthetic import serving_trace

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_equals_alone(precision):
    from paper_1505_07865_amd import ibr, serve
    trace = serving_trace(1, 16, 1.0)
    print("serving", precision, [(r["problem"].dim, r["problem"].n, r["problem"].nbodies) for r in trace],
          flush=True)
    with serve.Server(precision=precision, workers=3, reserve_bytes=1 << 30) as srv:
        out = serve.replay(trace, srv, qps=None)
    assert out["requests"] == len(trace)
    for req, r in zip(trace, out["results"]):
        p = req["problem"]
        s = ibr.from_problem(p, rtol=1e-8, precision=ibr.MIXED if precision == "mixed" else ibr.FP64,
                             rho=0.0, graphs=0)
        info = s.solve()
        F, T = s.forces()
        s.close()
        assert r["info"]["rel_residual"] <= 1e-8
        assert r["info"]["iters"] == info["iters"]
        assert np.array_equal(r["F"], F) and np.array_equal(r["T"], T)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_trajectories_equal_alone(precision):
    """Unsteady trajectories (from rest, 4 steps) served by 2 workers among
    steady requests, with contexts reused between trajectories (ibr_reset),
    equal the same trajectories run alone in fresh contexts, bitwise."""
    from paper_1505_07865_amd import ibr, serve
    from synthetic import config2_spheres_ns
    probs = [config2_spheres_ns(seed, re=10.0, n=32, nbodies=3, radius_h=4.0, nmark=50, nsteps=4)
             for seed in range(4)]
    steady = [r["problem"] for r in serving_trace(2, 3, 1.0)]
    print("trajectories", precision, [p.nmarkers for p in probs], "steady", [(p.dim, p.n) for p in steady],
          flush=True)
    with serve.Server(precision=precision, workers=2, reserve_bytes=1 << 30) as srv:
        futs = [srv.submit_trajectory(p, 4) for p in probs[:2]] + [srv.submit(p) for p in steady] + \
               [srv.submit_trajectory(p, 4) for p in probs[2:]]
        res = [f.result() for f in futs]
    traj = res[:2] + res[-2:]
    for p, r in zip(probs, traj):
        s = ibr.from_problem(p, rtol=1e-8, precision=ibr.MIXED if precision == "mixed" else ibr.FP64, graphs=0)
        infos = [s.step() for _ in range(4)]
        F, T = s.forces()
        s.close()
        assert [st["iters"] for st in r["steps"]] == [i["iters"] for i in infos]
        assert all(st["rel_residual"] <= 1e-8 for st in r["steps"])
        assert np.array_equal(r["F"], F) and np.array_equal(r["T"], T)


def test_served_mix_with_walls_equals_alone():
    """Slit-channel requests served among periodic requests of the same grid
    sizes (their own contexts, N_s = 4 between walls) equal the same requests
    solved alone, bitwise; so do the periodic ones."""
    from paper_1505_07865_amd import ibr, serve
    from synthetic import slit_problem, small_problem
    probs = [slit_problem(s, dim=3, n=32, nbodies=2, radius_h=3.0) for s in range(2)] + \
            [small_problem(s, 3, 32, nbodies=2, radius_h=3.0) for s in range(2)] + \
            [slit_problem(7, dim=2, n=64, nbodies=2, radius_h=4.0)]
    with serve.Server(precision="mixed", workers=3, reserve_bytes=1 << 30) as srv:
        futs = [srv.submit(p) for p in probs]
        res = [f.result() for f in futs]
    for p, r in zip(probs, res):
        kw = dict(n_s=4) if p.walls else {}
        s = ibr.from_problem(p, rtol=1e-8, precision=ibr.MIXED, graphs=0, **kw)
        info = s.solve()
        F, T = s.forces()
        s.close()
        assert r["info"]["iters"] == info["iters"]
        assert np.array_equal(r["F"], F) and np.array_equal(r["T"], T)
