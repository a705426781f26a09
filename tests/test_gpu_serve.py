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
