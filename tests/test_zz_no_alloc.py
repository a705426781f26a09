"""The allocation-free spreading entry point (ibr_spread_noalloc) against the
context's ibr_spread on the same markers: equal to the last bit (same kernels,
same taps), on two calls in a row with the second input smaller (fewer
markers, a smaller grid and dimension), with f prefilled with NaN (the call
overwrites it), and sizes beyond the static scratch refused before any
device work."""
import numpy as np
import pytest

from synthetic import small_problem

pytestmark = pytest.mark.gpu


def _ctx_spread(prob, lam):
    from paper_1505_07865_amd import ibr
    s = ibr.from_problem(prob)
    f = s.spread(lam)
    s.close()
    return f


def _noalloc_spread(prob, lam, stream=None):
    import torch
    from paper_1505_07865_amd import ibr
    dev = torch.device("cuda:0")
    R = torch.tensor(np.ascontiguousarray(prob.R), dtype=torch.float64, device=dev)
    L = torch.tensor(np.ascontiguousarray(lam), dtype=torch.float64, device=dev)
    f = torch.full((prob.dim,) + (prob.n,) * prob.dim, float("nan"), dtype=torch.float64, device=dev)
    s = stream or torch.cuda.current_stream()
    ibr.spread_noalloc(R, L, f, stream=s, dim=prob.dim, n=prob.n, h=prob.h, walls=getattr(prob, "walls", 0))
    s.synchronize()
    return f.cpu().numpy()


def test_noalloc_spread_equals_context_spread_twice():
    import torch
    probs = [small_problem(21, 3, 32, nbodies=3, radius_h=3.0), small_problem(22, 2, 16, nbodies=1, radius_h=2.0)]
    stream = torch.cuda.Stream()
    for prob in probs:
        print("noalloc spread: %dD %d^%d, %d markers" % (prob.dim, prob.n, prob.dim, prob.nmarkers), flush=True)
        rng = np.random.default_rng(prob.nmarkers)
        lam = rng.standard_normal((prob.nmarkers, prob.dim))
        ref = _ctx_spread(prob, lam)
        got = _noalloc_spread(prob, lam, stream)
        assert np.array_equal(got, ref), np.abs(got - ref).max()


def test_noalloc_spread_with_walls_and_no_markers():
    import torch
    from paper_1505_07865_amd import ibr
    from synthetic import slit_problem
    prob = slit_problem(3, dim=3, n=16, nbodies=2, radius_h=2.5)
    print("noalloc spread: slit 16^3, %d markers" % prob.nmarkers, flush=True)
    lam = np.random.default_rng(5).standard_normal((prob.nmarkers, 3))
    assert np.array_equal(_noalloc_spread(prob, lam), _ctx_spread(prob, lam))
    f = torch.full((3, 16, 16, 16), 1.0, dtype=torch.float64, device="cuda:0")
    ibr.spread_noalloc(None, None, f, nmarkers=0, dim=3, n=16, h=1.0 / 16)
    torch.cuda.synchronize()
    assert float(f.abs().max()) == 0.0


def test_noalloc_spread_refuses_sizes_beyond_scratch():
    import torch
    from paper_1505_07865_amd import ibr
    f = torch.zeros((3, 8, 8, 8), dtype=torch.float64, device="cuda:0")
    R = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(ibr.IbrError) as e:
        ibr.spread_noalloc(R, R, f, nmarkers=104851, dim=3, n=8, h=1.0 / 8)
    assert e.value.status == 1 and "104850 markers fit" in str(e.value)
    with pytest.raises(ibr.IbrError) as e:
        ibr.spread_noalloc(R, R, f, nmarkers=88470, dim=3, n=512, h=1.0 / 512)
    assert e.value.status == 1 and "88469 markers fit" in str(e.value)
    # host memory is refused too
    Rh = np.zeros((4, 3))
    with pytest.raises(ibr.IbrError) as e:
        ibr.spread_noalloc(Rh.ctypes.data, Rh.ctypes.data, f, nmarkers=4, dim=3, n=8, h=1.0 / 8)
    assert e.value.status == 1
