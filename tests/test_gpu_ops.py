"""GPU parity of single operators against the oracle (through the C ABI).

Sizes span several tiles/levels with a ragged tail (bodies crossing the
periodic boundary, more than one body, both dimensions).  Floating-point
tolerances follow from the arithmetic: fp64 stencils and sums differ from the
oracle only in rounding order (1e-12 relative); fp32 paths are checked at
1e-5.
"""
import numpy as np
import pytest

from oracle import constrained, dense, grid, ib, mobility, multigrid, navier, precond
from synthetic import small_problem

pytestmark = pytest.mark.gpu

CASES = {
    "3d32_steady": dict(dim=3, n=32, nbodies=3, radius_h=3.0),
    "3d16_unsteady": dict(dim=3, n=16, nbodies=1, radius_h=2.5, rho=1.0, dt=0.5 / 16, eta=0.05),
    "2d64_steady": dict(dim=2, n=64, nbodies=2, radius_h=5.0),
    "2d32_unsteady": dict(dim=2, n=32, nbodies=1, radius_h=4.0, rho=1.0, dt=0.5 / 32, eta=0.02),
}


def _solver(prob, **kw):
    """The oracle's preconditioner uses the analytic approximate mobility."""
    from paper_1505_07865_amd import ibr
    kw.setdefault("mobility", ibr.MOB_ANALYTIC)
    return ibr.from_problem(prob, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(params=sorted(CASES))
def case(request):
    return small_problem(21, **CASES[request.param]), request.param


def test_operator_matches_oracle(case):
    prob, name = case
    print("case", name, flush=True)
    s = _solver(prob)
    sysm = constrained.System.from_problem(prob)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(s.NV)
    y = s.apply_operator(x)
    ye = dense.apply_operator(sysm, x)
    assert _rel(y, ye) < 1e-12, _rel(y, ye)
    s.close()


def test_spread_interp_match_oracle(case):
    prob, name = case
    s = _solver(prob)
    rng = np.random.default_rng(6)
    lam = rng.standard_normal((prob.nmarkers, prob.dim))
    f = s.spread(lam)
    fe = ib.spread(lam, prob.R, prob.n, prob.h)
    assert _rel(f, fe) < 1e-13
    u = rng.standard_normal((prob.dim,) + (prob.n,) * prob.dim)
    V = s.interp(u)
    Ve = ib.interp(u, prob.R, prob.h)
    assert _rel(V, Ve) < 1e-13
    # adjointness on the device: <J u, lam> = h^d <u, S lam>
    lhs = (V * lam).sum()
    rhs = prob.h ** prob.dim * (u * f).sum()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # deterministic (atomic-free gather): bitwise equal on repeat
    assert np.array_equal(f, s.spread(lam))
    s.close()


@pytest.mark.parametrize("dim,n", [(3, 8), (3, 32), (2, 16), (2, 128)])
@pytest.mark.parametrize("c0,c1", [(0.0, 1.0), (2.5, 0.7), (0.0, -1.0)])
def test_vcycle_matches_oracle_fp64(dim, n, c0, c1):
    from paper_1505_07865_amd import ibr
    s = ibr.Solver(dim=dim, n=n, h=1.0 / n)
    rng = np.random.default_rng(n + dim)
    nf = dim
    b = rng.standard_normal((nf,) + (n,) * dim)
    if c0 == 0.0:
        b -= b.reshape(nf, -1).mean(axis=1).reshape((nf,) + (1,) * dim)
    x = s.vcycle(c0, c1, b)
    xe = np.stack([multigrid.vcycle(b[f], c0, c1) for f in range(nf)])
    assert _rel(x, xe) < 1e-11, _rel(x, xe)
    s.close()


@pytest.mark.parametrize("dim,n", [(3, 16), (3, 32), (3, 64), (2, 64), (2, 128), (2, 256)])
@pytest.mark.parametrize("c0,c1", [(0.0, 1.0), (2.5, 0.7)])
def test_vcycle_mixed_precision(dim, n, c0, c1):
    """fp32 V-cycles: multi-kernel levels above the one-workgroup tail (32^3 /
    128^2 in fp32), the tail alone, and the tail with its second level's
    right-hand side outside LDS (3D from 32^3 down)."""
    from paper_1505_07865_amd import ibr
    s = ibr.Solver(dim=dim, n=n, h=1.0 / n, precision=ibr.MIXED)
    rng = np.random.default_rng(3)
    nf = dim
    b = rng.standard_normal((nf,) + (n,) * dim)
    if c0 == 0.0:
        b -= b.reshape(nf, -1).mean(axis=1).reshape((nf,) + (1,) * dim)
    x = s.vcycle(c0, c1, b)
    for f in range(nf):
        xe = multigrid.vcycle(b[f], c0, c1)
        assert _rel(x[f], xe) < 1e-5, (f, _rel(x[f], xe))
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,nf", [(64, 3), (64, 1), (128, 1), (128, 3)])
@pytest.mark.parametrize("c0,c1", [(0.0, 1.0), (2.5, 0.7)])
def test_vcycle_large_levels_match_oracle(precision, n, nf, c0, c1):
    """The V-cycle shapes of the 128^3 workload and its 64^3 level: the
    velocity cycle (3 fields: per-step kernels on 128^3 and 64^3, fused LDS
    tiles from 32^3) and the pressure cycle (1 field: the 64^3 level fused
    too) equal the oracle's cycle (fp64 1e-11, fp32 1e-5) and repeat bitwise
    (the fused post-smoothing writes a second array; an in-place version
    raced)."""
    from paper_1505_07865_amd import ibr
    print("V-cycle %s %d^3 nf %d c0 %g" % (precision, n, nf, c0), flush=True)
    s = ibr.Solver(dim=3, n=n, h=1.0 / n, precision=ibr.MIXED if precision == "mixed" else ibr.FP64)
    rng = np.random.default_rng(7 * n + nf)
    b = rng.standard_normal((nf,) + (n,) * 3)
    if c0 == 0.0:
        b -= b.reshape(nf, -1).mean(axis=1).reshape((nf, 1, 1, 1))
    x = s.vcycle(c0, c1, b if nf > 1 else b[0])
    x = x.reshape((nf,) + (n,) * 3)
    bar = 1e-11 if precision == "fp64" else 1e-5
    for f in range(nf):
        xe = multigrid.vcycle(b[f], c0, c1)
        assert _rel(x[f], xe) < bar, (f, _rel(x[f], xe))
    x2 = s.vcycle(c0, c1, b if nf > 1 else b[0]).reshape(x.shape)
    assert np.array_equal(x, x2)
    s.close()


def test_mobility_blocks_match_oracle(case):
    prob, name = case
    s = _solver(prob)
    blocks, p = mobility.blocks_for_problem(prob)
    f0 = mobility.self_term(p)
    for b, Me in enumerate(blocks):
        M, sh = s.mobility_block(b)
        assert _rel(M, Me) < 1e-13
        _, she = mobility.factor_block(Me, f0)
        assert sh == she
    s.close()


@pytest.mark.parametrize("full", [False, True])
def test_preconditioner_matches_oracle(case, full):
    from paper_1505_07865_amd import ibr
    prob, name = case
    s = _solver(prob, pc=ibr.PC_FULL if full else ibr.PC_LOWER, n_s=2)
    sysm = constrained.System.from_problem(prob)
    P = precond.for_problem(prob, sysm, ns=2, full=full)
    rng = np.random.default_rng(8)
    d, n, N = prob.dim, prob.n, prob.nmarkers
    r = dense.apply_operator(sysm, rng.standard_normal(s.NV))   # in the range of K
    z = s.precondition(r)
    nv, npr = d * n ** d, n ** d
    zv, zp, zl = P.apply(r[:nv].reshape((d,) + (n,) * d), r[nv:nv + npr].reshape((n,) * d),
                         r[nv + npr:].reshape(N, d))
    gv = z[:nv].reshape(zv.shape)
    gp = z[nv:nv + npr].reshape(zp.shape)
    gl = z[nv + npr:].reshape(zl.shape)
    assert _rel(gv, zv) < 1e-9
    assert _rel(gp - gp.mean(), zp - zp.mean()) < 1e-9
    assert _rel(gl, zl) < 1e-9
    s.close()


@pytest.mark.parametrize("ns", [1, 2, 3, 4])
@pytest.mark.parametrize("name", ["3d32_steady", "2d32_unsteady"])
def test_preconditioner_inner_ns(name, ns):
    """Inner GMRES(N_s): normal equations over the power basis for N_s <= 3,
    Arnoldi for larger N_s; both must give the oracle's GMRES(N_s) iterate."""
    from paper_1505_07865_amd import ibr
    prob = small_problem(21, **CASES[name])
    s = _solver(prob, pc=ibr.PC_LOWER, n_s=ns)
    sysm = constrained.System.from_problem(prob)
    P = precond.for_problem(prob, sysm, ns=ns, full=False)
    rng = np.random.default_rng(10 + ns)
    d, n, N = prob.dim, prob.n, prob.nmarkers
    r = dense.apply_operator(sysm, rng.standard_normal(s.NV))
    z = s.precondition(r)
    nv, npr = d * n ** d, n ** d
    zv, zp, zl = P.apply(r[:nv].reshape((d,) + (n,) * d), r[nv:nv + npr].reshape((n,) * d),
                         r[nv + npr:].reshape(N, d))
    assert _rel(z[:nv].reshape(zv.shape), zv) < 1e-9
    assert _rel(z[nv + npr:].reshape(zl.shape), zl) < 1e-9
    # a zero residual maps to exactly zero (rank-deficient normal equations)
    assert not np.any(s.precondition(np.zeros(s.NV)))
    s.close()


def test_preconditioner_mixed_close(case):
    from paper_1505_07865_amd import ibr
    prob, name = case
    s = _solver(prob, precision=ibr.MIXED)
    sysm = constrained.System.from_problem(prob)
    P = precond.for_problem(prob, sysm, ns=2)
    rng = np.random.default_rng(9)
    d, n, N = prob.dim, prob.n, prob.nmarkers
    r = dense.apply_operator(sysm, rng.standard_normal(s.NV))
    z = s.precondition(r)
    nv, npr = d * n ** d, n ** d
    zv, zp, zl = P.apply(r[:nv].reshape((d,) + (n,) * d), r[nv:nv + npr].reshape((n,) * d),
                         r[nv + npr:].reshape(N, d))
    assert _rel(z[:nv].reshape(zv.shape), zv) < 1e-4
    assert _rel(z[nv + npr:].reshape(zl.shape), zl) < 1e-3
    s.close()


def test_advection_matches_oracle():
    from paper_1505_07865_amd import ibr
    for dim, n in ((3, 16), (2, 32)):
        s = ibr.Solver(dim=dim, n=n, h=1.0 / n, rho=1.0, dt=0.01)
        u = np.random.default_rng(dim).standard_normal((dim,) + (n,) * dim)
        N = s.advect(u)
        Ne = navier.advection(u, 1.0 / n)
        assert _rel(N, Ne) < 1e-13
        s.close()


def test_grid_stokes_operator_consistency():
    """The fluid block of K is the oracle's [[A, G], [-D, 0]] (Sec. 3.2)."""
    prob = small_problem(4, 3, 16, radius_h=2.5)
    s = _solver(prob)
    rng = np.random.default_rng(2)
    d, n = 3, 16
    x = np.zeros(s.NV)
    x[:(d + 1) * n ** d] = rng.standard_normal((d + 1) * n ** d)
    y = s.apply_operator(x)
    v = x[:d * n ** d].reshape((d,) + (n,) * d)
    p = x[d * n ** d:(d + 1) * n ** d].reshape((n,) * d)
    rm, rc = grid.stokes_apply(v, p, 0.0, 1.0, prob.h)
    assert _rel(y[:d * n ** d].reshape(rm.shape), rm) < 1e-12
    assert _rel(y[d * n ** d:(d + 1) * n ** d].reshape(rc.shape), rc) < 1e-12
    s.close()


@pytest.mark.parametrize("which", ["case", "sphere600"])
def test_mobility_inverse_matches_oracle(which):
    """Dense per-body solve (Sec. 5.3): the MFMA Cholesky + inverse equals LAPACK's."""
    from synthetic import config1_sphere3d
    if which == "case":
        prob = small_problem(21, **CASES["3d32_steady"])
    else:
        prob = config1_sphere3d(0)          # one 600 x 600 block (38 MFMA panels)
    s = _solver(prob)
    blocks, p = mobility.blocks_for_problem(prob)
    f0 = mobility.self_term(p)
    for b, Me in enumerate(blocks):
        Lc, sh = mobility.factor_block(Me, f0)
        ref = np.linalg.inv(Me + sh * f0 * np.eye(len(Me)))
        Mi = s.mobility_inverse(b)
        assert _rel(Mi, ref) < 1e-10, _rel(Mi, ref)
    s.close()


@pytest.mark.parametrize("pre,post", [(1, 1), (2, 3), (2, 0), (0, 2)])
@pytest.mark.parametrize("dim,n,nf", [(3, 64, 3), (2, 128, 2)])
def test_vcycle_sweep_counts_match_oracle(pre, post, dim, n, nf):
    """Other smoothing sweep counts take other kernel sequences: one post
    sweep is the red sweep with the prolongation folded in plus one black
    sweep; three sweeps leave the fused LDS levels for the per-step kernels;
    no post-smoothing uses the plain prolongation, no pre-smoothing starts
    from zero.  Each equals the oracle's cycle with the same counts (fp64,
    1e-11) and repeats bitwise."""
    from paper_1505_07865_amd import ibr
    print("V-cycle sweeps %d/%d dim %d n %d nf %d" % (pre, post, dim, n, nf), flush=True)
    s = ibr.Solver(dim=dim, n=n, h=1.0 / n, precision=ibr.FP64, mg_pre=pre, mg_post=post)
    rng = np.random.default_rng(100 * pre + 10 * post + dim)
    b = rng.standard_normal((nf,) + (n,) * dim)
    c0, c1 = 2.5, 0.7
    x = s.vcycle(c0, c1, b).reshape(b.shape)
    for f in range(nf):
        xe = multigrid.vcycle(b[f], c0, c1, nu_pre=pre, nu_post=post)
        assert _rel(x[f], xe) < 1e-11, (f, _rel(x[f], xe))
    assert np.array_equal(x, s.vcycle(c0, c1, b).reshape(b.shape))
    s.close()
