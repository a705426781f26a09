"""Host logic of the request server (queue, resident contexts, admission),
with stand-in solvers: no GPU needed."""
import threading
import time
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1505_07865_amd import serve


class FakeSolver:
    created = []

    def __init__(self, prob, delay=0.0):
        self.key = (prob.dim, prob.n)
        self.delay = delay
        self.closed = False
        self.prob = None
        FakeSolver.created.append(self)

    def set_bodies(self, R, offsets, centres):
        self.prob_R = R

    def set_velocities(self, U, Om):
        self.U = U

    def solve(self, warm_start=False):
        assert not warm_start
        time.sleep(self.delay)
        return {"iters": 1, "rel_residual": 0.0}

    def forces(self):
        return self.U * 2.0 + getattr(self, "t", 0), np.zeros((len(self.U), 1))

    def reset(self):
        self.t = 0

    def step(self):
        self.t += 1
        time.sleep(self.delay)
        return {"iters": 1, "rel_residual": 0.0}

    def close(self):
        self.closed = True


def _prob(dim, n, nb=1, u=1.0, rho=0.0, dt=0.0):
    return SimpleNamespace(dim=dim, n=n, h=1.0 / n, rho=rho, eta=1.0, dt=dt, nbodies=nb, nmarkers=4 * nb,
                           R=np.zeros((4 * nb, dim)), offsets=np.arange(0, 4 * nb + 1, 4),
                           centres=np.zeros((nb, dim)), U=np.full((nb, dim), u),
                           Omega=np.zeros((nb, 1)))


def test_fifo_results_and_resident_contexts():
    FakeSolver.created = []
    probs = [_prob(2, 32, u=i) for i in range(10)] + [_prob(3, 16, u=100 + i) for i in range(10)]
    with serve.Server(workers=2, factory=lambda p: FakeSolver(p), footprint=lambda p: 1,
                      free_bytes=lambda: 1 << 40, reserve_bytes=0) as srv:
        futs = [srv.submit(p) for p in probs]
        res = [f.result(timeout=10) for f in futs]
    for p, r in zip(probs, res):
        assert np.array_equal(r["F"], p.U * 2.0)
    assert [r["id"] for r in res] == list(range(20))
    # at most one context per (worker, grid size), all closed at shutdown
    assert len(FakeSolver.created) <= 4
    assert all(s.closed for s in FakeSolver.created)


def test_admission_evicts_lru_then_refuses():
    FakeSolver.created = []
    free = {"b": 100}
    sizes = {(2, 32): 30, (2, 64): 60, (3, 64): 500}

    def factory(p):
        s = FakeSolver(p)
        free["b"] -= sizes[(p.dim, p.n)]
        orig = s.close

        def close():
            free["b"] += sizes[(p.dim, p.n)]
            orig()
        s.close = close
        return s

    with serve.Server(workers=1, factory=factory, footprint=lambda p: sizes[(p.dim, p.n)],
                      free_bytes=lambda: free["b"], reserve_bytes=0) as srv:
        a = srv.submit(_prob(2, 32)).result(timeout=10)
        b = srv.submit(_prob(2, 64)).result(timeout=10)   # 30 + 60 fit in 100
        assert free["b"] == 10
        c = srv.submit(_prob(2, 32)).result(timeout=10)   # resident, no new context
        assert len(FakeSolver.created) == 2
        f = srv.submit(_prob(3, 64))                      # 500 never fits: evicts both, then refuses
        with pytest.raises(MemoryError):
            f.result(timeout=10)
        assert free["b"] == 100
        d = srv.submit(_prob(2, 64)).result(timeout=10)   # still serves afterwards
    assert a and b and c and d


def test_replay_latency_and_throughput():
    trace = [{"t": 0.01 * i, "problem": _prob(2, 32)} for i in range(20)]
    with serve.Server(workers=2, factory=lambda p: FakeSolver(p, delay=0.002), footprint=lambda p: 1,
                      free_bytes=lambda: 1 << 40, reserve_bytes=0) as srv:
        out = serve.replay(trace, srv, qps=2.0)     # arrivals every 5 ms
        assert out["requests"] == 20
        assert out["makespan_s"] >= 0.095 * 0.99
        assert 0 < out["p50_ms"] <= out["p99_ms"] < 1000
        sat = serve.replay(trace, srv, qps=None)
        assert sat["solves_per_s"] > 0


def test_trajectories_restart_from_rest_on_shared_contexts():
    FakeSolver.created = []
    probs = [_prob(3, 16, u=i, rho=1.0, dt=0.5 / 16) for i in range(6)]
    with serve.Server(workers=2, factory=lambda p: FakeSolver(p, delay=0.001), footprint=lambda p: 1,
                      free_bytes=lambda: 1 << 40, reserve_bytes=0) as srv:
        futs = [srv.submit_trajectory(p, 3 + i % 2) for i, p in enumerate(probs)]
        steady = srv.submit(_prob(3, 16, u=7)).result(timeout=10)
        res = [f.result(timeout=10) for f in futs]
        with pytest.raises(ValueError):
            srv.submit_trajectory(probs[0], 0)
    for i, (p, r) in enumerate(zip(probs, res)):
        # every trajectory starts from rest, whatever its context ran before
        assert len(r["steps"]) == 3 + i % 2
        assert np.array_equal(r["F"], p.U * 2.0 + 3 + i % 2)
        assert all(st["wall_ms"] >= 0 for st in r["steps"])
    assert np.array_equal(steady["F"], np.full((1, 3), 14.0))
    # unsteady and steady problems of one grid use different contexts: at most 2 per worker
    assert len(FakeSolver.created) <= 4


def test_walls_get_their_own_contexts():
    """A slit-channel request never lands on a periodic context of the same
    grid (and the other way round), and the solver is built with its walls."""
    FakeSolver.created = []
    made = []

    def factory(p):
        made.append(getattr(p, "walls", 0))
        return FakeSolver(p)

    per = _prob(3, 16)
    slit = _prob(3, 16)
    slit.walls = 1
    with serve.Server(workers=1, factory=factory, footprint=lambda p: 1,
                      free_bytes=lambda: 1 << 40, reserve_bytes=0) as srv:
        for p in (per, slit, per, slit):
            srv.submit(p).result(timeout=10)
    assert sorted(made) == [0, 1]
    assert serve._context_key(per) != serve._context_key(slit)
    srv2 = serve.Server(workers=1, factory=factory, footprint=lambda p: 1, free_bytes=lambda: 1 << 40,
                        reserve_bytes=0)
    try:
        assert srv2._params(slit)["walls"] == 1 and srv2._params(per)["walls"] == 0
        assert srv2._params(slit)["n_s"] == 4 and "n_s" not in srv2._params(per)
    finally:
        srv2.close()


def test_concurrent_admission_waits_for_memory():
    """Four workers take requests for four grid sizes at once; each context
    needs 40 of 100 bytes.  Admission is serialised: at no time do more than
    two contexts exist, requests that do not fit yet wait for a context to be
    released (then evict it) instead of failing, and every request is served."""
    FakeSolver.created = []
    lock = threading.Lock()
    state = {"free": 100, "alive": 0, "max_alive": 0}

    def factory(p):
        s = FakeSolver(p, delay=0.02)
        with lock:
            state["free"] -= 40
            state["alive"] += 1
            state["max_alive"] = max(state["max_alive"], state["alive"])
        assert state["free"] >= 0
        orig = s.close

        def close():
            with lock:
                state["free"] += 40
                state["alive"] -= 1
            orig()
        s.close = close
        return s

    probs = [_prob(2, n, u=i) for i, n in enumerate((16, 32, 64, 128) * 4)]
    with serve.Server(workers=4, factory=factory, footprint=lambda p: 40, free_bytes=lambda: state["free"],
                      reserve_bytes=0) as srv:
        futs = [srv.submit(p) for p in probs]
        res = [f.result(timeout=20) for f in futs]
        assert srv.admission_waits > 0 and srv.evictions > 0
    for p, r in zip(probs, res):
        assert np.array_equal(r["F"], p.U * 2.0)
    assert state["max_alive"] <= 2
    assert state["free"] == 100 and state["alive"] == 0


def test_admission_evicts_other_workers_idle_contexts():
    """An idle context held by one worker is evicted for another worker's
    request when memory is short (least recently used first, any worker)."""
    FakeSolver.created = []
    state = {"free": 100}
    gate = threading.Event()

    class Slow(FakeSolver):
        def solve(self, warm_start=False):
            if self.key == (2, 64):
                gate.wait(5)
            return super().solve(warm_start)

    def factory(p):
        s = Slow(p)
        state["free"] -= 60
        orig = s.close

        def close():
            state["free"] += 60
            orig()
        s.close = close
        return s

    with serve.Server(workers=2, factory=factory, footprint=lambda p: 60, free_bytes=lambda: state["free"],
                      reserve_bytes=0) as srv:
        srv.submit(_prob(2, 32)).result(timeout=10)        # one worker now holds an idle 32^2 context
        f = srv.submit(_prob(2, 64))                        # needs the 32^2 context's memory
        gate.set()
        f.result(timeout=10)
        assert srv.evictions == 1
        assert sum(len(w.contexts) for w in srv.workers) == 1


def test_admission_counts_body_blocks_not_yet_allocated():
    """A context takes 30 of its 100-byte footprint when created and the other
    70 when its first request sets the bodies, outside the admission lock.  Two
    workers take requests for two grids at once with 150 bytes free: the
    second admission must count the first context's 70 pending bytes and wait,
    so the free memory never goes negative."""
    FakeSolver.created = []
    lock = threading.Lock()
    state = {"free": 150, "min_free": 150}

    def take(nbytes):
        with lock:
            state["free"] -= nbytes
            state["min_free"] = min(state["min_free"], state["free"])

    class Bodies(FakeSolver):
        def __init__(self, p):
            super().__init__(p, delay=0.01)
            self.held = 30
            take(30)

        def set_bodies(self, R, offsets, centres):
            time.sleep(0.05)      # the other worker's admission runs meanwhile
            if self.held == 30:
                take(70)
                self.held = 100
            super().set_bodies(R, offsets, centres)

        def close(self):
            take(-self.held)
            super().close()

    probs = [_prob(2, n, u=i) for i, n in enumerate((16, 32) * 3)]
    with serve.Server(workers=2, factory=Bodies, footprint=lambda p: 100, free_bytes=lambda: state["free"],
                      reserve_bytes=0) as srv:
        futs = [srv.submit(p) for p in probs]
        res = [f.result(timeout=20) for f in futs]
        assert srv.admission_waits > 0
        assert not srv._pending
    for p, r in zip(probs, res):
        assert np.array_equal(r["F"], p.U * 2.0)
    assert state["min_free"] >= 0
    assert state["free"] == 150
