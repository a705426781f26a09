"""Request server for independent constrained solves on one GPU.

A request is one rigid-body problem (grid, fluid parameters, bodies,
prescribed velocities) and asks either for one steady solve (``submit``) or
for an unsteady trajectory of several time steps from rest
(``submit_trajectory``); the answer is the drag force and torque on every body
and the solve reports.  Requests are independent, so the server scales by data
parallelism over requests: several host worker threads each own resident
solver contexts (one per grid size and fluid parameters, every context with
its own HIP stream) and take requests from one FIFO queue as they arrive.
While one request's solve waits on its stream, the others' kernels run: work
of different requests overlaps on the device, small grids with large ones,
and no request pays for allocating or tearing down a context.

Admission: contexts are created under one server-wide lock.  A new context
is admitted when its device footprint (``ibr_footprint_bytes``) fits in the
free device memory minus a reserve and minus what admitted contexts have yet
to allocate; otherwise the least recently used idle context of any worker is
closed first, and when every remaining context is in use the request waits
until a worker releases one.  Only a request that does not fit with no
context left on the device fails, with MemoryError.  A context's body blocks
are allocated when its first request sets the bodies, outside the lock: until
then the part of its footprint that creation did not take from the free
memory stays counted as pending, so that concurrent admissions cannot spend
it twice.  A resident context that takes a request with larger body blocks
than it holds grows by the difference without a new admission: a request's
body blocks (under about 100 MB for the requests served) are small next to
a context's grids and hierarchies.

Every steady solve starts from a zero initial guess and every trajectory from
a fluid at rest, so a request's result does not depend on what the context
solved before: served alone or in a mix, it is bitwise the same.
"""
import collections
import queue
import threading
import time

import numpy as np

__all__ = ["Server", "replay"]


class _Worker(threading.Thread):
    def __init__(self, server, wid):
        super().__init__(name="ibr-serve-%d" % wid, daemon=True)
        self.server = server
        self.wid = wid

    @property
    def contexts(self):
        """This worker's resident contexts, key -> solver (a snapshot)."""
        srv = self.server
        with srv._adm:
            return {k: s for (w, k), s in srv._lru.items() if w == self.wid}

    def _context(self, prob):
        """The worker's context for prob's grid and fluid, marked in use;
        admitted by footprint (see the module notes).  Release with _release."""
        srv = self.server
        ck = (self.wid, _context_key(prob))
        with srv._adm:
            if ck in srv._lru:
                srv._lru.move_to_end(ck)
                srv._busy.add(ck)
                return srv._lru[ck]
            need = srv.footprint(prob)
            while srv.free_bytes() - srv.reserve_bytes - sum(srv._pending.values()) < need:
                victim = next((k for k in srv._lru if k not in srv._busy), None)
                if victim is not None:
                    srv._lru.pop(victim).close()
                    srv.evictions += 1
                    continue
                if not srv._busy:
                    raise MemoryError("request of %d bytes does not fit on the device" % need)
                srv.admission_waits += 1
                srv._adm.wait()
            before = srv.free_bytes()
            s = srv.factory(prob)
            left = need - max(0, before - srv.free_bytes())
            if left > 0:
                srv._pending[ck] = left
            srv._lru[ck] = s
            srv._busy.add(ck)
            return s

    def _settled(self, prob):
        """The context's bodies are set: what it allocates now shows in the
        free memory, so none of its footprint is pending any more."""
        srv = self.server
        with srv._adm:
            if srv._pending.pop((self.wid, _context_key(prob)), None) is not None:
                srv._adm.notify_all()

    def _release(self, prob):
        srv = self.server
        with srv._adm:
            ck = (self.wid, _context_key(prob))
            srv._pending.pop(ck, None)
            srv._busy.discard(ck)
            srv._adm.notify_all()

    def run(self):
        srv = self.server
        while True:
            item = srv.queue.get()
            if item is None:
                break
            rid, prob, nsteps, fut = item
            held = False
            try:
                s = self._context(prob)
                held = True
                s.set_bodies(prob.R, prob.offsets, prob.centres)
                self._settled(prob)
                s.set_velocities(prob.U, prob.Omega)
                if nsteps is None:
                    info = s.solve(warm_start=False)
                    F, T = s.forces()
                    fut._finish(result={"id": rid, "info": info, "F": F, "T": T, "worker": self.wid})
                else:
                    s.reset()
                    steps = []
                    for _ in range(nsteps):
                        t0 = time.perf_counter()
                        info = s.step()
                        info["wall_ms"] = (time.perf_counter() - t0) * 1e3
                        steps.append(info)
                    F, T = s.forces()
                    fut._finish(result={"id": rid, "steps": steps, "F": F, "T": T, "worker": self.wid})
            except BaseException as e:   # reported through the future
                fut._finish(error=e)
            finally:
                if held:
                    self._release(prob)
        with srv._adm:
            for ck in [k for k in srv._lru if k[0] == self.wid]:
                srv._lru.pop(ck).close()
            srv._adm.notify_all()


def _context_key(prob):
    # contexts are shared by requests with the same grid, boundaries and fluid parameters
    return (prob.dim, prob.n, prob.h, getattr(prob, "walls", 0), prob.rho, prob.eta,
            prob.dt if prob.rho > 0 else 0.0)


class Future:
    def __init__(self, t_arrive):
        self.t_arrive = t_arrive
        self.t_done = None
        self._ev = threading.Event()
        self._result = None
        self._error = None

    def _finish(self, result=None, error=None):
        self.t_done = time.perf_counter()
        self._result = result
        self._error = error
        self._ev.set()

    def result(self, timeout=None):
        if not self._ev.wait(timeout):
            raise TimeoutError("request not finished")
        if self._error is not None:
            raise self._error
        return self._result

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive


class Server:
    """FIFO request server over ``workers`` threads with resident contexts.

    factory(problem) -> solver object with set_bodies, set_velocities,
    solve(warm_start), forces() and close(); the default builds
    ``ibr.Solver`` contexts for steady Stokes with the given precision.
    A trajectory request additionally needs reset() and step().
    footprint(problem) and free_bytes() default to the library's footprint
    query and the device's free memory.
    """

    def __init__(self, precision="mixed", workers=4, rtol=1e-8, device=0, reserve_bytes=8 << 30,
                 factory=None, footprint=None, free_bytes=None, graphs=0, **solver_kw):
        self.precision = precision
        self.rtol = rtol
        self.device = device
        self.reserve_bytes = reserve_bytes
        self.graphs = graphs
        self.solver_kw = solver_kw
        self.factory = factory or self._default_factory
        self.footprint = footprint or self._default_footprint
        self.free_bytes = free_bytes or self._default_free_bytes
        self.queue = queue.Queue()
        self.next_id = 0
        # admission state, shared by all workers under _adm: resident contexts
        # in least-recently-used order, (worker, key) -> solver, and those in use
        self._adm = threading.Condition()
        self._lru = collections.OrderedDict()
        self._busy = set()
        # (worker, key) -> bytes of an admitted context's footprint that the
        # device's free memory does not show yet (its bodies are not set)
        self._pending = {}
        self.evictions = 0
        self.admission_waits = 0
        self.workers = [_Worker(self, w) for w in range(workers)]
        for w in self.workers:
            w.start()

    # ---------------------------------------------------------------- defaults
    def _params(self, prob):
        from . import ibr
        walls = getattr(prob, "walls", 0)
        kw = dict(n_s=4) if walls else {}     # between walls P_S^-1 is a weaker Stokes preconditioner
        kw.update(self.solver_kw)
        return dict(dim=prob.dim, n=prob.n, h=prob.h, rho=prob.rho, eta=prob.eta, dt=prob.dt,
                    walls=walls, rtol=self.rtol,
                    precision=ibr.MIXED if self.precision == "mixed" else ibr.FP64, device=self.device,
                    graphs=self.graphs, **kw)

    def _default_factory(self, prob):
        from . import ibr
        return ibr.Solver(**self._params(prob))

    def _default_footprint(self, prob):
        from . import ibr
        return ibr.footprint_bytes(np.diff(prob.offsets), **self._params(prob))

    def _default_free_bytes(self):
        import torch
        free, _ = torch.cuda.mem_get_info(self.device)
        return free

    # ---------------------------------------------------------------- requests
    def submit(self, prob, t_arrive=None):
        """One steady solve of prob from a zero initial guess (prob.rho == 0)."""
        return self._put(prob, None, t_arrive)

    def submit_trajectory(self, prob, nsteps, t_arrive=None):
        """nsteps unsteady time steps of prob (prob.rho > 0) from a fluid at
        rest; the result holds every step's solve report and the final forces."""
        if nsteps < 1:
            raise ValueError("a trajectory needs at least one step")
        return self._put(prob, int(nsteps), t_arrive)

    def _put(self, prob, nsteps, t_arrive):
        fut = Future(time.perf_counter() if t_arrive is None else t_arrive)
        self.queue.put((self.next_id, prob, nsteps, fut))
        self.next_id += 1
        return fut

    def close(self):
        for _ in self.workers:
            self.queue.put(None)
        for w in self.workers:
            w.join()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def prewarm(self, problems):
        """Give every worker a resident context for each grid size among these
        problems (created here, with one solve each, before any measured
        request) so that no measured request pays for a context."""
        seen = {}
        for p in problems:
            seen.setdefault(_context_key(p), p)
        for w in self.workers:
            for key, p in seen.items():
                if key not in w.contexts:
                    s = w._context(p)
                    try:
                        s.set_bodies(p.R, p.offsets, p.centres)
                        w._settled(p)
                        s.set_velocities(p.U, p.Omega)
                        if p.rho > 0:
                            s.reset()
                            s.step()
                        else:
                            s.solve(warm_start=False)
                    finally:
                        w._release(p)


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def replay(trace, server, qps=None):
    """Offer the trace's requests at their arrival times scaled to ``qps``
    (None = all at once, saturation) and wait for all of them.

    trace: list of {"t": arrival time at rate 1, "problem": Problem}.
    Returns throughput (requests / makespan), p50/p99 latency (arrival to
    completion, queueing included) and per-request results in trace order.
    """
    t0 = time.perf_counter()
    futs = []
    for req in trace:
        if qps is not None:
            t_arr = t0 + req["t"] / qps
            dt = t_arr - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        else:
            t_arr = t0
        futs.append(server.submit(req["problem"], t_arrive=t_arr))
    results = [f.result() for f in futs]
    t_end = max(f.t_done for f in futs)
    lat = [f.latency * 1e3 for f in futs]
    return {"requests": len(trace), "makespan_s": t_end - t0, "solves_per_s": len(trace) / (t_end - t0),
            "p50_ms": _percentile(lat, 50), "p99_ms": _percentile(lat, 99), "qps_offered": qps,
            "results": results}
