"""Benchmark: constrained-solve throughput on the 3D 128^3 unsteady workload.

Workload (one MI355X): periodic unit cube, 128^3 MAC grid, rho = 1, Re = 10
(eta = R/Re, R = 6h), dt = 0.5h; 16 non-overlapping spheres of radius 6h with
110 Fibonacci markers each (1760 markers, 16 per-body 330x330 mobility blocks),
each body translating with a seeded velocity U ~ U[-1,1]^3.  A step is one
time step of the method: explicit advection right-hand side, markers moved and
re-binned, warm-started FGMRES solve of the constrained system to relative
residual 1e-8 with the Schur-complement preconditioner (N_s = 2, one V-cycle per
field).  Inputs are resident in HBM when the timed region starts.

The headline value is the mixed-precision solver's solves/s (fp32
preconditioner, fp64 outer FGMRES/Arnoldi/Hessenberg/mobility blocks); the
plain fp64 solver runs the same trajectory for comparison.  The ``served``
object gives the served form: 8 independent simulations of the workload (one
per seed, 20 steps each from rest) offered at once to the request server,
with 4 workers whose solves overlap on the device, and with 1 worker (the
plain solver), in both precisions.  The ``second_re`` object runs the same
workload at Re = 100, where the advection is the semi-Lagrangian transport
(the centred form with AB2 is unstable at that cell Reynolds number).  The
``serving_mix`` object runs the first requests of the serving trace (steady
solves of mixed grid sizes and body counts) through the request server, at
saturation and as Poisson arrivals at 0.7x the fp64 capacity, in both
precisions.

    python bench.py [--steps K] [--warmup W] [--re 10] [--advection auto|centred|sl] [--seed 0]
                    [--no-cpu-baseline]
    python bench.py --serving | --ablation | --free | --blocks | --walls | --large | --small
                                                                 (other workloads, one JSON line each)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of a timed kernel class, from two rocprofv3 --pmc runs:
# the L2's read requests to memory by size (TCC_EA0_RDREQ_32B/_64B/_128B x
# 32/64/128 bytes), then its write requests (TCC_EA0_WRREQ_64B x 64 + the rest
# x 32), averaged over the launches of one step.  On a plain 1 GiB device copy
# both read 1.0000 of the bytes moved.  (FETCH_SIZE takes TCC_BUBBLE as its
# 128-byte count, which reads half of the 128-byte requests here, so no single
# scale factor fits kernels with different request sizes.)  A figure holds
# only for the kernel source it was taken on: the digest of that file is
# checked and the figure dropped (null) once the source differs.
MEASURED_TRAFFIC = {
    "rb_fine": {"bytes_per_launch": 27629000.0, "file": "paper_1505_07865_amd/csrc/ops_mg.hip",
                "sha256_16": "6464b3451ec49239", "summary": "profiles/rb_fine_128cube_mixed_hbm_counters.md"},
}
# strides coprime with the launch pattern (12 finest-level sweeps per P_S^-1, 2 V-cycle calls
# per P_S^-1) so the samples cycle through it; sparse enough that the sampled launches' events
# cost about 1% of the step
TIMER_STRIDE = {"rb_fine": 29, "ortho_dot": 7, "ortho_axpy": 7, "stokes_apply": 7, "vcycle": 9, "wall_rb_fine": 29,
                "rb_red_prolong": 7}
# composite classes (several kernels per sample): reported, never the roofline kernel
COMPOSITE_TIMERS = ("vcycle",)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=54,
                    help="timed steps in all, spread over the trajectories of --seeds")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--re", type=float, default=10.0)
    ap.add_argument("--advection", choices=("auto", "centred", "sl"), default="auto",
                    help="centred advective form with AB2, or semi-Lagrangian transport; auto takes the "
                         "centred form while the cell Reynolds number Re h/R is at most 8 (where it is stable)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--seeds", default="0,1,2",
                    help="default line: the workload's trajectories (comma-separated seeds) timed as one job, "
                         "extended by the next seeds when --steps needs more; the first is the one compared "
                         "with the oracle")
    ap.add_argument("--n-s", type=int, default=2, help="inner GMRES(N_s) iterations of the preconditioner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--serving", action="store_true",
                    help="serving workload instead: Poisson arrivals of mixed-size steady solves")
    ap.add_argument("--ablation-parts", default="periodic,slit,box",
                    help="ablation: comma-separated subset of periodic, slit, box")
    ap.add_argument("--analytic-mobility", action="store_true",
                    help="ablation: the analytic approximate mobility instead of the default (fitted in 3D)")
    ap.add_argument("--mobility-study", action="store_true",
                    help="fitted vs analytic approximate mobility: P_S^-1 applications (not the headline)")
    ap.add_argument("--ablation", action="store_true",
                    help="solver study instead: preconditioner variant and N_s vs P_S^-1 applications")
    ap.add_argument("--nreq", type=int, default=2000, help="serving: requests in the trace")
    ap.add_argument("--mix-requests", type=int, default=300,
                    help="default line: requests of the serving trace run as its serving_mix leg (0 = skip)")
    ap.add_argument("--workers", type=int, default=4, help="serving and served form: host worker threads")
    ap.add_argument("--served-trajectories", type=int, default=8,
                    help="served form: independent simulations of the workload offered at once")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form leg")
    ap.add_argument("--second-re", type=float, default=100.0,
                    help="the workload's other Reynolds number, run after the headline one in both precisions "
                         "(0 = skip)")
    ap.add_argument("--free", action="store_true",
                    help="free-kinematics workload instead: a sedimenting suspension of 16 free spheres at 128^3")
    ap.add_argument("--free-solves", type=int, default=5, help="free kinematics: timed solves per precision")
    ap.add_argument("--walls", action="store_true",
                    help="slit channel (no-slip walls along z) at 128^3 against the same bodies in the periodic box")
    ap.add_argument("--slit-solves", type=int, default=5, help="slit channel: timed solves per precision and box")
    ap.add_argument("--large", action="store_true",
                    help="the 256^3 configuration (100 spheres, steady), mixed and fp64 solves")
    ap.add_argument("--large-solves", type=int, default=2, help="large: timed solves per precision")
    ap.add_argument("--small", action="store_true",
                    help="the 2D 64^2 disk and 3D 64^3 sphere configurations, per seed, beside the oracle")
    ap.add_argument("--small-seeds", type=int, default=5, help="small: seeds 0 .. K-1 per configuration")
    ap.add_argument("--small-solves", type=int, default=20, help="small: timed solves per seed and precision")
    ap.add_argument("--blocks", action="store_true",
                    help="per-body mobility set-up of the 256^3 configuration (100 blocks of 600 x 600, fp64 MFMA)")
    ap.add_argument("--block-reps", type=int, default=5, help="blocks: timed set-ups")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (scale for the HBM byte counters)")
    return ap.parse_args()


def calibrate_copy(torch, reps=5):
    """A plain device copy of known size: reads 1 GiB and writes 1 GiB per launch.
    The HBM byte counters read on it give the factor that converts the counter
    units into bytes."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                      "launches": reps}), flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def advection_scheme(args):
    """The advection form for the workload's Reynolds number: the centred
    form with AB2 needs viscous damping per step and grows without bound at
    cell Reynolds number Re h/R = Re/6 of about 17 (Re = 100)."""
    if args.advection != "auto":
        return args.advection
    return "centred" if args.re / 6.0 <= 8.0 else "sl"


def run_precision(prob, prec, steps, warmup, torch, scheme="centred", n_s=2):
    from paper_1505_07865_amd import ibr
    # kernels go straight onto the stream (iteration graphs measured no faster,
    # and the live event timers bracket individual launches)
    s = ibr.from_problem(prob, rtol=1e-8, precision=ibr.MIXED if prec == "mixed" else ibr.FP64, device=0,
                         graphs=0, advection=ibr.ADVECT_SL if scheme == "sl" else ibr.ADVECT_CENTRED, n_s=n_s)
    # sampled event timing keeps the instrumentation cost small; enabling
    # again before the timed region resets the counters
    for t in ibr.TIMERS:
        ibr.timer_enable(t, TIMER_STRIDE[t])
    ref_state = None
    for w in range(warmup):
        s.step()
        if w == 1:
            # state after the first two steps (outside the timed region), for the error against the oracle
            sol = s.solution()
            ref_state = {"u": sol.u, "F": sol.F}
    for t in ibr.TIMERS:
        ibr.timer_enable(t, TIMER_STRIDE[t])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, its, ps, vc, res = [], [], [], [], []
    for _ in range(steps):
        t1 = time.perf_counter()
        info = s.step()
        lat.append((time.perf_counter() - t1) * 1e3)
        its.append(info["iters"])
        ps.append(info["ps_applications"])
        vc.append(info["vcycles"])
        res.append(info["rel_residual"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    timers = {t: ibr.timer_read(t) for t in ibr.TIMERS}
    for t in ibr.TIMERS:
        ibr.timer_enable(t, 0)
    s.close()
    return summarise_steps(steps, total, lat, its, ps, vc, res, timers, ref_state)


def summarise_steps(steps, total, lat, its, ps, vc, res, timers, ref_state):
    return {
        "solves_per_s": steps / total,
        "ms_per_step": total * 1e3 / steps,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "fgmres_iters_mean": sum(its) / len(its),
        "ps_applications_mean": sum(ps) / len(ps),
        "vcycles_mean": sum(vc) / len(vc),
        "max_rel_residual": max(res),
        "timers": timers,
        "state_after_2_steps": ref_state,
        "raw": {"steps": steps, "total_s": total, "lat": lat, "its": its, "ps": ps, "vc": vc, "res": res},
    }


def settle(torch):
    import gc
    gc.collect()
    torch.cuda.synchronize()


# steps of one trajectory of the workload (its bodies keep their gap of 4h over them)
TRAJECTORY_STEPS = 20


def split_steps(args):
    """The K timed steps spread over the workload's trajectories (--seeds);
    each trajectory stays within the 20 steps over which its bodies keep
    their gap."""
    seeds = [int(x) for x in args.seeds.split(",") if x.strip()]
    room = TRAJECTORY_STEPS - args.warmup
    if args.steps < 1 or room < 1 or not seeds:
        print("bench.py: need --steps >= 1, --warmup < %d and at least one seed" % TRAJECTORY_STEPS, file=sys.stderr)
        sys.exit(2)
    # more trajectories (the next seeds) when K steps do not fit in the given ones
    while len(seeds) * room < args.steps:
        seeds.append(max(seeds) + 1)
    # the fewest of them that hold K steps, K spread evenly
    n = min(len(seeds), args.steps)
    n = max(n, -(-args.steps // room))
    seeds = seeds[:n]
    per_seed = [args.steps // n + (1 if i < args.steps % n else 0) for i in range(n)]
    return seeds, per_seed


def merge_runs(runs):
    """Several trajectories' timed steps as one job: throughput over the summed
    time, percentiles and means over every step, timer samples summed; the
    first run's state after two steps is kept for the oracle comparison."""
    raw = [r["raw"] for r in runs]
    cat = lambda k: [x for r in raw for x in r[k]]
    timers = {}
    for r in runs:
        for k, v in r["timers"].items():
            acc = timers.setdefault(k, {kk: 0 for kk in v})
            for kk, vv in v.items():
                acc[kk] += vv
    return summarise_steps(sum(r["steps"] for r in raw), sum(r["total_s"] for r in raw), cat("lat"), cat("its"),
                           cat("ps"), cat("vc"), cat("res"), timers, runs[0]["state_after_2_steps"])


def measured_traffic(name):
    import hashlib
    rec = MEASURED_TRAFFIC.get(name)
    if rec is None:
        return None
    with open(os.path.join(ROOT, rec["file"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != rec["sha256_16"]:
            return None
    return rec["bytes_per_launch"]


def roofline(timers):
    """Dominant timed kernel class: algorithmic bytes per launch / mean launch time.

    Classes are sampled with different strides, so the dominant one is chosen
    by the estimated total time (sampled time x stride)."""
    best = max(((k, v) for k, v in timers.items() if k not in COMPOSITE_TIMERS),
               key=lambda kv: kv[1]["ms"] * TIMER_STRIDE[kv[0]])
    name, t = best
    if t["launches"] == 0 or t["ms"] <= 0:
        return None, {}
    per_launch_s = t["ms"] / 1e3 / t["launches"]
    gbs = t["bytes"] / t["launches"] / per_launch_s / 1e9
    others = {}
    for k, v in timers.items():
        if v["launches"] and v["ms"] > 0:
            others[k] = {"gbs": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                         "est_ms_total": round(v["ms"] * TIMER_STRIDE[k], 3),
                         "timed_launches": v["launches"], "sample_stride": TIMER_STRIDE[k],
                         "us_per_launch": round(v["ms"] * 1e3 / v["launches"], 3)}
    return name, {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name), "kernel": name,
                  "us_per_launch": round(per_launch_s * 1e6, 3),
                  "bytes_per_launch": t["bytes"] / t["launches"]}, others


def host_cores():
    """Cores this process may run on, and the CPU model."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def host_threads(n):
    """Context running the oracle's FFTs (SciPy) and BLAS on n threads."""
    import contextlib
    import scipy.fft
    from threadpoolctl import threadpool_limits
    stack = contextlib.ExitStack()
    stack.enter_context(threadpool_limits(limits=n))
    stack.enter_context(scipy.fft.set_workers(n))
    return stack


def cpu_baseline(prob, nsteps=2, scheme="centred"):
    """The oracle's exact solves of the workload's first time steps, timed on
    all host cores (its FFTs and BLAS calls threaded, the rest of its NumPy
    code single-threaded).  Returns the baseline record and the oracle's
    solution of the last of those steps (the reference the GPU solutions are
    compared with)."""
    from oracle import navier
    ncores, model = host_cores()
    with host_threads(ncores):
        t0 = time.perf_counter()
        sols = navier.run(prob, nsteps, scheme=scheme, dense_limit=0, tol=1e-10)
        dt = time.perf_counter() - t0
    rec = {"value": round(nsteps / dt, 5), "unit": "solves/s", "cores": ncores, "kind": "oracle",
           "cpu_model": model, "nproc": os.cpu_count(),
           "sample": "exact constrained solves of the workload's first %d time steps (explicit advection "
                     "right-hand side, Fourier Stokes solves + CG on the 5280x5280 mobility system to 1e-10, "
                     "%s CG iterations), %.1f s; FFTs (SciPy) and BLAS on %d threads, elementwise NumPy on one" %
                     (nsteps, "+".join(str(q.cg_iters) for q in sols), dt, ncores)}
    return rec, sols[-1]


def second_re(args, torch):
    """The same workload at its other Reynolds number (both precisions, the
    same steps), with the advection form chosen for it and the error of the
    state after two steps against the oracle's exact solution."""
    from synthetic import config2_spheres_ns
    re = args.second_re
    scheme = advection_scheme(argparse.Namespace(advection=args.advection, re=re))
    seeds, per_seed = split_steps(args)
    probs = [config2_spheres_ns(sd, re=re) for sd in seeds]
    prob = probs[0]
    out = {"re": re, "advection": scheme}
    res = {}
    for p in ("fp64", "mixed"):
        print("bench: Re %g, %s, seeds %s, %d warmup + %d timed steps in all" % (re, p, args.seeds, args.warmup,
                                                                               args.steps), file=sys.stderr,
              flush=True)
        res[p] = merge_runs([run_precision(pr, p, k, args.warmup, torch, scheme, args.n_s)
                             for pr, k in zip(probs, per_seed)])
        out[p] = {"solves_per_s": round(res[p]["solves_per_s"], 3), "p50_ms": round(res[p]["p50_ms"], 3),
                  "p99_ms": round(res[p]["p99_ms"], 3),
                  "fgmres_iters_mean": round(res[p]["fgmres_iters_mean"], 2),
                  "max_rel_residual": float("%.4g" % res[p]["max_rel_residual"])}
    out["mixed_over_fp64"] = round(res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"], 3)
    if not args.no_cpu_baseline and args.warmup >= 2:
        print("bench: the oracle's first two steps at Re %g" % re, file=sys.stderr, flush=True)
        _, ref = cpu_baseline(prob, scheme=scheme)
        out["err_vs_oracle"] = {
            p: {"u": float("%.3g" % (np.linalg.norm(res[p]["state_after_2_steps"]["u"] - ref.v) /
                                     np.linalg.norm(ref.v))),
                "F": float("%.3g" % (np.linalg.norm(res[p]["state_after_2_steps"]["F"] - ref.F) /
                                     np.linalg.norm(ref.F)))} for p in res}
    return out


def served(args, torch):
    """The served form of the 128^3 workload: independent simulations (seeds
    seed .. seed + T - 1, each a trajectory of warmup + steps time steps from
    rest) offered at once to the request server.  With W workers their
    solves overlap on the device (one context and stream per worker); with
    one worker the server is the plain solver, one simulation after another.
    Every context is created before the timed region (prewarm)."""
    from paper_1505_07865_amd import serve
    from synthetic import config2_spheres_ns
    nsteps = min(args.warmup + args.steps, TRAJECTORY_STEPS)
    probs = [config2_spheres_ns(args.seed + i, re=args.re) for i in range(args.served_trajectories)]
    out = {"trajectories": len(probs), "steps_each": nsteps, "workers": args.workers}
    for prec, workers, tag in (("fp64", 1, "fp64_plain"), ("mixed", 1, "mixed_plain"),
                               ("fp64", args.workers, "fp64_served"), ("mixed", args.workers, "mixed_served")):
        print("bench: served form, %s, %d worker(s), %d trajectories x %d steps" % (prec, workers, len(probs),
                                                                                    nsteps),
              file=sys.stderr, flush=True)
        with serve.Server(precision=prec, workers=workers,
                          advection=1 if advection_scheme(args) == "sl" else 0) as srv:
            srv.prewarm(probs[:1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            futs = [srv.submit_trajectory(p, nsteps) for p in probs]
            res = [f.result() for f in futs]
            torch.cuda.synchronize()
            total = time.perf_counter() - t0
        steps = [st for r in res for st in r["steps"]]
        lat = [st["wall_ms"] for st in steps]
        out[tag] = {"solves_per_s": round(len(steps) / total, 3), "p50_step_ms": round(percentile(lat, 50), 3),
                    "p99_step_ms": round(percentile(lat, 99), 3),
                    "fgmres_iters_mean": round(sum(st["iters"] for st in steps) / len(steps), 2),
                    "max_rel_residual": float("%.4g" % max(st["rel_residual"] for st in steps))}
    out["mixed_served_over_fp64_plain"] = round(out["mixed_served"]["solves_per_s"] /
                                                out["fp64_plain"]["solves_per_s"], 3)
    out["mixed_served_over_fp64_served"] = round(out["mixed_served"]["solves_per_s"] /
                                                 out["fp64_served"]["solves_per_s"], 3)
    return out


def serving_leg(args, torch, nreq):
    """Serving workload: a seeded trace of nreq independent steady constrained
    solves (grids 32^2, 128^2, 256^2, 32^3, 64^3, 128^3; 1-8 bodies of radius
    4h-8h with markers at ~2h; U, Omega ~ U[-1,1]; rtol 1e-8) offered to the
    request server, first all at once (saturation: solves/s), then as Poisson
    arrivals at 0.7 x the measured fp64 capacity (p50/p99 latency, queueing
    included), for the mixed-precision and the fp64 solver on the same trace.
    Returns the per-precision results."""
    from paper_1505_07865_amd import serve
    from synthetic import serving_trace
    trace = serving_trace(args.seed, nreq, 1.0)
    res = {}
    for prec in ("fp64", "mixed"):
        with serve.Server(precision=prec, workers=args.workers) as srv:
            srv.prewarm([r["problem"] for r in trace])
            print("bench: serving %s, %d requests at saturation" % (prec, len(trace)), file=sys.stderr,
                  flush=True)
            sat = serve.replay(trace, srv, qps=None)
            res[prec] = {"saturation": {k: v for k, v in sat.items() if k != "results"}}
            res[prec]["iters_mean"] = sum(r["info"]["iters"] for r in sat["results"]) / len(trace)
            res[prec]["max_rel_residual"] = max(r["info"]["rel_residual"] for r in sat["results"])
    qps = 0.7 * res["fp64"]["saturation"]["solves_per_s"]
    for prec in ("fp64", "mixed"):
        with serve.Server(precision=prec, workers=args.workers) as srv:
            srv.prewarm([r["problem"] for r in trace])
            print("bench: serving %s, Poisson arrivals at %.1f req/s" % (prec, qps), file=sys.stderr, flush=True)
            lat = serve.replay(trace, srv, qps=qps)
            res[prec]["at_0.7x_fp64_capacity"] = {k: v for k, v in lat.items() if k != "results"}
    return res


def serving_summary(res, nreq, workers):
    return {"requests": nreq, "workers": workers,
            "mixed_solves_per_s": round(res["mixed"]["saturation"]["solves_per_s"], 3),
            "fp64_solves_per_s": round(res["fp64"]["saturation"]["solves_per_s"], 3),
            "mixed_over_fp64": round(res["mixed"]["saturation"]["solves_per_s"] /
                                     res["fp64"]["saturation"]["solves_per_s"], 3),
            "qps_at_0.7x_fp64": round(res["mixed"]["at_0.7x_fp64_capacity"]["qps_offered"], 3),
            "mixed_p50_ms": round(res["mixed"]["at_0.7x_fp64_capacity"]["p50_ms"], 3),
            "mixed_p99_ms": round(res["mixed"]["at_0.7x_fp64_capacity"]["p99_ms"], 3),
            "fp64_p50_ms": round(res["fp64"]["at_0.7x_fp64_capacity"]["p50_ms"], 3),
            "fp64_p99_ms": round(res["fp64"]["at_0.7x_fp64_capacity"]["p99_ms"], 3),
            "mixed_iters_mean": round(res["mixed"]["iters_mean"], 2),
            "fp64_iters_mean": round(res["fp64"]["iters_mean"], 2),
            "max_rel_residual": float("%.4g" % max(res["mixed"]["max_rel_residual"],
                                                   res["fp64"]["max_rel_residual"]))}


def serving(args, torch):
    """The serving workload alone, on the whole trace (``--nreq``)."""
    res = serving_leg(args, torch, args.nreq)
    trace_len = args.nreq
    line = {
        "metric": "serving: solves/s at saturation and p50/p99 latency at 0.7x fp64 capacity, mixed vs fp64",
        "value": round(res["mixed"]["saturation"]["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f32 preconditioner + f64 outer",
        "data": "synthetic",
        "config": {"workload": "steady constrained solves, seeded Poisson trace of %d requests over grids "
                               "32^2/128^2/256^2/32^3/64^3/128^3 with 1-8 bodies, rtol 1e-8, %d workers"
                               % (trace_len, args.workers), "seed": args.seed},
        "p50_ms": round(res["mixed"]["at_0.7x_fp64_capacity"]["p50_ms"], 3),
        "p99_ms": round(res["mixed"]["at_0.7x_fp64_capacity"]["p99_ms"], 3),
        "mixed": res["mixed"],
        "fp64": res["fp64"],
        "mixed_over_fp64": round(res["mixed"]["saturation"]["solves_per_s"] /
                                 res["fp64"]["saturation"]["solves_per_s"], 3),
    }
    print(json.dumps(line), flush=True)


def free_kinematics(args, torch):
    """Free kinematics (bodies under applied loads): a sedimenting suspension
    of 16 spheres (radius 6h, 110 markers each) in a periodic 128^3 box,
    steady Stokes, every body free under the same weight along -z and zero
    torque.  Per precision: the set-up of the free bodies (body mobilities),
    repeated solves from a zero initial guess to relative residual 1e-8, and
    beside them the prescribed-motion solve at the velocities the free solve
    returned (the same fields), so the difference is the cost of the free
    rows."""
    from paper_1505_07865_amd import ibr
    from synthetic import sedimentation_problem
    prob, F, T = sedimentation_problem(args.seed)
    mask = [1] * prob.nbodies
    out = {}
    for prec in ("fp64", "mixed"):
        s = ibr.from_problem(prob, rtol=1e-8, precision=ibr.MIXED if prec == "mixed" else ibr.FP64, graphs=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_free_bodies(mask, F, T)
        setup_ms = (time.perf_counter() - t0) * 1e3
        s.solve()

        def timed(nrep):
            infos, wall = [], []
            for _ in range(nrep):
                t1 = time.perf_counter()
                infos.append(s.solve())
                wall.append((time.perf_counter() - t1) * 1e3)
            return infos, wall

        infos, wall = timed(args.free_solves)
        U, Om = s.velocities()
        sol = s.solution()
        s.set_free_bodies(None)
        s.set_velocities(U, Om)
        s.solve()
        pinfos, pwall = timed(args.free_solves)
        s.close()
        out[prec] = {
            "free": {"solves_per_s": round(len(wall) / (sum(wall) / 1e3), 3), "p50_ms": round(percentile(wall, 50), 3),
                     "p99_ms": round(percentile(wall, 99), 3), "iters": infos[-1]["iters"],
                     "ps_applications": infos[-1]["ps_applications"],
                     "max_rel_residual": float("%.4g" % max(i["rel_residual"] for i in infos)),
                     "setup_ms": round(setup_ms, 3)},
            "prescribed_same_motion": {"solves_per_s": round(len(pwall) / (sum(pwall) / 1e3), 3),
                                       "iters": pinfos[-1]["iters"],
                                       "ps_applications": pinfos[-1]["ps_applications"]},
            "mean_settling_velocity_z": float("%.6g" % U[:, 2].mean()),
            "max_load_mismatch": float("%.3g" % np.abs(sol.F - F).max()),
        }
        print("bench: free kinematics %s: %.2f solves/s, %d iterations (prescribed at the same motion: %d)"
              % (prec, out[prec]["free"]["solves_per_s"], out[prec]["free"]["iters"],
                 out[prec]["prescribed_same_motion"]["iters"]), file=sys.stderr, flush=True)
    line = {"metric": "free-kinematics solves/s at 1e-8 residual, sedimenting suspension, mixed vs FP64, 3D 128^3",
            "value": out["mixed"]["free"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f32 preconditioner + f64 outer",
            "data": "synthetic",
            "config": {"workload": "3D steady Stokes, periodic 128^3, 16 free spheres R=6h x 110 markers under "
                                   "weight 1 along -z, zero torque, rtol 1e-8, solves from rest",
                       "seed": args.seed, "solves": args.free_solves},
            "mixed": out["mixed"], "fp64": out["fp64"],
            "mixed_over_fp64": round(out["mixed"]["free"]["solves_per_s"] / out["fp64"]["free"]["solves_per_s"], 3)}
    print(json.dumps(line), flush=True)


def slit_channel(args, torch):
    """Slit channel: steady Stokes between no-slip walls at z = 0 and z = L
    (periodic along x and y), 3D 128^3, 16 spheres of radius 6h (113 markers
    each) with prescribed velocities U ~ U[-1, 1]^3, every surface at least 2h
    from the walls.  Per precision: repeated solves from a zero initial guess
    to relative residual 1e-8 (host clock around each synchronous solve) with
    N_s = 4 and N_s = 2 inner iterations, and beside them the same bodies in
    the periodic box (N_s = 2), so the difference is the cost of the walls:
    their multigrid is the plain one-cell-per-thread cycle, not the
    bandwidth-tuned periodic one, and P_S^-1 approximates the wall-bounded
    Stokes operator less well than the periodic one, as Sec. 7.1 notes (which
    also finds N_s = 4 the robust choice there).  The headline value is the
    mixed-precision N_s = 4 rate; its roofline is the finest-level wall half
    sweep (timed live with HIP events, every 29th launch)."""
    from paper_1505_07865_amd import ibr
    from synthetic import slit_problem
    prob = slit_problem(args.seed, dim=3, n=128, nbodies=16, radius_h=6.0, wall_gap_h=2.0, rotate=False)
    out = {}
    roof = None
    for prec in ("fp64", "mixed"):
        res = {}
        for walls, ns in ((1, 4), (1, 2), (0, 2)):
            s = ibr.from_problem(prob, rtol=1e-8, precision=ibr.MIXED if prec == "mixed" else ibr.FP64,
                                 walls=walls, n_s=ns)
            s.solve()
            timed = prec == "mixed" and walls and ns == 4
            if timed:
                ibr.timer_enable("wall_rb_fine", TIMER_STRIDE["wall_rb_fine"])
            infos, wall = [], []
            for _ in range(args.slit_solves):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                infos.append(s.solve())
                wall.append((time.perf_counter() - t1) * 1e3)
            if timed:
                t = ibr.timer_read("wall_rb_fine")
                ibr.timer_enable("wall_rb_fine", 0)
                if t["launches"] and t["ms"] > 0:
                    per_s = t["ms"] / 1e3 / t["launches"]
                    gbs = t["bytes"] / t["launches"] / per_s / 1e9
                    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "wall_rb_fine",
                            "us_per_launch": round(per_s * 1e6, 3), "bytes_per_launch": t["bytes"] / t["launches"]}
            F, _ = s.forces()
            s.close()
            key = ("walls_ns%d" % ns) if walls else "periodic_same_bodies"
            res[key] = {
                "solves_per_s": round(len(wall) / (sum(wall) / 1e3), 3), "p50_ms": round(percentile(wall, 50), 3),
                "p99_ms": round(percentile(wall, 99), 3), "iters": infos[-1]["iters"],
                "ps_applications": infos[-1]["ps_applications"],
                "max_rel_residual": float("%.4g" % max(i["rel_residual"] for i in infos)),
                "mean_abs_force": float("%.6g" % np.abs(F).mean())}
        out[prec] = res
        print("bench: slit channel %s: N_s = 4 %.2f solves/s, %d iterations; N_s = 2 %.2f, %d; periodic box %.2f "
              "solves/s, %d iterations"
              % (prec, res["walls_ns4"]["solves_per_s"], res["walls_ns4"]["iters"], res["walls_ns2"]["solves_per_s"],
                 res["walls_ns2"]["iters"], res["periodic_same_bodies"]["solves_per_s"],
                 res["periodic_same_bodies"]["iters"]),
              file=sys.stderr, flush=True)
    line = {"metric": "slit-channel solves/s at 1e-8 residual, mixed vs FP64, 3D 128^3",
            "value": out["mixed"]["walls_ns4"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f32 preconditioner + f64 outer",
            "data": "synthetic",
            "config": {"workload": "3D steady Stokes, 128^3, no-slip walls at z = 0 and z = L, periodic x and y, "
                                   "16 spheres R=6h x 113 markers, U ~ U[-1,1]^3, N_s = 4, rtol 1e-8, solves "
                                   "from rest", "seed": args.seed, "solves": args.slit_solves},
            "roofline": roof, "mixed": out["mixed"], "fp64": out["fp64"],
            "mixed_over_fp64": round(out["mixed"]["walls_ns4"]["solves_per_s"] /
                                     out["fp64"]["walls_ns4"]["solves_per_s"], 3)}
    print(json.dumps(line), flush=True)


def large(args, torch):
    """The 256^3 configuration: steady Stokes in a periodic 256^3 box with 100
    spheres of radius 8h (200 markers each, 20 000 markers, 100 mobility
    blocks of 600 x 600), restart 50, rtol 1e-8.  Per precision: the
    context's set-up and one untimed solve, then timed solves from a zero
    initial guess (host clock around each synchronous solve).  The mixed
    run carries the live kernel timers; its roofline is that of the dominant
    timed class, as in the default line."""
    from paper_1505_07865_amd import ibr
    from synthetic import config4_spheres256
    prob = config4_spheres256(args.seed)
    out, roof, others = {}, None, {}
    for prec in ("fp64", "mixed"):
        s = ibr.from_problem(prob, rtol=1e-8, restart=50, precision=ibr.MIXED if prec == "mixed" else ibr.FP64,
                             graphs=0)
        s.solve()
        if prec == "mixed":
            for t in ibr.TIMERS:
                ibr.timer_enable(t, TIMER_STRIDE[t])
        infos, wall = [], []
        for _ in range(args.large_solves):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            infos.append(s.solve())
            wall.append((time.perf_counter() - t1) * 1e3)
        if prec == "mixed":
            timers = {t: ibr.timer_read(t) for t in ibr.TIMERS}
            for t in ibr.TIMERS:
                ibr.timer_enable(t, 0)
            _, roof, others = roofline(timers)
        s.close()
        out[prec] = {"solves_per_s": round(len(wall) / (sum(wall) / 1e3), 4), "p50_ms": round(percentile(wall, 50), 2),
                     "iters": infos[-1]["iters"], "restarts": infos[-1]["restarts"],
                     "ps_applications": infos[-1]["ps_applications"],
                     "max_rel_residual": float("%.4g" % max(i["rel_residual"] for i in infos))}
        print("bench: 256^3 %s: %.3f solves/s (%.0f ms), %d iterations" % (prec, out[prec]["solves_per_s"],
              out[prec]["p50_ms"], out[prec]["iters"]), file=sys.stderr, flush=True)
    line = {"metric": "solves/s at 1e-8 residual, mixed vs FP64, 3D 256^3 steady, 100 spheres",
            "value": out["mixed"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "vs_baseline": None, "dtype": "f32 preconditioner + f64 outer", "data": "synthetic",
            "config": {"workload": "3D steady Stokes, periodic 256^3, 100 spheres R=8h x 200 markers, "
                                   "U, Omega ~ U[-1,1]^3, restart 50, rtol 1e-8, solves from rest",
                       "seed": args.seed, "solves": args.large_solves},
            "roofline": roof, "kernels": others, "mixed": out["mixed"], "fp64": out["fp64"],
            "mixed_over_fp64": round(out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"], 3)}
    print(json.dumps(line), flush=True)


def small(args, torch):
    """The two small configurations, every seed: the 2D disk (64^2, eta = 1,
    steady, one disk of radius 8h with 25 markers, U = (1, 0); fp64 to rtol
    1e-10) and the 3D sphere (64^3, steady, one sphere of radius 8h with 200
    markers, U, Omega ~ U[-1,1]^3; fp64 and mixed to rtol 1e-8).  Per seed and
    precision: the context's set-up and one untimed solve, then timed solves
    from a zero initial guess (host clock around each synchronous solve,
    captured iteration graphs as a caller gets them by default); the error of
    the solution against the oracle's exact solve (dense mobility solve for
    the disk, CG to 1e-11 for the sphere), itself timed on the host's cores
    (FFTs and BLAS threaded).  The disk's drag F_x/(eta V) is reported beside
    the periodic drag law at the geometric radius."""
    from oracle import constrained, hasimoto
    from paper_1505_07865_amd import ibr
    from synthetic import config0_disk2d, config1_sphere3d
    ncores, _ = host_cores()
    cases = (("disk2d_64", config0_disk2d, ("fp64",), 1e-10), ("sphere3d_64", config1_sphere3d, ("fp64", "mixed"), 1e-8))
    out = {}
    for name, make, precs, rtol in cases:
        rec = {"rtol": rtol, "seeds": []}
        for seed in range(args.small_seeds):
            prob = make(seed)
            with host_threads(ncores):
                t0 = time.perf_counter()
                ex = constrained.solve_problem(prob, **({} if prob.dim == 2 else dict(dense_limit=0, tol=1e-11)))
                t_or = time.perf_counter() - t0
            srec = {"seed": seed, "markers": int(prob.nmarkers), "oracle_ms": round(t_or * 1e3, 2)}
            if prob.dim == 2:
                srec["drag_oracle"] = round(float(ex.F[0, 0]), 4)
            for prec in precs:
                s = ibr.from_problem(prob, rtol=rtol, precision=ibr.MIXED if prec == "mixed" else ibr.FP64)
                s.solve()
                wall, infos = [], []
                for _ in range(args.small_solves):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    infos.append(s.solve())
                    wall.append((time.perf_counter() - t1) * 1e3)
                sol = s.solution()
                s.close()
                r = {"solves_per_s": round(len(wall) / (sum(wall) / 1e3), 2),
                     "p50_ms": round(percentile(wall, 50), 3), "p99_ms": round(percentile(wall, 99), 3),
                     "iters": infos[-1]["iters"], "ps_applications": infos[-1]["ps_applications"],
                     "max_rel_residual": float("%.4g" % max(i["rel_residual"] for i in infos)),
                     "err_vs_oracle": {"u": float("%.3g" % (np.linalg.norm(sol.u - ex.v) / np.linalg.norm(ex.v))),
                                       "F": float("%.3g" % (np.linalg.norm(sol.F - ex.F) / np.linalg.norm(ex.F)))}}
                if prob.dim == 2:
                    r["drag"] = round(float(sol.F[0, 0]), 4)
                srec[prec] = r
                print("bench: %s seed %d %s: %.1f solves/s, %d iterations, err u %.2g" %
                      (name, seed, prec, r["solves_per_s"], r["iters"], r["err_vs_oracle"]["u"]),
                      file=sys.stderr, flush=True)
            rec["seeds"].append(srec)
        for prec in precs:
            rates = [x[prec]["solves_per_s"] for x in rec["seeds"]]
            rec[prec + "_solves_per_s_mean"] = round(sum(rates) / len(rates), 2)
        if "mixed" in precs:
            rec["mixed_over_fp64"] = round(rec["mixed_solves_per_s_mean"] / rec["fp64_solves_per_s_mean"], 3)
        if name.startswith("disk"):
            rec["drag_law_at_geometric_radius"] = round(hasimoto.drag2d(8.0 / 64, 1.0), 4)
        out[name] = rec
    line = {"metric": "solves/s + p50/p99 latency, small steady configurations (2D 64^2 disk, 3D 64^3 sphere)",
            "value": out["sphere3d_64"]["mixed_solves_per_s_mean"], "unit": "solves/s", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f64 (disk); f32 preconditioner + f64 outer "
            "(sphere value)", "data": "synthetic",
            "config": {"workload": "2D 64^2 disk R=8h x 25 markers (fp64, rtol 1e-10) and 3D 64^3 sphere R=8h x "
                                   "200 markers (fp64 and mixed, rtol 1e-8), steady, seeds 0-%d" %
                                   (args.small_seeds - 1), "solves": args.small_solves},
            "cpu_baseline_kind": "oracle exact solve (Fourier Stokes + dense or CG mobility solve), FFTs and BLAS on %d host threads" % ncores,
            "cases": out}
    print(json.dumps(line), flush=True)


def blocks(args, torch):
    """Per-body mobility set-up (assembly, shifted Cholesky on fp64 MFMA
    tiles, triangular inverse, M~^-1 = X^T X) for the 256^3 configuration's
    100 spheres of 200 markers (100 blocks of 600 x 600): the synchronous
    ibr_set_bodies call timed by the host clock; the flop count is the dense
    one, n^3/3 each for the factor, the triangular inverse and X^T X."""
    from paper_1505_07865_amd import ibr
    from synthetic import config4_spheres256
    prob = config4_spheres256(args.seed)
    s = ibr.from_problem(prob, rtol=1e-8, precision=ibr.MIXED, graphs=0)
    sizes = np.diff(prob.offsets) * prob.dim
    flops = float(np.sum(sizes.astype(np.float64) ** 3))
    wall = []
    for _ in range(args.block_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_bodies(prob.R, prob.offsets, prob.centres)
        wall.append((time.perf_counter() - t0) * 1e3)
    s.close()
    ms = percentile(wall, 50)
    tf = flops / (ms * 1e-3) / 1e12
    line = {"metric": "per-body mobility set-up (assembly + Cholesky + inverse), 100 blocks of 600 x 600",
            "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "3D 256^3 steady, 100 spheres R=8h x 200 markers (config of the 256^3 solve)",
                       "seed": args.seed, "reps": args.block_reps},
            "wall_ms": [round(w, 3) for w in wall],
            "roofline": {"bound": "mfma", "achieved": round(tf, 4), "peak": 78.6, "unit": "TFLOP/s",
                         "frac": round(tf / 78.6, 5), "traffic": None, "flops": flops,
                         "note": "end-to-end set-up time (host marker checks, binning and the block kernels)"}}
    print(json.dumps(line), flush=True)


def ablation(args, torch):
    """The periodic half of the paper's solver study (Sec. 7.1): P_S^-1
    applications (the paper's cost proxy) and FGMRES iterations to reach
    relative residual 1e-8 (and 1e-6, 1e-10), for
      (a) a 162-marker icosahedral shell, empty or filled, in 32^3, steady and
          one Re = 10 step, N_s in {1, 2, 4, 8}, full and lower-triangular
          Schur preconditioner;
      (b) shells of 162 / 642 / 2562 markers in 32^3 / 64^3 / 128^3 (spacing
          2h), steady, N_s = 4, full and lower-triangular;
    and its non-periodic half in the slit channel (no-slip walls at z = 0
    and z = 1): (a) for the empty 162-marker shell, steady, and (b); and in
    the paper's closed box (no-slip walls on every side, side 4.35 sphere
    radii, the sphere at its centre): (a) for the empty and the filled
    sphere, steady, and (b); fp64 and mixed precision, restart 100, with the
    solve time."""
    from paper_1505_07865_amd import ibr
    from synthetic import box_shell, shell_problem
    rows = []

    def run(prob, pc, ns, prec, rtol):
        s = ibr.from_problem(prob, rtol=rtol, pc=ibr.PC_FULL if pc == "full" else ibr.PC_LOWER, n_s=ns,
                             precision=ibr.MIXED if prec == "mixed" else ibr.FP64, graphs=0, max_iters=2000,
                             mobility=ibr.MOB_ANALYTIC if args.analytic_mobility else ibr.MOB_AUTO)
        s.solve(check=False)           # first solve: warm caches / allocation
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve(check=False)    # a case that does not converge in 2000 iterations is a result
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        s.close()
        return {"case": prob.name, "markers": int(prob.nmarkers), "pc": pc, "n_s": ns, "precision": prec,
                "rtol": rtol, "iters": info["iters"], "ps_applications": info["ps_applications"],
                "rel_residual": info["rel_residual"], "converged": info["rel_residual"] <= rtol,
                "ms": round(ms, 3)}

    parts = set(args.ablation_parts.split(","))
    for filled in (False, True) if "periodic" in parts else ():
        for re in (0.0, 10.0):
            prob = shell_problem(args.seed, 32, 2, filled=filled, re=re)
            for pc in ("full", "lower"):
                for ns in (1, 2, 4, 8):
                    for rtol in (1e-6, 1e-8, 1e-10):
                        rows.append(run(prob, pc, ns, "fp64", rtol))
                    rows.append(run(prob, pc, ns, "mixed", 1e-8))
            print("bench: ablation %s done" % prob.name, file=sys.stderr, flush=True)
    for level, n in ((2, 32), (3, 64), (4, 128)) if "periodic" in parts else ():
        prob = shell_problem(args.seed, n, level)
        for pc in ("full", "lower"):
            for prec in ("fp64", "mixed"):
                rows.append(run(prob, pc, 4, prec, 1e-8))
        print("bench: ablation %s done" % prob.name, file=sys.stderr, flush=True)
    # the non-periodic half, in the slit channel (no-slip walls at z = 0 and z = 1)
    for pc in ("full", "lower") if "slit" in parts else ():
        prob = shell_problem(args.seed, 32, 2, walls=True)
        for ns in (1, 2, 4, 8):
            rows.append(run(prob, pc, ns, "fp64", 1e-8))
            rows.append(run(prob, pc, ns, "mixed", 1e-8))
        print("bench: ablation %s %s done" % (prob.name, pc), file=sys.stderr, flush=True)
    for level, n in ((2, 32), (3, 64), (4, 128)) if "slit" in parts else ():
        prob = shell_problem(args.seed, n, level, walls=True)
        for pc in ("full", "lower"):
            for prec in ("fp64", "mixed"):
                rows.append(run(prob, pc, 4, prec, 1e-8))
        print("bench: ablation %s done" % prob.name, file=sys.stderr, flush=True)
    # ... and in the paper's own non-periodic domain: the closed box (no-slip walls on every side, 4.35 radii)
    for filled in (False, True) if "box" in parts else ():
        prob = box_shell(32, 2, filled=filled)
        for pc in ("full", "lower"):
            for ns in (1, 2, 4, 8):
                rows.append(run(prob, pc, ns, "fp64", 1e-8))
                rows.append(run(prob, pc, ns, "mixed", 1e-8))
        print("bench: ablation %s done" % prob.name, file=sys.stderr, flush=True)
    for level, n in ((2, 32), (3, 64), (4, 128)) if "box" in parts else ():
        prob = box_shell(n, level)
        for pc in ("full", "lower"):
            for prec in ("fp64", "mixed"):
                rows.append(run(prob, pc, 4, prec, 1e-8))
        print("bench: ablation %s done" % prob.name, file=sys.stderr, flush=True)
    cand = [r for r in rows if r["rtol"] == 1e-8 and r["precision"] == "fp64" and r["converged"]]
    best = min([r for r in cand if r["case"].startswith("shell_l2_empty_n32_re0")] or cand,
               key=lambda r: r["ps_applications"])
    line = {"metric": "P_S^-1 applications to relative residual 1e-8 (solver study, periodic)",
            "value": best["ps_applications"], "unit": "P_S^-1 applications", "n_gpus": 1,
            "higher_is_better": False, "vs_baseline": None, "data": "synthetic",
            "config": {"workload": "icosahedral shells (162/642/2562 markers, spacing 2h, empty or filled), "
                                   "periodic 32^3/64^3/128^3, steady and Re = 10, and the same shells in the "
                                   "slit channel and in the closed box, restart 100",
                       "seed": args.seed, "best_case": best},
            "rows": rows}
    print(json.dumps(line), flush=True)


def mobility_study(args, torch):
    """The approximate mobility's effect on the solver (Secs. 4.2 and 5.3):
    P_S^-1 applications and FGMRES iterations to relative residual 1e-8,
    fp64, with the analytic M~ (RPY / Brinkmanlet readings) and with the
    fitted M~ of Appendix A's forms, on
      the solver study's shells (162 markers in 32^3, empty or filled,
      steady and one Re = 10 step, beta = 0.36; lower-triangular
      preconditioner, N_s = 2 and 4) and Sec. 7.1's shell in the closed box;
      the 128^3 moving-spheres workload at Re = 10 (beta = 0.3): the first
      three time steps, mixed precision as benchmarked;
      the 256^3 configuration (steady, 100 spheres of 200 markers): one
      solve from rest, mixed precision, restart 50;
      in 2D (Appendix B's forms): the 64^2 disk (rtol 1e-10), 8 disks of
      radius 6h at 256^2 (both precisions) and 4 disks at 128^2, one
      unsteady solve at beta = 0.3."""
    from paper_1505_07865_amd import ibr
    from synthetic import (box_shell, config0_disk2d, config2_spheres_ns, config4_spheres256, shell_problem,
                           small_problem)
    rows = []
    mobs = (("analytic", ibr.MOB_ANALYTIC), ("fitted", ibr.MOB_FITTED))

    def solve_row(prob, label, **kw):
        for name, mob in mobs:
            s = ibr.from_problem(prob, mobility=mob, graphs=0, **kw)
            info = s.solve()
            s.close()
            rows.append({"case": label, "mobility": name, "iters": info["iters"],
                         "ps_applications": info["ps_applications"], "rel_residual": info["rel_residual"],
                         **{k: v for k, v in kw.items() if k in ("n_s", "precision")}})

    for filled in (False, True):
        for re in (0.0, 10.0):
            prob = shell_problem(args.seed, 32, 2, filled=filled, re=re)
            for ns in (2, 4):
                solve_row(prob, prob.name, rtol=1e-8, pc=ibr.PC_LOWER, n_s=ns, max_iters=2000)
            print("bench: mobility study %s done" % prob.name, file=sys.stderr, flush=True)
    for filled in (False, True):
        prob = box_shell(32, 2, filled=filled)
        solve_row(prob, prob.name, rtol=1e-8, pc=ibr.PC_LOWER, n_s=4, max_iters=2000)
    print("bench: mobility study box shells done", file=sys.stderr, flush=True)
    prob = config2_spheres_ns(args.seed, re=10.0, n=128)
    for name, mob in mobs:
        s = ibr.from_problem(prob, mobility=mob, rtol=1e-8, precision=ibr.MIXED)
        its, aps = [], []
        for _ in range(3):
            info = s.step()
            its.append(info["iters"])
            aps.append(info["ps_applications"])
        s.close()
        rows.append({"case": "spheres_ns_128_re10_steps1-3", "mobility": name, "iters": its, "ps_applications": aps,
                     "precision": ibr.MIXED})
    print("bench: mobility study 128^3 done", file=sys.stderr, flush=True)
    prob = config4_spheres256(args.seed)
    solve_row(prob, "spheres_256_steady", rtol=1e-8, precision=ibr.MIXED, restart=50, max_iters=400)
    # two dimensions (Appendix B's forms): the 64^2 disk, many disks at 256^2 (the serving trace's hard
    # case), and an unsteady solve (beta = 0.3)
    solve_row(config0_disk2d(args.seed), "disk_64", rtol=1e-10)
    for prec in (ibr.FP64, ibr.MIXED):
        solve_row(small_problem(args.seed, 2, 256, nbodies=8, radius_h=6.0), "disks8_256_steady", rtol=1e-8,
                  precision=prec, max_iters=1000)
    h = 1.0 / 128
    solve_row(small_problem(args.seed, 2, 128, nbodies=4, radius_h=6.0, rho=1.0, eta=0.6 * h, dt=0.5 * h),
              "disks4_128_beta0.3", rtol=1e-8, max_iters=1000)
    print("bench: mobility study 2D done", file=sys.stderr, flush=True)
    line = {"metric": "P_S^-1 applications to relative residual 1e-8, fitted vs analytic approximate mobility",
            "value": None, "unit": "P_S^-1 applications", "n_gpus": 1, "higher_is_better": False,
            "vs_baseline": None, "data": "synthetic",
            "config": {"workload": "solver-study shells (periodic 32^3, closed box 32^3), 128^3 spheres at Re 10, "
                                   "256^3 steady spheres", "seed": args.seed},
            "rows": rows}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); the path is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from synthetic import config2_spheres_ns

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    if args.serving:
        serving(args, torch)
        return
    if args.ablation:
        ablation(args, torch)
        return
    if args.mobility_study:
        mobility_study(args, torch)
        return
    if args.free:
        free_kinematics(args, torch)
        return
    if args.blocks:
        blocks(args, torch)
        return
    if args.walls:
        slit_channel(args, torch)
        return
    if args.large:
        large(args, torch)
        return
    if args.small:
        small(args, torch)
        return
    seeds, per_seed = split_steps(args)
    probs = [config2_spheres_ns(sd, re=args.re) for sd in seeds]
    prob = probs[0]
    scheme = advection_scheme(args)
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for p in precs:
        print("bench: %s, seeds %s, %d warmup + %d timed steps each" % (p, args.seeds, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        res[p] = merge_runs([run_precision(pr, p, k, args.warmup, torch, scheme, args.n_s)
                             for pr, k in zip(probs, per_seed)])
        print("bench: %s %.2f solves/s, %.1f FGMRES iters/step" % (p, res[p]["solves_per_s"],
                                                                   res[p]["fgmres_iters_mean"]),
              file=sys.stderr, flush=True)
    head = res["mixed"] if "mixed" in res else res[precs[0]]
    name, roof, others = roofline(head["timers"])
    line = {
        "metric": "solves/s + p50/p99 latency at 1e-8 residual, mixed vs FP64, 3D 128^3",
        "value": round(head["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "trajectories": len(seeds),
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner + f64 outer" if "mixed" in res else "f64",
        "data": "synthetic",
        "config": {"workload": "3D unsteady NS, periodic 128^3 MAC grid, Re=%g, dt=0.5h, 16 moving spheres "
                               "R=6h x 110 markers, rtol 1e-8, N_s=%d, lower-triangular Schur preconditioner "
                               "with the fitted approximate mobility, %s advection"
                               % (args.re, args.n_s, "semi-Lagrangian" if scheme == "sl" else "centred AB2"),
                   "grid": 128, "bodies": 16, "markers": int(prob.nmarkers), "re": args.re, "seeds": seeds,
                   "rtol": 1e-8, "n_s": args.n_s, "advection": scheme,
                   "approximate_mobility": "fitted (Appendix A forms)"},
        "p50_ms": round(head["p50_ms"], 3),
        "p99_ms": round(head["p99_ms"], 3),
        "fgmres_iters_per_step": round(head["fgmres_iters_mean"], 2),
        "ps_applications_per_step": round(head["ps_applications_mean"], 2),
        "roofline": roof,
        "kernels": others,
    }
    if "vcycle" in others:
        # whole V-cycle calls: each P_S^-1 makes one on the 3 velocity fields and one on the pressure
        line["ms_per_vcycle_call"] = round(others["vcycle"]["us_per_launch"] / 1e3, 4)
        line["vcycle_calls_per_step"] = round(2 * head["ps_applications_mean"], 2)
        line["field_vcycles_per_step"] = round(head["vcycles_mean"], 2)
    for p in precs:
        line[p] = {k: (float("%.4g" % v) if isinstance(v, float) else v) for k, v in res[p].items()
                   if k not in ("timers", "state_after_2_steps", "raw")}
    if "mixed" in res and "fp64" in res:
        line["mixed_over_fp64"] = round(res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"], 3)
    # each further leg starts from a settled device and host (the previous
    # legs' contexts destroyed, their host arrays collected): the serving
    # mix's Poisson latencies are sensitive to stalls
    if args.precision == "both" and args.mix_requests > 0:
        settle(torch)
        # the serving trace (mixed grid sizes and body counts, Poisson arrivals), a short prefix of it
        print("bench: serving mix, %d requests" % args.mix_requests, file=sys.stderr, flush=True)
        line["serving_mix"] = serving_summary(serving_leg(args, torch, args.mix_requests), args.mix_requests,
                                              args.workers)
    if args.precision == "both" and args.second_re > 0 and args.second_re != args.re:
        settle(torch)
        line["second_re"] = second_re(args, torch)
    if args.precision == "both" and not args.no_served:
        settle(torch)
        line["served"] = served(args, torch)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on the workload's first two steps", file=sys.stderr, flush=True)
        line["cpu_baseline"], ref = cpu_baseline(prob, scheme=scheme)
        err = {}
        for p in precs:
            st = res[p]["state_after_2_steps"]
            if st is not None:
                err[p] = {"u": float("%.3g" % (np.linalg.norm(st["u"] - ref.v) / np.linalg.norm(ref.v))),
                          "F": float("%.3g" % (np.linalg.norm(st["F"] - ref.F) / np.linalg.norm(ref.F)))}
        if err:
            err["reference"] = "the oracle's exact solution of the second time step (CG to 1e-10); relative L2"
            line["err_vs_oracle"] = err
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
