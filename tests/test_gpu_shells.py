"""Concentric-shells accuracy study on the GPU (Sec. 7.3): Stokes flow between
a sphere and a spherical cavity, both represented by icosahedral shells of
markers, against the analytic flow of ``oracle.shells``.

Per resolution (32^3, 64^3, 128^3 with 12/162, 42/642, 162/2562 markers):
the inner shell alone in the periodic box gives its hydrodynamic radius R1
from its drag (periodic drag law, ``oracle.hasimoto``); the drag on it inside
the cavity gives the cavity's radius R2 through the drag law of the paper's
appendix; then the velocity and pressure errors against the analytic flow
with those radii.  fp64, rtol 1e-8 (the errors are of order 1e-2; an
isolated 162-marker shell at 128^3 cannot reach 1e-10: with its small
right-hand side, rounding in the h^-2-scaled operator leaves a relative
residual of about 1.3e-10).

Checks: at 32^3 the GPU numbers equal the oracle's exact solve's; under
refinement R1/R1_geometric falls and R2/R2_geometric rises toward 1, and the
velocity errors fall at a rate above 0.7 per refinement (first order is the
method's; the paper reports rates of 1.0-1.8).  The table is printed and
written to shells_table.json in the results folder.
"""
import json
import math
import os

from conftest import results_dir

import numpy as np
import pytest

from oracle import constrained, hasimoto, shells
from synthetic import concentric_shells, single_shell

pytestmark = pytest.mark.gpu

LEVELS = ((32, 0), (64, 1), (128, 2))


def _study(n, level, solver, walls=False, lab=False):
    """lab: the paper's own frame in the walled box: the inner shell at rest,
    the cavity and the box's walls moving with V (instead of the cavity's
    frame, where the inner shell moves with -V and the walls rest)."""
    p1 = single_shell(n, level)
    s = solver(p1)
    s.solve()
    F1, _ = s.forces()
    s.close()
    R1h = hasimoto.radius3d(abs(F1[0, 0]), 1.0)
    p2 = concentric_shells(n, level, walls=walls)
    if lab:
        p2.U = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    s = solver(p2)
    if lab:
        s.set_wall_velocity([1.0, 0.0, 0.0])
    info = s.solve()
    sol = s.solution()
    s.close()
    R2h = R1h / shells.lambda_from_drag(-sol.F[0, 0], R1h)
    err = shells.flow_errors(sol.u, sol.p, n, p2.h, p2.centres[0], R1h, R2h, frame=0.0 if lab else 1.0)
    return {"n": n, "markers": [int(np.diff(p2.offsets)[0]), int(np.diff(p2.offsets)[1])],
            "R1h_over_R1g": R1h / p2.radius[0], "R2h_over_R2g": R2h / p2.radius[1],
            "v": err["v"], "p": err["p"], "iters": info["iters"], "rel_residual": info["rel_residual"]}


def test_concentric_shells_accuracy_table():
    from paper_1505_07865_amd import ibr

    def solver(prob):
        return ibr.from_problem(prob, rtol=1e-8, restart=100, max_iters=3000, graphs=0)

    rows = []
    for n, level in LEVELS:
        print("concentric shells", n, level, flush=True)
        rows.append(_study(n, level, solver))
        print(json.dumps(rows[-1]), flush=True)
    # parity at 32^3 with the oracle's exact solve
    p1 = single_shell(32, 0)
    R1h = hasimoto.radius3d(abs(constrained.solve_problem(p1).F[0, 0]), 1.0)
    p2 = concentric_shells(32, 0)
    ex = constrained.solve_problem(p2)
    R2h = R1h / shells.lambda_from_drag(-ex.F[0, 0], R1h)
    err = shells.flow_errors(ex.v, ex.p, 32, p2.h, p2.centres[0], R1h, R2h, frame=1.0)
    r0 = rows[0]
    assert abs(r0["R1h_over_R1g"] - R1h / p2.radius[0]) < 1e-6
    assert abs(r0["R2h_over_R2g"] - R2h / p2.radius[1]) < 1e-6
    for nm in ("L1", "L2", "Linf"):
        assert abs(r0["v"][nm] - err["v"][nm]) < 1e-6 * err["v"][nm]
    # convergence under refinement
    for a, b in zip(rows, rows[1:]):
        assert b["R1h_over_R1g"] < a["R1h_over_R1g"]
        assert b["R2h_over_R2g"] > a["R2h_over_R2g"]
        for nm in ("L1", "L2"):
            rate = math.log2(a["v"][nm] / b["v"][nm])
            b["v"]["rate_" + nm] = rate
            assert rate > 0.7, (nm, rate)
    out = results_dir()
    with open(os.path.join(out, "shells_table.json"), "w") as f:
        json.dump(rows, f, indent=1)


def test_concentric_shells_lab_frame_table():
    """Sec. 7.3 as the paper sets it up: the sphere at rest inside the cavity,
    the cavity and the box's walls moving with V (moving-wall data).  Stokes
    flow has no inertia, so this equals the cavity-frame study shifted by V:
    the drag and every error norm agree with it to the solves' tolerance.
    Written to shells_lab_table.json in the results folder."""
    from paper_1505_07865_amd import ibr

    def solver(prob):
        return ibr.from_problem(prob, rtol=1e-8, restart=100, max_iters=3000, graphs=0)

    rows, cav = [], []
    for n, level in LEVELS[:2]:
        print("concentric shells, lab frame", n, level, flush=True)
        rows.append(_study(n, level, solver, walls=True, lab=True))
        cav.append(_study(n, level, solver, walls=True))
        print(json.dumps(rows[-1]), flush=True)
    for a, b in zip(rows, cav):
        assert abs(a["R2h_over_R2g"] - b["R2h_over_R2g"]) < 1e-6
        for nm in ("L1", "L2", "Linf"):
            assert abs(a["v"][nm] - b["v"][nm]) < 1e-5 * b["v"][nm]
    out = results_dir()
    with open(os.path.join(out, "shells_lab_table.json"), "w") as f:
        json.dump(rows, f, indent=1)


def test_concentric_shells_walled_box_table():
    """The same study in the paper's closed box (no-slip walls on every side,
    at rest in the cavity's frame; the inner radius still comes from the
    periodic lattice's drag law, as in the paper).  The cavity isolates its
    interior, so the errors converge as in the periodic box and stay close to
    its numbers; written to shells_box_table.json in the results folder."""
    from paper_1505_07865_amd import ibr

    def solver(prob):
        return ibr.from_problem(prob, rtol=1e-8, restart=100, max_iters=3000, graphs=0)

    rows = []
    for n, level in LEVELS:
        print("concentric shells in the walled box", n, level, flush=True)
        rows.append(_study(n, level, solver, walls=True))
        print(json.dumps(rows[-1]), flush=True)
    for a, b in zip(rows, rows[1:]):
        assert b["R2h_over_R2g"] > a["R2h_over_R2g"]
        for nm in ("L1", "L2"):
            rate = math.log2(a["v"][nm] / b["v"][nm])
            b["v"]["rate_" + nm] = rate
            assert rate > 0.7, (nm, rate)
    out = results_dir()
    with open(os.path.join(out, "shells_box_table.json"), "w") as f:
        json.dump(rows, f, indent=1)
