"""Host logic of bench.py that decides what the timed region contains.

The default line times K steps of the 128^3 workload spread over its
trajectories; each trajectory may hold at most 20 steps (its bodies keep their
gap over those), warm-up included.  The split must time exactly K steps, use
the given seeds first, add the next seeds only when K does not fit, and refuse
impossible requests.
"""
import argparse
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("steps,warmup,seeds", [(54, 2, "0,1,2"), (18, 2, "0,1,2"), (1, 0, "0,1,2"),
                                                (100, 2, "0,1,2"), (5, 2, "0"), (40, 2, "0"), (3, 1, "4,7,9"),
                                                (19, 1, "0")])
def test_split_times_exactly_k_steps(steps, warmup, seeds):
    b = _bench()
    got_seeds, per = b.split_steps(argparse.Namespace(steps=steps, warmup=warmup, seeds=seeds))
    given = [int(x) for x in seeds.split(",")]
    assert sum(per) == steps
    assert len(got_seeds) == len(per) and min(per) >= 1
    assert max(per) + warmup <= b.TRAJECTORY_STEPS
    assert max(per) - min(per) <= 1
    assert len(set(got_seeds)) == len(got_seeds)
    # the given seeds come first; extra trajectories only when K does not fit in them
    assert got_seeds[:min(len(given), len(got_seeds))] == given[:len(got_seeds)]
    if len(got_seeds) > len(given):
        assert len(given) * (b.TRAJECTORY_STEPS - warmup) < steps


def test_split_refuses_impossible(capsys):
    b = _bench()
    for steps, warmup in ((0, 2), (10, 20), (10, 25)):
        with pytest.raises(SystemExit) as e:
            b.split_steps(argparse.Namespace(steps=steps, warmup=warmup, seeds="0,1,2"))
        assert e.value.code == 2
