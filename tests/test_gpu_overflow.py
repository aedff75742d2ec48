"""Neighbour-capacity overflow inside md_step (the boundary's error contract).

A context whose capacity is the longest row of the first list build
overflows at a later rebuild, when the liquid's density fluctuations grow.
md_step then halts the queued steps, grows the capacity, rebuilds the
interrupted step's lists on its state and finishes the call: the run must be
bit for bit the run of a context with enough capacity (FP64 and mixed, fused
direct steps, graph replays with the thermostat, the staged path, and a
batch where one replica overflows while the others keep their lists).
"""
import numpy as np
import pytest

import initconf
from gpu_common import lib_params

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def first_build_max(params_kw, n, L, x, v, t):
    from paper_1105_5613_amd import System
    s = System(lib_params(**params_kw), n, L)
    s.set_state(x, v, t)
    s.build_cells()
    mx = [s.list_stats(r)[1] for r in range(len(n))]
    s.close()
    return mx


def run(params_kw, n, L, x, v, t, calls):
    """calls: list of (nsteps, kwargs) for System.step; returns every output."""
    from paper_1105_5613_amd import System
    s = System(lib_params(**params_kw), n, L)
    s.set_state(x, v, t)
    logs = [s.step(k, **kw) for k, kw in calls]
    xs, vs, img = (a.cpu().numpy() for a in s.get_state())
    F = s.get_forces().cpu().numpy()
    obs = s.observables()
    caps = s.replica_info(0)["max_neighbors"]
    s.close()
    return dict(x=xs, v=vs, img=img, F=F, obs=obs, logs=logs, cap=caps)


def assert_same(a, b):
    for k in ("x", "v", "img", "F"):
        assert np.array_equal(a[k], b[k]), k
    for oa, ob in zip(a["obs"], b["obs"]):
        assert oa == ob
    for la, lb in zip(a["logs"], b["logs"]):
        if la is None:
            assert lb is None
            continue
        for k in la:
            assert np.array_equal(la[k], lb[k]), k


CASES = {
    "fp64-fused": (dict(), [(60, dict(log_every=5)), (41, dict())]),
    "mixed-fused": (dict(precision=1), [(60, dict(log_every=5)), (41, dict())]),
    "fp64-split": (dict(split_kick=1), [(101, dict(log_every=1))]),
    "fp64-graph-thermo": (dict(graph_steps=10),
                          [(65, dict(T0=2.0, T1=1.5, ramp=60, log_every=5)),
                           (36, dict(T0=1.5, log_every=4))]),
    "fp64-staged": (dict(path=2), [(101, dict(log_every=10))]),
}


@pytest.mark.parametrize("case", list(CASES))
def test_overflow_mid_call_matches_uncapped(torch_cuda, case):
    kw, calls = CASES[case]
    say(f"case overflow {case}")
    s = initconf.fcc_system(4000, seed=17, temperature=2.0)
    n, L = [4000], [s["L"]]
    m0 = first_build_max(kw, n, L, s["x"], s["v"], s["type"])[0]
    ref = run(kw, n, L, s["x"], s["v"], s["type"], calls)
    capped = run(dict(kw, max_neighbors=m0), n, L, s["x"], s["v"], s["type"], calls)
    say(f"  first build max {m0}, capacity after the run {capped['cap']} "
        f"(uncapped {ref['cap']}), rebuilds {capped['obs'][0]['n_rebuild']}")
    assert capped["cap"] > m0, "no rebuild overflowed: the case tests nothing"
    assert_same(ref, capped)


def test_overflow_one_replica_of_a_batch(torch_cuda):
    """Three replicas in one context (whole FCC lattices, so the first
    build's rows are all short); the capacity is that build's longest row
    over all of them, so a later rebuild of the hot replica overflows while
    the cold ones keep their lists (moved to the grown layout)."""
    say("case overflow in a batch")
    systems = initconf.batched_systems([4000, 2048, 6912], [2.0, 0.4, 0.4], seed=23)
    x, v, t, n, L = initconf.concat_replicas(systems)
    m0 = max(first_build_max({}, n, L, x, v, t))
    calls = [(80, dict(T0=[2.0, 0.4, 0.4], log_every=8)), (20, dict())]
    ref = run({}, n, L, x, v, t, calls)
    capped = run(dict(max_neighbors=m0), n, L, x, v, t, calls)
    say(f"  capacity {m0} -> {capped['cap']}")
    assert capped["cap"] > m0
    assert_same(ref, capped)
