"""The small-box kernels (the one-block rebuild chain and the 32-lane list
build of a one-box context) against the general kernels, bit for bit, at
the sizes where they switch: 8,192 particles (the chain's limit: every
thread of its block holds its full eight particles), 8,193 (general chain,
small-box list build), 16,384 (the list build's limit) and 16,385 (general
kernels only).  Each box runs NVE steps with several list builds in both
precisions, with md_params.small_box = 0 and = 1, and must give the same
positions, velocities, image counters, energies, cells and lists.  The
general kernels are held to the oracle by the parity tests; this holds the
small-box ones to them."""
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


def run(s, precision, small_box, steps):
    from paper_1105_5613_amd import System
    sysm = System(lib_params(precision=precision, small_box=small_box), [s["n"]], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    log = sysm.step(steps, log_every=5)
    x, v, img = (a.cpu().numpy() for a in sysm.get_state())
    sysm.build_cells()
    cs, order = sysm.get_cells(0)
    count, ids = sysm.get_neighbors(0)
    rebuilds = sysm.observables()[0]["n_rebuild"]
    sysm.close()
    return dict(x=x, v=v, img=img, log=log, cs=cs, order=order, count=count, ids=ids,
                rebuilds=rebuilds)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [8192, 8193, 16384, 16385])
def test_small_box_kernels_match_general(torch_cuda, n, precision):
    say(f"case small-box kernels vs general n={n} precision={precision}")
    s = initconf.fcc_system(n, seed=n % 97, temperature=2.0)
    a = run(s, precision, 0, 40)
    b = run(s, precision, 1, 40)
    say(f"  rebuilds {a['rebuilds']}")
    assert a["rebuilds"] >= 4 and a["rebuilds"] == b["rebuilds"]
    for k in ("x", "v", "img", "cs", "order", "count"):
        assert np.array_equal(a[k], b[k]), k
    # rows in the same order, entry for entry
    assert np.array_equal(a["ids"], b["ids"])
    for k in a["log"]:
        assert np.array_equal(a["log"][k], b["log"][k]), k
