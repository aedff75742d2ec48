"""md_rdf_static, the entry point that allocates nothing, against md_rdf.

Both compute g(r) of one replica from the same pair counts; md_rdf_static
keeps its histogram in a fixed device array shared by every call on the GPU
instead of allocating one.  Two calls in a row, the second with a smaller
input (another replica, fewer bins, a shorter range), and an all-pairs call
must give md_rdf's values bit for bit: nothing of an earlier call may leak
into a later one.
"""
import ctypes as C

import numpy as np
import pytest

import initconf
from gpu_common import lib_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def rdf_static(sysm, rep, rmax, nbins):
    from paper_1105_5613_amd import md
    g = np.full(nbins, np.nan)
    rc = md.lib().md_rdf_static(sysm._h, rep, float(rmax), int(nbins),
                                g.ctypes.data_as(C.POINTER(C.c_double)))
    return rc, g


def test_rdf_static_matches_rdf(torch_cuda):
    from paper_1105_5613_amd import System
    from paper_1105_5613_amd.md import MD_ESTATE
    print("case md_rdf_static vs md_rdf", flush=True)
    systems = initconf.batched_systems([4000, 13500], [2.0, 1.0], seed=51)
    x, v, t, n, L = initconf.concat_replicas(systems)
    sysm = System(lib_params(), n, L)
    sysm.set_state(x, v, t)
    # the cell sweep needs built cells, and this entry point builds nothing
    rc, _ = rdf_static(sysm, 1, 2.4, 100)
    assert rc == MD_ESTATE
    sysm.step(40, T0=[2.0, 1.0])
    calls = [(1, 2.4, 4000),   # cell sweep over the larger replica
             (0, 2.0, 500),    # smaller replica, fewer bins, shorter range
             (0, 6.0, 300)]    # beyond the cell side: every pair of the replica
    for rep, rmax, nbins in calls:
        rc, g = rdf_static(sysm, rep, rmax, nbins)
        assert rc == 0, rc
        ref = sysm.rdf(rep=rep, rmax=rmax, nbins=nbins)
        print(f"  rep {rep} rmax {rmax} bins {nbins}: peak g {g.max():.4f}", flush=True)
        assert np.array_equal(g, ref)
        assert g.sum() > 0
    # bins beyond the limit are refused before any work
    rc, _ = rdf_static(sysm, 0, 2.0, 8193)
    assert rc != 0
    sysm.close()
