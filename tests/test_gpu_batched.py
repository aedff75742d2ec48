"""Batched replicas stepped in one context, replica by replica against the
FP64 oracle.

Seven replicas of uneven size (1,000 to 20,000 particles, from 3 to 8 cells
per side) and temperature share one context and advance 30 thermostatted
steps in 10-step hipGraph chunks: per-replica rebuild gating, the
XCD-spread rebuild chain and graph replays across replicas are all on this
path.  Every replica is compared with its own oracle simulation (velocity
Verlet with the isokinetic rescale) on its trajectory -- 30 steps, far
below the horizon where round-off differences grow to the tolerance -- and,
after the run, its cells, lists and forces are rebuilt on the downloaded
state and compared with the oracle's on that state.  The same replicas run
one per context must give the same bits.
"""
import numpy as np
import pytest

import initconf
import oracle
from gpu_common import (canonical, floored_err, lib_params, oracle_cells_lists, oracle_params,
                        pair_abs_sums, tables)

pytestmark = pytest.mark.gpu

SIZES = [1000, 20000, 2500, 7001, 13500, 4321, 1729]
TEMPS = [0.5, 2.0, 1.2, 0.8, 1.6, 0.4, 1.0]
STEPS = 30


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def replicas():
    systems = initconf.batched_systems(SIZES, TEMPS, seed=41)
    return systems, initconf.concat_replicas(systems)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_steps_match_oracle_per_replica(torch_cuda, precision):
    from paper_1105_5613_amd import System
    say(f"case batched stepping vs oracle precision={precision}")
    systems, (x, v, t, n, L) = replicas()
    sysm = System(lib_params(precision=precision, graph_steps=10), n, L)
    sysm.set_state(x, v, t)
    log = sysm.step(STEPS, T0=TEMPS, log_every=1)
    gx, gv, gimg = (a.cpu().numpy() for a in sysm.get_state())
    p = oracle_params()
    off = 0
    patterns = []
    # FP64: round-off only.  Mixed: the FP32 forces (floored error e <= 1e-5,
    # |dF| <= 4e-4 at F_rms ~ 40) move the trajectory by at most dt |dF| per
    # step in v and dt^2 |dF| / 2 per step in x: over 30 steps |dv| <= 6e-5
    # and |dx| <= 5e-6, times 4 for the growth of differences in a liquid;
    # |dE|/N <= F_rms |dx|.  Energies are compared per particle: the total E
    # of a hot replica can be close to zero.
    tx, tv, te = (1e-9, 1e-8, 1e-12) if precision == 0 else (2e-5, 2.4e-4, 8e-4)
    for r, sy in enumerate(systems):
        nr = sy["n"]
        sim = oracle.Sim(p, nr, sy["L"], 0.005)
        sim.set_state(sy["x"], sy["v"], sy["type"])
        ref = sim.step(STEPS, T0=TEMPS[r])
        xo, vo, io = sim.get_state()
        sl = slice(off, off + nr)
        du = np.max(np.abs((gx[sl] + gimg[sl] * sy["L"]) - (xo + io * sy["L"])))
        dv = np.max(np.abs(gv[sl] - vo))
        de = np.max(np.abs(log["E"][:, r] - ref["E"])) / nr
        patterns.append(tuple(np.flatnonzero(ref["rebuilt"])))
        say(f"  replica {r}: n={nr} T={TEMPS[r]} max|du|={du:.2e} max|dv|={dv:.2e} "
            f"max |dE|/N={de:.2e} rebuilds={int(ref['rebuilt'].sum())}")
        assert du < tx and dv < tv and de < te, r
        assert np.allclose(log["T"][:, r], TEMPS[r], rtol=1e-12)
        assert np.array_equal(log["step"][:, r], np.arange(1, STEPS + 1))
        if precision == 0:
            # the skin rule decides the same rebuild steps from the same maxima
            assert np.allclose(log["max_disp"][:, r], np.sqrt(ref["max_disp2"]), rtol=1e-8)
            nb = log["n_rebuild"][:, r]
            steps_rebuilt = np.diff(np.concatenate([[nb[0] - ref["rebuilt"][0]], nb]))
            assert np.array_equal(steps_rebuilt, ref["rebuilt"]), r
        off += nr
    # replicas rebuilt at different steps: the per-replica gating was exercised
    say(f"  rebuild steps per replica: {patterns}")
    assert sum(1 for q in patterns if q) >= 2 and len(set(patterns)) >= 3

    # cells, lists and forces rebuilt on the downloaded state, per replica
    sysm.build_cells()
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    obs = sysm.observables()
    off = 0
    for r, sy in enumerate(systems):
        nr = sy["n"]
        xs = gx[off:off + nr]
        xw, cs, order, count, ids, nc = oracle_cells_lists(p, xs, sy["type"], sy["L"])
        gcs, gorder = sysm.get_cells(r)
        assert sysm.replica_info(r)["nc"] == nc
        assert np.array_equal(gcs, cs) and np.array_equal(gorder, order), r
        gcount, gids = sysm.get_neighbors(r, cap=ids.shape[1])
        assert np.array_equal(gcount, count), r
        assert np.array_equal(canonical(gcount, gids), canonical(count, ids)), r
        Fo, peo, wo = oracle.forces_list(p, xw, sy["type"], sy["L"], count, ids)
        e = floored_err(F[off:off + nr], Fo)
        tol = 1e-12 if precision == 0 else 1e-5
        assert e <= tol, (r, e)
        # energy and virial relative to the magnitude sums of their terms
        eps, sig, rc, _ = tables()
        cpe, cw = pair_abs_sums(eps, sig, rc, sy["type"], xw, sy["L"], count, ids)
        rel = 1e-12 if precision == 0 else 1e-6
        say(f"  replica {r}: e={e:.2e} |dPE|/sum|V*|={abs(obs[r]['pe'] - peo) / cpe:.2e} "
            f"|dW|/sum|rf|={abs(obs[r]['virial'] - wo) / cw:.2e}")
        assert abs(obs[r]["pe"] - peo) <= rel * cpe, r
        assert abs(obs[r]["virial"] - wo) <= rel * cw, r
        off += nr


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_one_context_per_replica(torch_cuda, precision):
    """The batch and the replicas run alone (same graphs and thermostat) give
    the same bits: positions, velocities, image counters and every log.  A
    context of one replica of at most 8,192 particles rebuilds with the
    one-block chain and the 32-lane list build, one of at most 16,384 with
    the latter (13,500 here), the batch with the general kernels: this also
    holds those to the general ones bit for bit."""
    from paper_1105_5613_amd import System
    say(f"case batched vs one context per replica, precision={precision}")
    systems, (x, v, t, n, L) = replicas()
    sysm = System(lib_params(precision=precision, graph_steps=10), n, L)
    sysm.set_state(x, v, t)
    log = sysm.step(STEPS, T0=TEMPS, log_every=3)
    log2 = sysm.step(12, T0=TEMPS, T1=[1.0] * len(SIZES), ramp=10, log_every=4)
    gx, gv, gimg = (a.cpu().numpy() for a in sysm.get_state())
    off = 0
    for r, sy in enumerate(systems):
        nr = sy["n"]
        one = System(lib_params(precision=precision, graph_steps=10), [nr], [sy["L"]])
        one.set_state(sy["x"], sy["v"], sy["type"])
        la = one.step(STEPS, T0=[TEMPS[r]], log_every=3)
        lb = one.step(12, T0=[TEMPS[r]], T1=[1.0], ramp=10, log_every=4)
        ox, ov, oimg = (a.cpu().numpy() for a in one.get_state())
        one.close()
        sl = slice(off, off + nr)
        assert np.array_equal(gx[sl], ox) and np.array_equal(gv[sl], ov), r
        assert np.array_equal(gimg[sl], oimg), r
        for big, small in ((log, la), (log2, lb)):
            for k in big:
                assert np.array_equal(big[k][:, r], small[k][:, 0]), (r, k)
        off += nr


@pytest.mark.parametrize("precision", [0, 1])
def test_nve_drift_1m(torch_cuda, precision):
    """The benchmark box (1,048,576 particles, T = 2 start, dt 0.005): the
    energy drift D over 1,100 NVE steps (slope of E/N after a 100-step
    burn-in, per 1,000 steps) stays below 1e-4 for FP64 and mixed forces."""
    from gpu_common import drift_slope
    from paper_1105_5613_amd import System
    say(f"case 1M drift precision={precision}")
    n = 1048576
    s = initconf.fcc_system(n, seed=2, temperature=2.0)
    sysm = System(lib_params(precision=precision), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    log = sysm.step(1100, log_every=1)
    E = log["E"][:, 0]
    D = drift_slope(E, n)
    tail = (E[100:] - E[100]) / n
    say(f"  D = {D:.3e}, max |E - E(100)|/N = {np.abs(tail).max():.3e}, "
        f"rebuilds = {log['n_rebuild'][-1, 0]}")
    assert D <= 1e-4
    assert log["n_rebuild"][-1, 0] > 100
    sysm.close()
