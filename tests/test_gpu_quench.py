"""Quench ensembles (glass-transition section, batched + mixed form):
statistical parity of the caloric curve and MSD between the FP64 and mixed
GPU forms and the FP64 oracle on a replica subset, and NVE energy drift of
the quenched replicas.  Trajectories themselves are chaotic and are not
compared beyond the first log point."""
import numpy as np
import pytest

import initconf
import oracle
from gpu_common import drift_slope, oracle_params

pytestmark = pytest.mark.gpu

NREP, N = 8, 4000
EQUIL, QUENCH, EVERY, NVE = 1000, 6000, 500, 1100
T_HOT, T_COLD = 2.0, 0.3


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def runs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1105_5613_amd.quench import run_quench
    out = {}
    for prec in (0, 1):
        say(f"case quench ensemble precision={prec}")
        out[prec] = run_quench(NREP, N, seed=11, precision=prec, T_hot=T_HOT, T_cold=T_COLD,
                               equil=EQUIL, quench=QUENCH, log_every=EVERY, nve=NVE)
    return out


def oracle_quench(system):
    sim = oracle.Sim(oracle_params(), N, system["L"], 0.005)
    sim.set_state(system["x"], system["v"], system["type"])
    sim.step(EQUIL, T0=T_HOT)
    x0, _, img0 = sim.get_state()
    u0 = x0 + img0 * system["L"]
    pe, msd = [], []
    for k in range(0, QUENCH, EVERY):
        ta = T_HOT + (T_COLD - T_HOT) * k / QUENCH
        tb = T_HOT + (T_COLD - T_HOT) * (k + EVERY) / QUENCH
        o = sim.step(EVERY, T0=ta, T1=tb, ramp=EVERY)
        pe.append(o["pe"][-1] / N)
        x, _, img = sim.get_state()
        msd.append(float(np.mean(np.sum((x + img * system["L"] - u0) ** 2, axis=1))))
    e = sim.step(NVE)["E"]
    return np.array(pe), np.array(msd), e


def test_quench_statistical_parity(runs):
    pe64 = np.asarray(runs[0]["pe_per_particle"])   # [nlog][nrep]
    pe32 = np.asarray(runs[1]["pe_per_particle"])
    assert pe64.shape == (QUENCH // EVERY, NREP)
    assert np.allclose(runs[0]["T_target"], T_HOT + (T_COLD - T_HOT) *
                       np.arange(1, QUENCH // EVERY + 1) / (QUENCH // EVERY))
    # the rescale thermostat holds every replica at the target
    assert np.allclose(np.asarray(runs[1]["T"]), np.asarray(runs[1]["T_target"])[:, None],
                       rtol=1e-12)
    se = np.sqrt(pe64.var(axis=1, ddof=1) / NREP + pe32.var(axis=1, ddof=1) / NREP)
    dev = np.abs(pe64.mean(axis=1) - pe32.mean(axis=1))
    say(f"  max |<PE/N>_fp64 - <PE/N>_mixed| / SE = {np.max(dev / se):.2f}")
    assert np.all(dev <= 4.0 * se + 1e-4)
    # the caloric curve falls as the ensemble cools
    assert pe64.mean(axis=1)[-1] < pe64.mean(axis=1)[0] - 1.0
    # the oracle on two replicas of the same ensemble
    systems = initconf.batched_systems([N] * NREP, [T_HOT] * NREP, seed=11)
    spread = np.sqrt(pe64.var(axis=1, ddof=1))
    for r in range(2):
        pe_o, msd_o, e_o = oracle_quench(systems[r])
        z = np.abs(pe_o - pe64.mean(axis=1)) / np.sqrt(spread ** 2 + spread ** 2 / NREP)
        say(f"  oracle replica {r}: max z = {np.max(z):.2f}")
        assert np.all(z <= 4.0)
        m64 = np.asarray(runs[0]["msd"])[-1]
        assert abs(msd_o[-1] - m64.mean()) <= 4.0 * m64.std(ddof=1) + 1e-3
        d = drift_slope(e_o, N)
        say(f"  oracle replica {r}: NVE drift {d:.2e}")
        assert d <= 1e-4


def test_quench_msd_and_drift(runs):
    for prec in (0, 1):
        msd = np.asarray(runs[prec]["msd"])
        # MSD from the start of the quench grows, and slows as the ensemble cools
        assert np.all(np.diff(msd.mean(axis=1)) > 0)
        growth = np.diff(msd.mean(axis=1))
        assert growth[-1] < growth[0]
        E = np.asarray(runs[prec]["nve_E_per_particle"])  # [NVE][nrep], already per particle
        for r in range(NREP):
            d = drift_slope(E[:, r] * N, N)
            assert d <= 1e-4, (prec, r, d)
        say(f"  precision {prec}: max NVE drift "
            f"{max(drift_slope(E[:, r] * N, N) for r in range(NREP)):.2e}")
