"""Pins of the oracle's velocity-Verlet integration, skin rule and thermostat.

Velocity Verlet (section "Parallel force calculation") is time reversible,
conserves total momentum exactly when the forces obey Newton's third law,
and its energy error scales as dt^2.  The isokinetic rescale used for the
canonical runs ("BBMD scaling results" section) sets the instantaneous
temperature to the target.  None of these properties is computed by the
oracle; each is an independent mathematical fact it must satisfy.
"""
import numpy as np
import pytest

import initconf


def make(o, n, seed, T=1.0, skin=0.3, dt=0.005, brute=False):
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=skin)
    s = initconf.fcc_system(n, seed=seed, temperature=T)
    sim = o.Sim(p, n, s["L"], dt, brute=brute)
    sim.set_state(s["x"], s["v"], s["type"])
    return sim, s


def unwrapped(sim):
    x, v, img = sim.get_state()
    return x + img * sim.L, v


@pytest.mark.parametrize("brute", [True, False])
def test_time_reversibility(oracle_lib, brute):
    sim, s = make(oracle_lib, 500, 41, T=1.0, brute=brute)
    x0, v0 = unwrapped(sim)
    sim.step(50)
    x, v, img = sim.get_state()
    # reverse: set v -> -v and integrate forward again
    sim2 = oracle_lib.Sim(sim.p, sim.n, sim.L, sim.dt, brute=brute)
    sim2.set_state(x + img * sim.L, -v, s["type"])
    sim2.step(50)
    x1, v1 = unwrapped(sim2)
    assert np.max(np.abs(x1 - x0)) <= 1e-9
    assert np.max(np.abs(v1 + v0)) <= 1e-9


def test_momentum_conservation(oracle_lib):
    sim, s = make(oracle_lib, 500, 42, T=2.0)
    _, v0 = unwrapped(sim)
    F0, _, _ = sim.forces()
    out = sim.step(40)
    _, v1 = unwrapped(sim)
    p0, p1 = v0.sum(axis=0), v1.sum(axis=0)
    assert np.max(np.abs(p1 - p0)) <= 1e-12 * np.sum(np.abs(F0)) * sim.dt * 40


def test_energy_error_scales_as_dt2(oracle_lib):
    res = []
    for dt, steps in [(0.004, 100), (0.002, 200)]:
        sim, _ = make(oracle_lib, 500, 43, T=1.0, dt=dt)
        _, pe0, _ = sim.forces()
        x, v, img = sim.get_state()
        e0 = 0.5 * np.sum(v * v) + pe0
        out = sim.step(steps)
        res.append(np.max(np.abs(out["E"] - e0)))
    ratio = res[0] / res[1]
    assert 2.8 < ratio < 5.5, ratio


def drift_slope(E, n, burn=100):
    """|least-squares slope of E/N| x 1000 steps over steps burn..end."""
    e = np.asarray(E)[burn:] / n
    k = np.arange(len(e), dtype=np.float64)
    slope = np.polyfit(k, e, 1)[0]
    return abs(slope) * 1000.0


@pytest.mark.slow
def test_nve_drift_4000(oracle_lib):
    """The 4,000-particle FP64 NVE run: steady-state drift below 1e-4 per particle."""
    sim, s = make(oracle_lib, 4000, 1, T=2.0)
    out = sim.step(1100)
    assert drift_slope(out["E"], 4000) <= 1e-4
    assert sim.rebuilds() > 10


def test_brute_and_list_modes_agree(oracle_lib):
    a, _ = make(oracle_lib, 500, 44, T=2.0, brute=True)
    b, _ = make(oracle_lib, 500, 44, T=2.0, brute=False)
    oa = a.step(20)
    ob = b.step(20)
    xa, va = unwrapped(a)
    xb, vb = unwrapped(b)
    assert np.max(np.abs(xa - xb)) < 1e-10
    assert np.allclose(oa["E"], ob["E"], rtol=1e-11)


def test_skin_rule(oracle_lib):
    sim, _ = make(oracle_lib, 500, 45, T=2.0, skin=0.3)
    out = sim.step(60)
    h2 = 0.15 ** 2
    md2, rb = out["max_disp2"], out["rebuilt"]
    assert np.all(md2[rb == 1] > h2)
    assert np.all(md2[rb == 0] <= h2)
    assert rb.sum() >= 3
    # skin = 0: a rebuild every step
    sim0, _ = make(oracle_lib, 500, 45, T=2.0, skin=0.0)
    out0 = sim0.step(5)
    assert np.all(out0["rebuilt"] == 1)


def test_thermostat_sets_temperature(oracle_lib):
    sim, _ = make(oracle_lib, 500, 46, T=2.0)
    out = sim.step(30, T0=0.8)
    assert np.allclose(out["T"], 0.8, rtol=1e-14)
    _, v = unwrapped(sim)
    T = np.sum(v * v) / (3 * 500 - 3)
    assert T == pytest.approx(0.8, rel=1e-14)
    # linear ramp
    out = sim.step(40, T0=0.8, T1=0.4, ramp=20)
    expect = 0.8 + (0.4 - 0.8) * np.minimum(np.arange(1, 41) / 20, 1.0)
    assert np.allclose(out["T"], expect, rtol=1e-13)


def test_observable_definitions(oracle_lib):
    sim, s = make(oracle_lib, 500, 47, T=1.5)
    out = sim.step(3)
    x, v, img = sim.get_state()
    F, pe, w = sim.forces()
    ke = 0.5 * np.sum(v * v)
    assert out["ke"][-1] == pytest.approx(ke, rel=1e-14)
    assert out["pe"][-1] == pytest.approx(pe, rel=1e-14)
    assert out["E"][-1] == pytest.approx(ke + pe, rel=1e-14)
    V = sim.L ** 3
    assert out["P"][-1] == pytest.approx((2 * ke + w) / (3 * V), rel=1e-14)


def test_thread_count_does_not_change_results(oracle_lib):
    """Every parallel loop of the oracle writes disjoint rows: one thread and
    all threads give the same bits (forces, a short run with rebuilds)."""
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=0.3)
    outs = []
    nmax = o.max_threads()
    try:
        for nt in (1, max(nmax, 2)):
            o.set_threads(nt)
            sim, s = make(o, 4000, 3, T=2.0)
            F, pe, w = o.forces_cells(p, s["x"], s["type"], s["L"])
            sim.step(20)
            x, v, img = sim.get_state()
            outs.append((F, pe, w, x, v, img))
    finally:
        o.set_threads(nmax)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
