"""GPU: glass-study observables (MSD, g(r)) and the autotuners, against the
FP64 oracle on the same states."""
import numpy as np
import pytest

import initconf
import oracle
from gpu_common import floored_err, lib_params, oracle_params

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _counts(g, n, L, rmax, nbins):
    dr = rmax / nbins
    r0 = np.arange(nbins) * dr
    shell = 4.0 / 3.0 * np.pi * ((r0 + dr) ** 3 - r0 ** 3)
    return np.round(g * n * n * shell / (2.0 * L ** 3)).astype(np.int64)


@pytest.mark.parametrize("n,seed,nbins", [(4000, 21, 300), (13500, 22, 1000), (700, 23, 7)])
def test_rdf_matches_oracle(torch_cuda, n, seed, nbins):
    """Pair counts per bin bit-exact; g within rounding of the normalisation."""
    from paper_1105_5613_amd import System
    say(f"case rdf n={n} seed={seed} nbins={nbins}")
    s = initconf.fcc_system(n, seed=seed, jitter=0.2)
    sysm = System(lib_params(), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    rmax = 0.5 * s["L"]
    g = sysm.rdf(0, rmax, nbins)
    go = oracle.rdf(s["x"], s["L"], rmax, nbins)
    assert np.array_equal(_counts(g, n, s["L"], rmax, nbins),
                          _counts(go, n, s["L"], rmax, nbins))
    np.testing.assert_allclose(g, go, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,seed,rmax,steps", [(32000, 24, 2.5, 0), (20000, 25, 2.45, 30)])
def test_rdf_cells_matches_oracle(torch_cuda, n, seed, rmax, steps):
    """rmax below the cell side minus the skin: pairs from the cell grid,
    also on a stepped state between list builds; counts bit-exact."""
    from paper_1105_5613_amd import System
    say(f"case rdf by cells n={n}")
    # a jittered lattice for a static state; a liquid reached by stepping otherwise
    s = initconf.fcc_system(n, seed=seed, jitter=0.05 if steps else 0.2)
    sysm = System(lib_params(), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    if steps:
        sysm.step(steps)
    info = sysm.replica_info(0)
    assert rmax <= s["L"] / info["nc"] - 0.3
    x = sysm.get_state()[0].cpu().numpy()
    g = sysm.rdf(0, rmax, 250)
    go = oracle.rdf(x, s["L"], rmax, 250)
    assert np.array_equal(_counts(g, n, s["L"], rmax, 250), _counts(go, n, s["L"], rmax, 250))
    np.testing.assert_allclose(g, go, rtol=1e-13, atol=0)


def test_rdf_batched_replica(torch_cuda):
    from paper_1105_5613_amd import System
    say("case rdf batched")
    sizes = [1500, 4000, 2048]
    systems = initconf.batched_systems(sizes, [1.0, 1.5, 0.6], seed=31)
    x, v, ty, n, L = initconf.concat_replicas(systems)
    sysm = System(lib_params(), n, L)
    sysm.set_state(x, v, ty)
    for r, sy in enumerate(systems):
        for rmax in (0.45 * sy["L"], 2.0):  # all pairs, then the cell sweep
            g = sysm.rdf(r, rmax, 200)
            go = oracle.rdf(sy["x"], sy["L"], rmax, 200)
            np.testing.assert_allclose(g, go, rtol=1e-13, atol=0)


def test_rdf_rejects_bad_arguments(torch_cuda):
    from paper_1105_5613_amd import MDError, System
    s = initconf.fcc_system(500, seed=2)
    sysm = System(lib_params(), [500], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    for args in [(1, 2.0, 10), (0, 0.6 * s["L"], 10), (0, 2.0, 0), (0, 2.0, 9000),
                 (0, -1.0, 10)]:
        with pytest.raises(MDError):
            sysm.rdf(*args)


def test_msd_matches_oracle_trajectory(torch_cuda):
    """MSD of 40 FP64 steps (across rebuilds and wraps) against the oracle's
    unwrapped positions."""
    from paper_1105_5613_amd import MDError, System
    say("case msd")
    n = 4000
    s = initconf.fcc_system(n, seed=24, temperature=2.0)
    sysm = System(lib_params(), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    with pytest.raises(MDError):
        sysm.msd()
    sysm.msd_reference()
    assert sysm.msd()[0] == 0.0
    sim = oracle.Sim(oracle_params(), n, s["L"], 0.005)
    sim.set_state(s["x"], s["v"], s["type"])
    sysm.step(40)
    sim.step(40)
    xo, _, imgo = sim.get_state()
    msd_o = np.mean(np.sum((xo + imgo * s["L"] - s["x"]) ** 2, axis=1))
    msd = sysm.msd()[0]
    assert sysm.replica_info(0)["n"] == n
    assert msd == pytest.approx(msd_o, rel=1e-7)
    # the GPU's own state: MSD is the plain mean over its unwrapped positions
    x, _, img = sysm.get_state()
    u = x.cpu().numpy() + img.cpu().numpy() * s["L"]
    assert msd == pytest.approx(np.mean(np.sum((u - s["x"]) ** 2, axis=1)), rel=1e-13)


def test_msd_batched_resets_reference(torch_cuda):
    from paper_1105_5613_amd import System
    say("case msd batched")
    sizes = [1000, 3000]
    systems = initconf.batched_systems(sizes, [0.8, 1.6], seed=32)
    xc, vc, ty, n, L = initconf.concat_replicas(systems)
    sysm = System(lib_params(precision=1), n, L)
    sysm.set_state(xc, vc, ty)
    sysm.msd_reference()
    sysm.step(30)
    x0, _, i0 = (t.cpu().numpy() for t in sysm.get_state())
    m30 = sysm.msd()
    sysm.msd_reference()
    sysm.step(20)
    x1, _, i1 = (t.cpu().numpy() for t in sysm.get_state())
    m = sysm.msd()
    Ls = np.repeat(L, sizes)[:, None]
    u0, u1 = x0 + i0 * Ls, x1 + i1 * Ls
    uc = xc
    off = np.cumsum([0] + sizes)
    for r in range(2):
        sl = slice(off[r], off[r + 1])
        assert m30[r] == pytest.approx(np.mean(np.sum((u0[sl] - uc[sl]) ** 2, axis=1)), rel=1e-12)
        assert m[r] == pytest.approx(np.mean(np.sum((u1[sl] - u0[sl]) ** 2, axis=1)), rel=1e-12)
    assert np.all(m30 > 0) and np.all(m > 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_md_autotune_keeps_parity(torch_cuda, precision):
    """The in-context tuner only picks a kernel variant: forces stay within
    the parity bar afterwards, and stepping continues."""
    from paper_1105_5613_amd import System
    say(f"case md_autotune precision={precision}")
    n = 32000
    s = initconf.fcc_system(n, seed=25)
    sysm = System(lib_params(precision=precision), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    sysm.step(5)
    t = sysm.autotune(reps=2)
    assert len(t["tried"]) >= 2 and t["force_ms"] > 0
    assert (t["tpp"], t["unroll"]) in [(a, b) for a, b, _ in t["tried"]]
    assert t["force_ms"] == min(ms for _, _, ms in t["tried"])
    sysm.build_cells()
    sysm.forces()
    x, v, _ = sysm.get_state()
    F = sysm.get_forces().cpu().numpy()
    Fo, peo, _ = oracle.forces_brute(oracle_params(), x.cpu().numpy(), s["type"], s["L"])
    assert floored_err(F, Fo) <= (1e-12 if precision == 0 else 1e-5)
    sysm.step(20)


def test_tune_module_picks_valid_choice(torch_cuda, tmp_path):
    """The path/skin tuner returns one of its candidates, caches it, and the
    tuned parameters give forces within the parity bar."""
    from paper_1105_5613_amd import System, tune
    say("case tune.autotune")
    n = 32000
    s = initconf.fcc_system(n, seed=26)
    cache = str(tmp_path / "tune.json")
    p0 = lib_params(precision=1)
    p, rep = tune.autotune(p0, n, s["L"], s["x"], s["v"], s["type"], steps=20, warmup=5,
                           skins=(0.3, 0.45), cache_path=cache)
    assert not rep["cached"] and len(rep["trials"]) >= 4
    ch = rep["choice"]
    assert ch["path"] in (1, 2) and ch["skin"] in (0.3, 0.45)
    assert (p.path, p.skin, p.tpp, p.unroll) == (ch["path"], ch["skin"], ch["tpp"], ch["unroll"])
    p2, rep2 = tune.autotune(p0, n, s["L"], s["x"], s["v"], s["type"], cache_path=cache)
    assert rep2["cached"] and (p2.path, p2.skin, p2.tpp) == (p.path, p.skin, p.tpp)
    sysm = System(p, [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    sysm.build_cells()
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    Fo, _, _ = oracle.forces_brute(oracle_params(skin=ch["skin"]), s["x"], s["type"], s["L"])
    assert floored_err(F, Fo) <= 1e-5
