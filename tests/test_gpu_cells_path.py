"""GPU parity of the list-free cell path (the paper's grid search, no
neighbour list) against the FP64 oracle, on the same states."""
import numpy as np
import pytest

import initconf
import oracle
from gpu_common import drift_slope, floored_err, lib_params, oracle_params

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def make(n, seed, precision=0, T=2.0):
    from paper_1105_5613_amd import System
    s = initconf.fcc_system(n, seed=seed, temperature=T)
    sysm = System(lib_params(precision=precision, path=3), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    return sysm, s


@pytest.mark.parametrize("n,seed,precision", [(4000, 51, 0), (32000, 52, 0), (4000, 53, 1),
                                              (32000, 54, 1)])
def test_cells_path_forces(torch_cuda, n, seed, precision):
    from paper_1105_5613_amd import MDError
    say(f"case cell path n={n} precision={precision}")
    sysm, s = make(n, seed, precision)
    sysm.step(12)
    x = sysm.get_state()[0].cpu().numpy()
    sysm.build_cells()
    p = oracle_params()
    _, _, _, cs, order, nc = oracle.build_cells(p, x, s["L"])
    gcs, gorder = sysm.get_cells(0)
    assert np.array_equal(gcs, cs) and np.array_equal(gorder, order)
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    Fo, pe_i, w_i = oracle.forces_cells(p, x, s["type"], s["L"])
    e = floored_err(F, Fo)
    say(f"  force error {e:.3e}")
    assert e <= (1e-12 if precision == 0 else 1e-5)
    ob = sysm.observables()[0]
    tol = 1e-12 if precision == 0 else 1e-6
    assert ob["pe"] == pytest.approx(float(pe_i.sum()), rel=tol)
    assert ob["virial"] == pytest.approx(float(w_i.sum()), rel=tol)
    with pytest.raises(MDError) as ex:
        sysm.get_neighbors(0)
    assert ex.value.code == -7


def test_cells_path_trajectory_matches_oracle(torch_cuda):
    say("case cell path trajectory")
    sysm, s = make(4000, 55)
    sim = oracle.Sim(oracle_params(), 4000, s["L"], 0.005)
    sim.set_state(s["x"], s["v"], s["type"])
    log = sysm.step(20, log_every=1)
    ref = sim.step(20)
    x, v, img = (t.cpu().numpy() for t in sysm.get_state())
    xo, vo, imgo = sim.get_state()
    assert np.max(np.abs(x + img * s["L"] - (xo + imgo * s["L"]))) < 1e-9
    assert np.max(np.abs(v - vo)) < 1e-8
    assert np.allclose(log["E"][:, 0], ref["E"], rtol=1e-10)


def test_cells_path_drift(torch_cuda):
    for precision in (0, 1):
        say(f"case cell path drift precision={precision}")
        sysm, s = make(4000, 56, precision)
        log = sysm.step(1100, log_every=1)
        d = drift_slope(log["E"][:, 0], 4000)
        say(f"  drift {d:.2e}")
        assert d <= 1e-4


def test_cells_path_batched(torch_cuda):
    from paper_1105_5613_amd import System
    say("case cell path batched")
    sizes = [1200, 4000, 2700, 9000]
    systems = initconf.batched_systems(sizes, [0.6, 2.0, 1.1, 1.5], seed=57)
    x, v, ty, n, L = initconf.concat_replicas(systems)
    sysm = System(lib_params(path=3), n, L)
    sysm.set_state(x, v, ty)
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    obs = sysm.observables()
    p = oracle_params()
    off = np.cumsum([0] + sizes)
    for r, sy in enumerate(systems):
        Fo, pe_i, _ = oracle.forces_cells(p, sy["x"], sy["type"], sy["L"])
        assert floored_err(F[off[r]:off[r + 1]], Fo) <= 1e-12
        assert obs[r]["pe"] == pytest.approx(float(pe_i.sum()), rel=1e-12)


def test_cells_path_1m_sampled(torch_cuda):
    say("case cell path 1M")
    n = 1048576
    for precision in (0, 1):
        sysm, s = make(n, 2, precision)
        sysm.step(10)
        x = sysm.get_state()[0].cpu().numpy()
        sysm.forces()
        F = sysm.get_forces().cpu().numpy().astype(np.float64)
        sel = np.random.default_rng(1).choice(n, 4096, replace=False)
        Fo, _, _ = oracle.forces_cells(oracle_params(), x, s["type"], s["L"], sel=sel)
        frms = float(np.sqrt(np.mean(np.sum(F ** 2, axis=1))))
        d = np.linalg.norm(F[sel] - Fo, axis=1)
        e = float(np.max(d / np.maximum(np.linalg.norm(Fo, axis=1), frms)))
        say(f"  precision {precision}: sampled force error {e:.3e}")
        assert e <= (1e-12 if precision == 0 else 1e-5)


def test_cells_path_beyond_list_index_range(torch_cuda):
    """The list-free path keeps no neighbour list, so it is not bound by the
    26-bit index of list entries: a 134,217,728-particle (2^27) box, FP64,
    after 3 steps.  Cell arrays bit-exact over the whole box; forces of 4,096
    sampled particles and the energy and virial totals against the oracle's
    cell-list sums over all particles.  The list paths refuse the box."""
    from paper_1105_5613_amd import MDError, System
    n = 1 << 27
    say(f"case cell path n={n}")
    s = initconf.fcc_system(n, seed=61, temperature=2.0)
    say("  inputs generated")
    with pytest.raises(MDError) as ex:
        System(lib_params(path=1), [n], [s["L"]])
    assert ex.value.code == -1
    sysm = System(lib_params(path=3), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    sysm.step(3)
    x = sysm.get_state()[0].cpu().numpy()
    sysm.build_cells()
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    ob = sysm.observables()[0]
    gcs, gorder = sysm.get_cells(0)
    sysm.close()
    del s["v"]
    say("  GPU done")
    p = oracle_params()
    _, _, _, cs, order, nc = oracle.build_cells(p, x, s["L"])
    assert nc == 172
    assert np.array_equal(gcs, cs) and np.array_equal(gorder, order)
    del gcs, gorder, cs, order
    say("  cells bit-exact")
    Fo, pe_i, w_i = oracle.forces_cells(p, x, s["type"], s["L"])
    say("  oracle forces done")
    sel = np.random.default_rng(7).choice(n, 4096, replace=False)
    frms = float(np.sqrt(np.mean(np.sum(F * F, axis=1))))
    d = np.linalg.norm(F[sel] - Fo[sel], axis=1)
    e = float(np.max(d / np.maximum(np.linalg.norm(Fo[sel], axis=1), frms)))
    pe, w = float(np.sum(pe_i)), float(np.sum(w_i))
    say(f"  sampled force error {e:.3e}; pe rel {abs(ob['pe'] - pe) / abs(pe):.2e}, "
        f"virial rel {abs(ob['virial'] - w) / abs(w):.2e}")
    assert e <= 1e-12
    assert ob["pe"] == pytest.approx(pe, rel=1e-12)
    assert ob["virial"] == pytest.approx(w, rel=1e-12)
