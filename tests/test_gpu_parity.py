"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: cell arrays and neighbour lists bit-exact (canonical sorted sets);
FP64 forces within e = max_i |dF_i| / max(|F_i|, F_rms) <= 1e-12 and
energies/virial within 1e-12 relative; mixed precision e <= 1e-5 and
energy/virial <= 1e-6 relative.  Every comparison is on the same state
(downloaded from the GPU when the GPU has been stepping): trajectories of two
chaotic integrations are never compared beyond a few steps.
"""
import math

import numpy as np
import pytest

import initconf
import oracle
from gpu_common import (SKIN, canonical, drift_slope, floored_err, force_error_report,
                        lib_params, oracle_cells_lists, oracle_params, pair_force_sums, tables)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def make_system(torch_cuda, n, seed, precision=0, T=2.0, **kw):
    from paper_1105_5613_amd import System
    s = initconf.fcc_system(n, seed=seed, temperature=T)
    sysm = System(lib_params(precision=precision, **kw), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    return sysm, s


def compare_cells_lists(sysm, p, x, types, L, rep=0, tag=""):
    xw, cs, order, count, ids, nc = oracle_cells_lists(p, x, types, L)
    gcs, gorder = sysm.get_cells(rep)
    assert sysm.replica_info(rep)["nc"] == nc
    assert np.array_equal(gcs, cs), f"{tag}: cell_start differs"
    assert np.array_equal(gorder, order), f"{tag}: cell order differs"
    gcount, gids = sysm.get_neighbors(rep, cap=ids.shape[1])
    assert np.array_equal(gcount, count), f"{tag}: neighbour counts differ"
    assert np.array_equal(canonical(gcount, gids), canonical(count, ids)), f"{tag}: lists differ"
    return xw, count, ids


PATHS = {"gather": dict(path=1), "staged": dict(path=2)}


@pytest.mark.parametrize("n,seed,kw", [
    (4000, 1, PATHS["gather"]), (4000, 1, PATHS["staged"]),
    (32000, 7, PATHS["gather"]), (32000, 7, PATHS["staged"]),
    (500, 3, {}),
    (32000, 8, dict(path=2, tile_cells=1)),                  # one home cell per tile
    (32000, 9, dict(path=2, tile_cells=64)),                 # whole rows: both wrap pieces
    (32000, 10, dict(path=2, stage_slots=256)),              # most slots from global memory
    (13500, 11, dict(path=2, tpp=1, unroll=8)),
], ids=["4k-gather", "4k-staged", "32k-gather", "32k-staged", "500-onecell", "32k-cell1",
        "32k-row", "32k-slots256", "13.5k-bt128"])
def test_cells_lists_forces_fp64(torch_cuda, n, seed, kw):
    say(f"case cells/lists/forces fp64 n={n} seed={seed} {kw}")
    sysm, s = make_system(torch_cuda, n, seed, **kw)
    p = oracle_params()
    sysm.build_cells()
    xw, count, ids = compare_cells_lists(sysm, p, s["x"], s["type"], s["L"], tag=f"n={n}")
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    Fo, peo, wo = oracle.forces_list(p, xw, s["type"], s["L"], count, ids)
    e = floored_err(F, Fo)
    say(f"  force error {e:.3e}")
    assert e <= 1e-12
    ob = sysm.observables()[0]
    assert ob["pe"] == pytest.approx(peo, rel=1e-12)
    assert ob["virial"] == pytest.approx(wo, rel=1e-12)
    ke = 0.5 * np.sum(s["v"] ** 2)
    assert ob["ke"] == pytest.approx(ke, rel=1e-12)
    V = s["L"] ** 3
    assert ob["P"] == pytest.approx((2 * ke + wo) / (3 * V), rel=1e-12)
    assert ob["n_rebuild"] == 1


@pytest.mark.parametrize("precision,small_box", [(0, 1), (1, 1), (0, 0), (1, 0)])
def test_dense_cells_groups_and_passes(torch_cuda, precision, small_box):
    """One cutoff of 3.0 for every pair in a 2,048-particle box: 3 cells per
    side of ~4.0, ~76 particles per cell, so the general list build takes
    each cell's home particles in three groups, and the 27-cell neighbourhood
    is the whole box (2,048 candidates: three passes of chunks, the later
    ones starting at each home's running count); the small-box kernels
    (small_box = 0) sort cells of more than 64 particles and walk 76-particle
    stencil cells per lane.  Lists bit-exact (canonical), forces within the
    bar, before and after steps."""
    from paper_1105_5613_amd import System, make_params
    say(f"case dense cells precision={precision} small_box={small_box}")
    eps, sig, rc, mass = initconf.mixture_tables(global_rc=3.0)
    s = initconf.fcc_system(2048, seed=31, temperature=1.5)
    sysm = System(make_params(eps, sig, rc, mass, skin=SKIN, dt=0.005, precision=precision,
                              small_box=small_box), [2048], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    po = oracle.make_params(eps, sig, rc, mass, skin=SKIN)
    for k in range(2):
        if k:
            sysm.step(12)
        x = sysm.get_state()[0].cpu().numpy()
        sysm.build_cells()
        assert sysm.replica_info(0)["nc"] == 3
        xw, _, cell, cs, order, nc = oracle.build_cells(po, x, s["L"])
        assert int(np.max(np.diff(cs))) > 64, "no cell holds three groups"
        count, ids = oracle.build_nlist(po, xw, s["type"], s["L"], cell, cs, order, nc)
        gcount, gids = sysm.get_neighbors(0, cap=ids.shape[1])
        assert np.array_equal(gcount, count)
        assert np.array_equal(canonical(gcount, gids), canonical(count, ids))
        sysm.forces()
        F = sysm.get_forces().cpu().numpy()
        Fo, _, _ = oracle.forces_list(po, xw, s["type"], s["L"], count, ids)
        e = floored_err(F, Fo)
        say(f"  after {12 * k} steps: max per cell {int(np.max(np.diff(cs)))}, force error {e:.3e}")
        assert e <= (1e-12 if precision == 0 else 1e-5)
    sysm.close()


def boundary_state(seed):
    """4,000-particle FCC state whose lattice planes coincide with the cell
    faces (cell side = 2 lattice constants): every coordinate within 0.05 of a
    face is snapped exactly onto it, and a few are set to the wrap cases of the
    one-wrap rule: 0.0, -0.0, a tiny negative value (x + L rounds to L, which
    the rule maps to 0), L itself, the largest double below L, and a value
    just past L."""
    s = initconf.fcc_system(4000, seed=seed, temperature=2.0)
    L = s["L"]
    x = s["x"].copy()
    p = oracle_params()
    nc, _ = oracle.cell_grid(p, L)
    side = L / nc
    k = np.rint(x / side)
    near = np.abs(x - k * side) < 0.05
    x[near] = (k * side)[near]
    rng = np.random.default_rng(seed)
    zero_plane = np.argwhere(near & (k % nc == 0))
    pick = zero_plane[rng.choice(len(zero_plane), 6, replace=False)]
    specials = [0.0, -0.0, -1e-17, L, np.nextafter(L, 0.0), L + 1e-14]
    for (i, d), v in zip(pick, specials):
        x[i, d] = v
    return s, x, int(near.sum())


@pytest.mark.parametrize("precision,path,small_box", [(0, 1, 0), (0, 1, 1), (0, 2, 0), (1, 1, 0),
                                                       (1, 1, 1), (0, 3, 0)])
def test_cell_faces_and_wrap_cases(torch_cuda, precision, path, small_box):
    """Particles exactly on cell faces and at the wrap edge cases: wrapped
    positions, image counters, cell arrays and lists bit-exact, forces within
    the bar (small_box = 1: the general kernels at this size)."""
    from paper_1105_5613_amd import System
    s, x, nsnap = boundary_state(31)
    say(f"case cell faces precision={precision} path={path} small_box={small_box}: "
        f"{nsnap} coordinates on faces")
    sysm = System(lib_params(precision=precision, path=path, small_box=small_box), [4000],
                  [s["L"]])
    sysm.set_state(x, s["v"], s["type"])
    sysm.build_cells()
    p = oracle_params()
    xw, img, _, cs, order, nc = oracle.build_cells(p, x, s["L"])
    gx, _, gimg = sysm.get_state()
    assert np.array_equal(gx.cpu().numpy(), xw), "wrapped positions differ"
    assert np.array_equal(gimg.cpu().numpy(), img), "image counters differ"
    gcs, gorder = sysm.get_cells(0)
    assert np.array_equal(gcs, cs) and np.array_equal(gorder, order)
    if path != 3:
        compare_cells_lists(sysm, p, x, s["type"], s["L"], tag="faces")
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    Fo, _, _ = oracle.forces_cells(p, xw, s["type"], s["L"])
    e = floored_err(F, Fo)
    say(f"  force error {e:.3e}")
    assert e <= (1e-12 if precision == 0 else 1e-5)


def threshold_pairs():
    """Isolated pairs at the list threshold of their species pair: along x at
    d = sqrt(thr) + k ulp (k = -3..3; the difference of the two coordinates is
    exact, so r^2 = round(d d) lands below, on and above thr), and along random
    directions at (1 + k 1e-16) sqrt(thr).  Pairs sit 8 sigma apart in a
    40-sigma box, so no other particle is within the threshold."""
    eps, sig, rc, mass = tables()
    L = 40.0
    xs, ts = [], []
    slots = [(a, b, c) for a in range(5) for b in range(5) for c in range(5)]
    rng = np.random.default_rng(12)
    q = 0
    for ta, tb in ((0, 0), (0, 1), (1, 1)):
        t = (rc[ta][tb] + SKIN) * (rc[ta][tb] + SKIN)
        d0 = math.sqrt(t)
        for k in range(-3, 4):
            d = d0
            for _ in range(abs(k)):
                d = np.nextafter(d, np.inf if k > 0 else -np.inf)
            o = 8.0 * np.array(slots[q], dtype=np.float64) + 1.0
            q += 1
            xs += [o, o + np.array([d, 0.0, 0.0])]
            ts += [ta, tb]
        for k in range(-3, 4):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            o = 8.0 * np.array(slots[q], dtype=np.float64) + 1.0
            q += 1
            xs += [o, o + u * d0 * (1.0 + k * 1e-16)]
            ts += [ta, tb]
    return np.array(xs), np.array(ts, dtype=np.int32), L


@pytest.mark.parametrize("precision,path,small_box", [(0, 1, 0), (0, 1, 1), (0, 2, 0), (1, 1, 0),
                                                       (1, 1, 1)])
def test_list_threshold_ties(torch_cuda, precision, path, small_box):
    """Pairs at r^2 just below, equal to and just above (r_c,ab + skin)^2: the
    strict inclusion test gives bit-identical lists to the oracle's, in the
    small-box search (which reads the threshold table) and in the general one
    (which forms the threshold from the home species, small_box = 1)."""
    from paper_1105_5613_amd import System
    x, types, L = threshold_pairs()
    n = len(x)
    say(f"case threshold ties precision={precision} path={path} small_box={small_box}: "
        f"{n // 2} pairs")
    sysm = System(lib_params(precision=precision, path=path, small_box=small_box), [n], [L])
    sysm.set_state(x, np.zeros_like(x), types)
    sysm.build_cells()
    p = oracle_params()
    _, count, _ = compare_cells_lists(sysm, p, x, types, L, tag="threshold ties")
    say(f"  pairs listed: {int(count.sum()) // 2} of {n // 2}")
    assert 0 < count.sum() < n  # some pairs in, some out


def test_dilute_box_cells_after_steps(torch_cuda):
    """512 particles on a jittered lattice in a 60-sigma box: 9,261 cells,
    more than the threads of the kick kernel, so the cell histogram is cleared
    by its own launch.  Cells and lists bit-exact after several rebuilds."""
    from paper_1105_5613_amd import System
    say("case dilute box")
    n, L = 512, 60.0
    g = (np.arange(8) + 0.5) * (L / 8)
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    rng = np.random.default_rng(14)
    x = x + rng.uniform(-1.0, 1.0, x.shape)
    v = rng.normal(0.0, math.sqrt(2.0), x.shape)
    v -= v.mean(axis=0)
    types = (rng.random(n) < 0.2).astype(np.int32)
    sysm = System(lib_params(), [n], [L])
    sysm.set_state(x, v, types)
    assert sysm.replica_info(0)["nc"] == 21
    sysm.step(200)
    assert sysm.observables()[0]["n_rebuild"] >= 3
    xs = sysm.get_state()[0].cpu().numpy()
    sysm.build_cells()
    compare_cells_lists(sysm, oracle_params(), xs, types, L, tag="dilute")


# Species tables beyond the binary mixture.  The list test forms the pair
# threshold either as one FMA over the home species value (one species, or two
# whose thresholds for each partner species lie within a factor of two) or by
# a select chain: "one" takes the first form, "two-wide" and "three" the second.
# At 13,500 particles a one-box context searches with the small-box kernel,
# which reads the threshold table directly; small_box = 1 runs the general one.
SPECIES_TABLES = {
    "one": ([[1.0]], [[1.0]], [[2.5]], [1.0]),
    "two-wide": ([[1.0, 1.5], [1.5, 0.5]], [[1.0, 0.7], [0.7, 0.4]],
                 [[2.5, 1.75], [1.75, 1.0]], [1.0, 0.5]),
    "three": ([[1.0, 1.2, 0.8], [1.2, 0.6, 1.0], [0.8, 1.0, 0.9]],
              [[1.0, 0.9, 0.8], [0.9, 0.85, 0.75], [0.8, 0.75, 0.7]],
              [[2.5, 2.25, 2.0], [2.25, 2.125, 1.875], [2.0, 1.875, 1.75]], [1.0, 0.9, 0.8]),
}


@pytest.mark.parametrize("name,precision,path,small_box", [
    ("one", 0, 1, 0), ("one", 0, 1, 1), ("two-wide", 0, 1, 0), ("two-wide", 0, 1, 1),
    ("two-wide", 0, 2, 0), ("three", 0, 1, 0), ("three", 0, 1, 1), ("three", 0, 2, 0),
    ("three", 1, 1, 0), ("three", 1, 1, 1)])
def test_species_tables(torch_cuda, name, precision, path, small_box):
    from paper_1105_5613_amd import System, make_params
    say(f"case species table {name} precision={precision} path={path} small_box={small_box}")
    eps, sig, rc, mass = SPECIES_TABLES[name]
    n = 13500
    s = initconf.fcc_system(n, seed=21, temperature=1.0)
    nt = len(eps)
    types = np.random.default_rng(22).integers(0, nt, n).astype(np.int32) if nt != 2 \
        else s["type"]
    sysm = System(make_params(eps, sig, rc, mass, skin=0.3, precision=precision, path=path,
                              small_box=small_box), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], types)
    p = oracle.make_params(eps, sig, rc, mass, skin=0.3)
    sysm.build_cells()
    xw, count, ids = compare_cells_lists(sysm, p, s["x"], types, s["L"], tag=name)
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    Fo, peo, wo = oracle.forces_list(p, xw, types, s["L"], count, ids)
    e = floored_err(F, Fo)
    say(f"  force error {e:.3e}")
    assert e <= (1e-12 if precision == 0 else 1e-5)
    ob = sysm.observables()[0]
    rel = 1e-12 if precision == 0 else 1e-6
    assert ob["pe"] == pytest.approx(peo, rel=rel)
    assert ob["virial"] == pytest.approx(wo, rel=rel)


@pytest.mark.parametrize("path", ["gather", "staged"])
def test_forces_mixed(torch_cuda, path):
    say(f"case forces mixed n=32000 {path}")
    sysm, s = make_system(torch_cuda, 32000, 7, precision=1, **PATHS[path])
    p = oracle_params()
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    assert F.dtype == np.float32
    Fo, pe_i, w_i = oracle.forces_cells(p, s["x"], s["type"], s["L"])
    e = floored_err(F, Fo)
    say(f"  mixed force error {e:.3e}")
    xw, _, _, count, ids, _ = oracle_cells_lists(p, s["x"], s["type"], s["L"])
    eps, sig, rc, _ = tables()
    cond = pair_force_sums(eps, sig, rc, s["type"], xw, s["L"], count, ids)
    rep = force_error_report(F, Fo, cond)
    say("  raw |dF|/|F|: p50 {raw_p50:.2e} p99.9 {raw_p999:.2e} max {raw_max:.2e}; "
        "global {global:.2e}; condition-normalised max {cond_max:.2e}".format(**rep))
    assert e <= 1e-5
    assert rep["global"] <= 1e-5 and rep["cond_max"] <= 1e-5
    ob = sysm.observables()[0]
    assert ob["pe"] == pytest.approx(pe_i.sum(), rel=1e-6)
    assert ob["virial"] == pytest.approx(w_i.sum(), rel=1e-6)


@pytest.mark.parametrize("precision,path", [(0, "gather"), (0, "staged"), (1, "gather"),
                                            (1, "staged")])
def test_states_after_steps(torch_cuda, precision, path):
    """Cells, lists and forces re-checked on states reached by stepping."""
    say(f"case stepped states precision={precision} {path}")
    sysm, s = make_system(torch_cuda, 4000, 1, precision=precision, **PATHS[path])
    p = oracle_params()
    done = 0
    for target in (10, 50, 100):
        sysm.step(target - done)
        done = target
        x, v, img = sysm.get_state()
        x = x.cpu().numpy()
        sysm.build_cells()
        xw, count, ids = compare_cells_lists(sysm, p, x, s["type"], s["L"], tag=f"step {target}")
        sysm.forces()
        F = sysm.get_forces().cpu().numpy()
        Fo, peo, wo = oracle.forces_list(p, xw, s["type"], s["L"], count, ids)
        e = floored_err(F, Fo)
        say(f"  step {target}: force error {e:.3e}")
        assert e <= (1e-12 if precision == 0 else 1e-5)
        ob = sysm.observables()[0]
        assert ob["pe"] == pytest.approx(peo, rel=1e-12 if precision == 0 else 1e-6)


def test_short_trajectory_matches_oracle(torch_cuda):
    """FP64: 20 steps from the same start agree far below the chaos horizon."""
    say("case short trajectory fp64")
    sysm, s = make_system(torch_cuda, 4000, 1)
    sim = oracle.Sim(oracle_params(), 4000, s["L"], 0.005)
    sim.set_state(s["x"], s["v"], s["type"])
    log = sysm.step(20, log_every=1)
    ref = sim.step(20)
    x, v, img = sysm.get_state()
    xo, vo, imgo = sim.get_state()
    xu = x.cpu().numpy() + img.cpu().numpy() * s["L"]
    xou = xo + imgo * s["L"]
    assert np.max(np.abs(xu - xou)) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - vo)) < 1e-8
    assert np.allclose(log["E"][:, 0], ref["E"], rtol=1e-10)
    assert np.array_equal(log["step"][:, 0], np.arange(1, 21))
    # the skin rule: same displacement maxima, rebuilds at the same steps
    assert np.allclose(log["max_disp"][:, 0], np.sqrt(ref["max_disp2"]), rtol=1e-8, atol=0)
    nb = log["n_rebuild"][:, 0]
    assert np.array_equal(np.diff(np.concatenate([[nb[0] - ref["rebuilt"][0]], nb])),
                          ref["rebuilt"])
    assert ref["rebuilt"].sum() >= 2


@pytest.mark.parametrize("precision,n,kw", [
    (0, 4000, {}), (1, 4000, {}), (0, 32000, dict(tpp=4, unroll=2)),
    (1, 32000, dict(tpp=1, unroll=8)), (0, 500, {}), (1, 864, dict(tpp=8, unroll=1)),
])
def test_fused_kick_matches_split(torch_cuda, precision, n, kw):
    """NVE steps whose force launch also applies the next step's kick and
    drift give bit for bit the trajectory of separate kick launches: state,
    forces, every logged observable and the rebuild steps, across call
    boundaries and with and without per-step energies."""
    say(f"case fused kick vs split precision={precision} n={n} {kw}")
    runs = []
    for split in (0, 1):
        sysm, s = make_system(torch_cuda, n, 5, precision, split_kick=split, **kw)
        logs = [sysm.step(23, log_every=1)]
        sysm.step(25)
        logs.append(sysm.step(1, log_every=1))
        logs.append(sysm.step(14, log_every=7))
        sysm.step(2)
        x, v, img = sysm.get_state()
        F = sysm.get_forces()
        runs.append((logs, x.cpu().numpy(), v.cpu().numpy(), img.cpu().numpy(),
                     F.cpu().numpy(), sysm.observables()[0]))
    (la, xa, va, ia, Fa, oa), (lb, xb, vb, ib, Fb, ob) = runs
    assert np.array_equal(xa, xb)
    assert np.array_equal(va, vb)
    assert np.array_equal(ia, ib)
    assert np.array_equal(Fa, Fb)
    for a, b in zip(la, lb):
        for key in a:
            assert np.array_equal(a[key], b[key]), key
    for key in oa:
        assert oa[key] == ob[key], key
    say(f"  rebuilds {oa['n_rebuild']} in {oa['step']} steps")
    assert oa["n_rebuild"] >= 4 and oa["step"] == 65


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_kick_matches_split_1m(torch_cuda, precision):
    """The benchmark's box (1,048,576 particles, lists read with non-temporal
    loads, two lanes per particle and four pipelined entries): 30 fused NVE
    steps give the state, forces and observables of separate kick launches
    bit for bit."""
    say(f"case fused kick vs split at 1M precision={precision}")
    outs = []
    for split in (0, 1):
        sysm, s = make_system(torch_cuda, 1048576, 2, precision, split_kick=split, tpp=2,
                              unroll=4)
        log = sysm.step(30, log_every=10)
        x, v, img = sysm.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), img.cpu().numpy(),
                     sysm.get_forces().cpu().numpy(), log, sysm.observables()[0]))
        sysm.close()
    (xa, va, ia, fa, la, oa), (xb, vb, ib, fb, lb, ob) = outs
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ia, ib)
    assert np.array_equal(fa, fb)
    for key in la:
        assert np.array_equal(la[key], lb[key]), key
    assert oa == ob
    say(f"  rebuilds {oa['n_rebuild']} in {oa['step']} steps")
    assert oa["n_rebuild"] >= 3


@pytest.mark.parametrize("path", ["gather", "staged"])
def test_nve_drift_fp64_and_mixed(torch_cuda, path):
    """4,000 particles, dt = 0.005: steady-state drift below 1e-4 per particle."""
    for precision in (0, 1):
        say(f"case drift precision={precision} {path}")
        sysm, s = make_system(torch_cuda, 4000, 1, precision=precision, **PATHS[path])
        log = sysm.step(1100, log_every=1)
        E = log["E"][:, 0]
        D = drift_slope(E, 4000)
        tail = (E[100:] - E[100]) / 4000
        say(f"  drift D = {D:.3e}, max |E - E(100)|/N = {np.abs(tail).max():.3e}, "
            f"std(E/N) = {np.std(E[100:] / 4000):.3e}, rebuilds = {log['n_rebuild'][-1, 0]}")
        assert D <= 1e-4
        assert log["n_rebuild"][-1, 0] > 10


def test_thermostat_and_ramp(torch_cuda):
    say("case thermostat")
    sysm, s = make_system(torch_cuda, 4000, 5, T=2.0)
    log = sysm.step(30, T0=0.8, log_every=1)
    assert np.allclose(log["T"][:, 0], 0.8, rtol=1e-13)
    _, v, _ = sysm.get_state()
    v = v.cpu().numpy()
    assert np.sum(v * v) / (3 * 4000 - 3) == pytest.approx(0.8, rel=1e-13)
    log = sysm.step(40, T0=0.8, T1=0.4, ramp=20, log_every=1)
    expect = 0.8 + (0.4 - 0.8) * np.minimum(np.arange(1, 41) / 20, 1.0)
    assert np.allclose(log["T"][:, 0], expect, rtol=1e-13)
    assert np.allclose(log["T_target"][:, 0], expect, rtol=1e-15)


def test_thermostat_matches_oracle(torch_cuda):
    say("case thermostat vs oracle")
    sysm, s = make_system(torch_cuda, 4000, 5, T=2.0)
    sim = oracle.Sim(oracle_params(), 4000, s["L"], 0.005)
    sim.set_state(s["x"], s["v"], s["type"])
    log = sysm.step(10, T0=1.0, T1=0.5, ramp=10, log_every=1)
    ref = sim.step(10, T0=1.0, T1=0.5, ramp=10)
    assert np.allclose(log["pe"][:, 0], ref["pe"], rtol=1e-10)
    assert np.allclose(log["T"][:, 0], ref["T"], rtol=1e-12)


def test_batched_replicas(torch_cuda):
    """Uneven replicas in one context: each matches the oracle on its own box."""
    from paper_1105_5613_amd import System
    say("case batched replicas")
    sizes = [1000, 3001, 500, 8788, 2048]
    temps = [0.4, 1.0, 2.0, 1.5, 0.7]
    systems = initconf.batched_systems(sizes, temps, seed=9)
    x, v, t, n, L = initconf.concat_replicas(systems)
    for precision, kw in ((0, {}), (1, {}), (0, dict(path=2))):
        if kw:   # every replica with >= 3 cells per side: the staged path
            keep = [r for r, sy in enumerate(systems) if sy["L"] >= 3 * 2.8]
            systems = [systems[r] for r in keep]
            temps = [temps[r] for r in keep]
            x, v, t, n, L = initconf.concat_replicas(systems)
        sysm = System(lib_params(precision=precision, **kw), n, L)
        sysm.set_state(x, v, t)
        sysm.build_cells()
        sysm.forces()
        F = sysm.get_forces().cpu().numpy()
        obs = sysm.observables()
        p = oracle_params()
        off = 0
        for r, sy in enumerate(systems):
            xw, count, ids = compare_cells_lists(sysm, p, sy["x"], sy["type"], sy["L"], rep=r,
                                                 tag=f"replica {r}")
            Fo, peo, wo = oracle.forces_list(p, xw, sy["type"], sy["L"], count, ids)
            e = floored_err(F[off:off + sy["n"]], Fo)
            assert e <= (1e-12 if precision == 0 else 1e-5), (r, e)
            assert obs[r]["pe"] == pytest.approx(peo, rel=1e-12 if precision == 0 else 1e-6)
            off += sy["n"]
        # stepping with per-replica thermostat targets
        log = sysm.step(20, T0=temps, log_every=5)
        assert np.allclose(log["T"][-1], temps, rtol=1e-12)


def test_error_paths(torch_cuda):
    from paper_1105_5613_amd import MDError, System
    say("case error paths")
    s = initconf.fcc_system(500, seed=3)
    # box smaller than 2 (rc + skin)
    with pytest.raises(MDError) as ex:
        System(lib_params(), [500], [5.0])
    assert ex.value.code == -3
    # unknown kick mode
    with pytest.raises(MDError) as ex:
        System(lib_params(split_kick=2), [500], [s["L"]])
    assert ex.value.code == -1
    # unknown small-box mode
    with pytest.raises(MDError) as ex:
        System(lib_params(small_box=2), [500], [s["L"]])
    assert ex.value.code == -1
    # bad species
    sysm = System(lib_params(), [500], [s["L"]])
    bad = s["type"].copy()
    bad[7] = 5
    with pytest.raises(MDError) as ex:
        sysm.set_state(s["x"], s["v"], bad)
    assert ex.value.code == -1
    # non-finite input
    xb = s["x"].copy()
    xb[3, 1] = np.nan
    with pytest.raises(MDError) as ex:
        sysm.set_state(xb, s["v"], s["type"])
    assert ex.value.code == -5
    # out of order
    fresh = System(lib_params(), [500], [s["L"]])
    with pytest.raises(MDError) as ex:
        fresh.forces()
    assert ex.value.code == -7
    # a tiny neighbour capacity grows on the first build
    small = System(lib_params(max_neighbors=8), [500], [s["L"]])
    small.set_state(s["x"], s["v"], s["type"])
    small.build_cells()
    assert small.replica_info()["max_neighbors"] > 8
    p = oracle_params()
    compare_cells_lists(small, p, s["x"], s["type"], s["L"], tag="grown capacity")


@pytest.mark.parametrize("path", ["gather", "staged"])
def test_large_box_sampled(torch_cuda, path):
    """1,048,576 particles: full lists bit-exact, sampled forces vs the oracle;
    energy, virial and kinetic totals through the one-level reduction and (FP64
    gather with eight lanes per particle: 32,768 partial blocks) the
    two-level one."""
    say(f"case 1M particles {path}")
    n = 1048576
    for precision in (0, 1):
        kw = dict(PATHS[path])
        if path == "gather" and precision == 0:
            kw.update(tpp=8, unroll=1)
        sysm, s = make_system(torch_cuda, n, 2, precision=precision, **kw)
        p = oracle_params()
        sysm.step(20)
        x, v, img = sysm.get_state()
        x = x.cpu().numpy()
        sysm.build_cells()
        xw, count, ids = compare_cells_lists(sysm, p, x, s["type"], s["L"], tag="1M")
        sysm.forces()
        F = sysm.get_forces().cpu().numpy()
        sel = np.random.default_rng(0).choice(n, 4096, replace=False)
        Fo, _, _ = oracle.forces_cells(p, x, s["type"], s["L"], sel=sel)
        Fall = np.linalg.norm(F, axis=1)
        frms = float(np.sqrt(np.mean(Fall ** 2)))
        d = np.linalg.norm(F[sel].astype(np.float64) - Fo, axis=1)
        e = float(np.max(d / np.maximum(np.linalg.norm(Fo, axis=1), frms)))
        say(f"  precision {precision}: sampled force error {e:.3e}")
        assert e <= (1e-12 if precision == 0 else 1e-5)
        ob = sysm.observables()[0]
        _, pe_i, w_i = oracle.forces_cells(p, x, s["type"], s["L"])
        tol = 1e-12 if precision == 0 else 1e-6
        assert ob["pe"] == pytest.approx(float(np.sum(pe_i)), rel=tol)
        assert ob["virial"] == pytest.approx(float(np.sum(w_i)), rel=tol)
        m = np.array(initconf.mixture_tables()[3])[s["type"]]
        ke = 0.5 * float(np.sum(m[:, None] * v.cpu().numpy() ** 2))
        assert ob["ke"] == pytest.approx(ke, rel=1e-12)
        # the total force vanishes to round-off (full list: both sides of a pair)
        assert np.max(np.abs(F.astype(np.float64).sum(axis=0))) <= \
            (1e-9 if precision == 0 else 1e-2) * np.sum(Fall)


def test_67m_mixed_sampled(torch_cuda):
    """One GPU's large share: 67,108,864 particles, mixed precision, after 10
    steps.  Cell arrays bit-exact over the whole box; forces of 131,072
    sampled particles against the oracle's cell-list forces, and the total
    potential energy and virial against the oracle's sums over all particles
    (the full neighbour list, about 50 GB on the host, is checked through the
    forces it produces)."""
    say("case 67M mixed")
    from paper_1105_5613_amd import System
    n = 67108864
    s = initconf.fcc_system(n, seed=3, temperature=2.0)
    sysm = System(lib_params(precision=1), [n], [s["L"]])
    sysm.set_state(s["x"], s["v"], s["type"])
    sysm.step(10)
    x = sysm.get_state()[0].cpu().numpy()
    sysm.build_cells()
    p = oracle_params()
    _, _, _, cs, order, nc = oracle.build_cells(p, x, s["L"])
    gcs, gorder = sysm.get_cells(0)
    assert sysm.replica_info(0)["nc"] == nc == 136
    assert np.array_equal(gcs, cs) and np.array_equal(gorder, order)
    del gcs, gorder, cs, order
    say("  cells bit-exact")
    sysm.forces()
    F = sysm.get_forces().cpu().numpy()
    ob = sysm.observables()[0]
    sysm.close()
    Fo, pe_i, w_i = oracle.forces_cells(p, x, s["type"], s["L"])
    say("  oracle forces done")
    sel = np.random.default_rng(5).choice(n, 131072, replace=False)
    frms = float(np.sqrt(np.mean(np.sum(F.astype(np.float64) ** 2, axis=1))))
    d = np.linalg.norm(F[sel].astype(np.float64) - Fo[sel], axis=1)
    e = float(np.max(d / np.maximum(np.linalg.norm(Fo[sel], axis=1), frms)))
    pe, w = float(np.sum(pe_i)), float(np.sum(w_i))
    say(f"  sampled force error {e:.3e}; pe {ob['pe']:.10e} vs {pe:.10e}, "
        f"virial {ob['virial']:.10e} vs {w:.10e}")
    assert e <= 1e-5
    assert ob["pe"] == pytest.approx(pe, rel=1e-6)
    assert ob["virial"] == pytest.approx(w, rel=1e-6)
    assert np.isfinite(ob["E"]) and ob["n_rebuild"] >= 2


@pytest.mark.parametrize("path", ["gather", "staged"])
def test_deterministic(torch_cuda, path):
    """Two runs from the same state give identical bits (fixed reduction order)."""
    say(f"case determinism {path}")
    outs = []
    for _ in range(2):
        sysm, s = make_system(torch_cuda, 32000, 7, **PATHS[path])
        log = sysm.step(30, log_every=1)
        x, v, img = sysm.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), log["E"]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_direct(torch_cuda, precision):
    """K-step graphs replayed several times (two calls, ramp, log) give the
    same bits as direct launches."""
    say(f"case graph replays precision={precision}")
    outs = []
    for K in (0, 10):
        sysm, s = make_system(torch_cuda, 4000, 5, precision=precision, graph_steps=K)
        logs = [sysm.step(35, T0=1.5, T1=0.9, ramp=30, log_every=5)]
        _ = sysm.get_state()  # eager work between the replays
        logs.append(sysm.step(27, T0=0.9, T1=0.9, ramp=0, log_every=9))
        x, v, img = sysm.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), img.cpu().numpy(), logs))
    (x0, v0, i0, l0), (x1, v1, i1, l1) = outs
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1) and np.array_equal(i0, i1)
    for a, b in zip(l0, l1):
        for k in ("E", "T", "pe", "virial", "step", "n_rebuild"):
            assert np.array_equal(a[k], b[k]), k


def test_nve_graphs_between_fused_direct_steps(torch_cuda):
    """NVE graph replays (separate kick launches) followed by directly launched
    fused steps, an odd number of position-buffer swaps and a second call
    that captures again: the same bits as plain direct launches."""
    say("case NVE graphs and fused direct steps")
    outs = []
    for kw in (dict(graph_steps=0, split_kick=1), dict(graph_steps=10)):
        sysm, s = make_system(torch_cuda, 4000, 5, **kw)
        logs = [sysm.step(26, log_every=2)]
        logs.append(sysm.step(20, log_every=5))
        sysm.step(3)
        x, v, img = sysm.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy(), img.cpu().numpy(), logs,
                     sysm.get_forces().cpu().numpy()))
    (x0, v0, i0, l0, f0), (x1, v1, i1, l1, f1) = outs
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1) and np.array_equal(i0, i1)
    assert np.array_equal(f0, f1)
    for a, b in zip(l0, l1):
        for k in a:
            assert np.array_equal(a[k], b[k]), k


def test_profiling_with_graph_steps(torch_cuda):
    """With force-kernel timing on, a graph-configured context launches the
    steps directly (bit-identical to its graph replays) and the timed
    launches can be read back."""
    say("case profiling with graph_steps")
    ref, _ = make_system(torch_cuda, 4000, 5, graph_steps=10)
    ref.step(20)
    xr, vr, _ = ref.get_state()
    sysm, _ = make_system(torch_cuda, 4000, 5, graph_steps=10)
    sysm.profile(2)
    sysm.step(20)
    pr = sysm.profile_read()
    assert pr["force_launches"] == 10
    assert pr["force_ms"] > 0.0
    x, v, _ = sysm.get_state()
    assert np.array_equal(x.cpu().numpy(), xr.cpu().numpy())
    assert np.array_equal(v.cpu().numpy(), vr.cpu().numpy())


def test_torch_allocator(torch_cuda):
    """Context buffers from torch's caching allocator (md_init_alloc), including
    a neighbour-capacity growth that frees and allocates through it: the same
    bits as hipMalloc buffers, and every block is handed back at close."""
    from paper_1105_5613_amd import System
    say("case torch allocator")
    s = initconf.fcc_system(4000, seed=5, temperature=2.0)
    outs = []
    for alloc in (None, "torch"):
        sysm = System(lib_params(max_neighbors=24), [4000], [s["L"]], allocator=alloc)
        sysm.set_state(s["x"], s["v"], s["type"])
        sysm.build_cells()  # 24 slots overflow: the capacity grows once
        assert sysm.replica_info(0)["max_neighbors"] > 24
        sysm.step(50)
        x, v, _ = sysm.get_state()
        outs.append((x.cpu().numpy(), v.cpu().numpy()))
        a = sysm.allocator
        if alloc:
            assert a.bytes_held() > 0
        sysm.close()
        if alloc:
            assert a.bytes_held() == 0
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_checkpoint_resume(torch_cuda):
    """200 steps straight vs 100 + get_state/set_state + 100.  The restored
    context builds its lists on the restored state at step 100, so the
    straight run rebuilds there too (md_build_cells): then the two runs do
    the same arithmetic and must agree bit for bit (FP64 path)."""
    say("case checkpoint")
    a, s = make_system(torch_cuda, 4000, 6)
    a.step(100)
    a.build_cells()
    a.step(100)
    xa, va, ia = (t.cpu().numpy() for t in a.get_state())
    Fa = a.get_forces().cpu().numpy()
    b, _ = make_system(torch_cuda, 4000, 6)
    b.step(100)
    x, v, img = b.get_state()
    c, _ = make_system(torch_cuda, 4000, 6)
    c.set_state(x, v, s["type"])
    c.step(100)
    xc, vc, ic = (t.cpu().numpy() for t in c.get_state())
    Fc = c.get_forces().cpu().numpy()
    assert np.array_equal(xa, xc)
    assert np.array_equal(va, vc)
    assert np.array_equal(ia, ic + img.cpu().numpy())
    assert np.array_equal(Fa, Fc)
    assert a.observables()[0]["E"] == c.observables()[0]["E"]
