"""Pins of the oracle's force sums, cell list and neighbour list.

What fixes the expected values here (never the oracle itself):
* analytic two- and three-body forces from exact rational pair functions;
* a perfect one-species FCC lattice: every site is an inversion centre, so
  each force vanishes, and the energy equals the lattice shell sum;
* Newton's third law (section "Grid-search method"): the total force is 0;
* F = -grad U by central differences, and W = -dU/ds under uniform box
  scaling x -> s x, L -> s L (the virial theorem form of the pressure);
* cell list and neighbour list against their definitions (the cell of a
  particle contains it; the list is the set of pairs closer than rc + skin,
  found by an independent numpy brute force).
"""
from fractions import Fraction as Q
import itertools
import math

import numpy as np
import pytest

import initconf
from test_oracle_pair import exact_pair


def floored_err(Fa, Fb):
    """max_i |Fa_i - Fb_i| / max(|Fb_i|, F_rms)."""
    nb = np.linalg.norm(Fb, axis=1)
    frms = math.sqrt(float(np.mean(nb ** 2))) if len(nb) else 1.0
    d = np.linalg.norm(Fa - Fb, axis=1)
    return float(np.max(d / np.maximum(nb, frms)))


def test_two_body_analytic(oracle_lib, mix_params):
    o = oracle_lib
    eps, sig, rc, _ = initconf.mixture_tables()
    L = 12.0
    rng = np.random.default_rng(3)
    for (a, b) in [(0, 0), (0, 1), (1, 1)]:
        for r in [0.85 * sig[a][b], 1.1 * sig[a][b], 0.9 * rc[a][b]]:
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            x = np.array([[3.0, 4.0, 5.0], [3.0, 4.0, 5.0]]) + np.vstack([np.zeros(3), r * u])
            F, pe, w = o.forces_brute(mix_params, x, [a, b], L)
            d = x[0] - x[1]
            rr = float(np.linalg.norm(d))
            ev, ef = exact_pair(eps[a][b], sig[a][b], rc[a][b], rr)
            expect = float(ef) * d / rr
            assert np.allclose(F[0], expect, rtol=1e-13, atol=1e-13 * abs(float(ef)))
            assert np.allclose(F[1], -expect, rtol=1e-13, atol=1e-13 * abs(float(ef)))
            assert pe == pytest.approx(float(ev), rel=1e-12, abs=1e-15)
            assert w == pytest.approx(float(ef) * rr, rel=1e-12, abs=1e-15)


def test_two_body_across_boundary(oracle_lib, mix_params):
    """The minimum image joins a pair that straddles the periodic boundary."""
    o = oracle_lib
    L = 10.0
    x = np.array([[0.2, 5.0, 5.0], [9.3, 5.0, 5.0]])  # separation 0.9 through x = 0
    F, pe, _ = o.forces_brute(mix_params, x, [0, 0], L)
    ev, ef = exact_pair(1.0, 1.0, 2.5, 0.9)
    rr = 0.2 + (L - 9.3)
    ev2, ef2 = exact_pair(1.0, 1.0, 2.5, rr)
    assert F[0][0] == pytest.approx(float(ef2), rel=1e-12)   # pushed to +x
    assert F[1][0] == pytest.approx(-float(ef2), rel=1e-12)
    assert pe == pytest.approx(float(ev2), rel=1e-12)


def test_three_body_superposition(oracle_lib, mix_params):
    o = oracle_lib
    eps, sig, rc, _ = initconf.mixture_tables()
    x = np.array([[5.0, 5.0, 5.0], [6.0, 5.1, 5.0], [5.3, 6.05, 4.8]])
    t = [0, 1, 1]
    F, pe, w = o.forces_brute(mix_params, x, t, 11.0)
    Fe = np.zeros((3, 3))
    pe_e = 0.0
    for i, j in itertools.combinations(range(3), 2):
        d = x[i] - x[j]
        r = float(np.linalg.norm(d))
        ev, ef = exact_pair(eps[t[i]][t[j]], sig[t[i]][t[j]], rc[t[i]][t[j]], r)
        Fe[i] += float(ef) * d / r
        Fe[j] -= float(ef) * d / r
        pe_e += float(ev)
    assert np.allclose(F, Fe, rtol=1e-12, atol=1e-12)
    assert pe == pytest.approx(pe_e, rel=1e-12)


def fcc(m, a):
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    return ((g[:, None, :] + basis[None]) * a).reshape(-1, 3)


@pytest.mark.parametrize("m", [4, 6])
def test_perfect_fcc_zero_force_and_shell_sum(oracle_lib, m):
    """One species on a perfect FCC lattice: F_i = 0 and U = N/2 sum_k z_k V*(r_k)."""
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=0.3)
    a = (4 / 1.2) ** (1 / 3)
    x = fcc(m, a)
    n = len(x)
    L = m * a
    F, pe, w = o.forces_brute(p, x, np.zeros(n, np.int32), L)
    # shell sum over lattice vectors R != 0 with |R| < rc (all fit in the box)
    lat = fcc(7, a) - np.array([3, 3, 3]) * a
    r = np.linalg.norm(lat, axis=1)
    r = r[(r > 1e-9) & (r < 2.5)]
    shell = sum(o.pair(p, 0, 0, float(ri))[0] for ri in r)
    fsum = sum(abs(o.pair(p, 0, 0, float(ri))[1]) for ri in r)
    assert np.max(np.abs(F)) <= 1e-13 * fsum
    assert pe == pytest.approx(0.5 * n * shell, rel=1e-13)
    wshell = sum(o.pair(p, 0, 0, float(ri))[1] * float(ri) for ri in r)
    assert w == pytest.approx(0.5 * n * wshell, rel=1e-12)


def jittered(n, seed, T=1.0):
    s = initconf.fcc_system(n, seed=seed, temperature=T)
    return s["x"], s["type"], s["L"]


def test_newton_third_law_and_invariances(oracle_lib, mix_params):
    o = oracle_lib
    x, t, L = jittered(500, 11)
    F, pe, w = o.forces_brute(mix_params, x, t, L)
    fsum = np.sum(np.abs(F))
    assert np.max(np.abs(F.sum(axis=0))) <= 1e-13 * fsum
    # translation (periodic) invariance
    x2 = np.mod(x + np.array([0.37, -1.21, 2.5]), L)
    F2, pe2, w2 = o.forces_brute(mix_params, x2, t, L)
    assert floored_err(F2, F) < 1e-12
    assert pe2 == pytest.approx(pe, rel=1e-12)
    # permutation equivariance
    perm = np.random.default_rng(5).permutation(len(x))
    F3, pe3, _ = o.forces_brute(mix_params, x[perm], t[perm], L)
    assert floored_err(F3, F[perm]) < 1e-12
    assert pe3 == pytest.approx(pe, rel=1e-12)


def test_force_is_minus_gradient(oracle_lib, mix_params):
    o = oracle_lib
    x, t, L = jittered(256, 12)
    F, pe, _ = o.forces_brute(mix_params, x, t, L)
    rng = np.random.default_rng(1)
    h = 1e-6
    for i in rng.choice(len(x), 8, replace=False):
        for k in range(3):
            xp = x.copy(); xp[i, k] += h
            xm = x.copy(); xm[i, k] -= h
            up = o.forces_brute(mix_params, xp, t, L)[1]
            um = o.forces_brute(mix_params, xm, t, L)[1]
            fd = -(up - um) / (2 * h)
            assert fd == pytest.approx(F[i, k], rel=1e-6, abs=1e-6 * max(1.0, abs(F[i, k])))


def test_virial_is_box_scaling_derivative(oracle_lib, mix_params):
    """W = sum r f(r) = -dU/ds with x -> s x, L -> s L (W = -3V dU/dV)."""
    o = oracle_lib
    x, t, L = jittered(500, 13)
    _, pe, w = o.forces_brute(mix_params, x, t, L)
    d = 1e-6
    up = o.forces_brute(mix_params, x * (1 + d), t, L * (1 + d))[1]
    um = o.forces_brute(mix_params, x * (1 - d), t, L * (1 - d))[1]
    assert -(up - um) / (2 * d) == pytest.approx(w, rel=1e-6)


def check_cells(xw, cell, cs, order, L, nc):
    n = len(xw)
    assert np.all(xw >= 0.0) and np.all(xw < L)
    side = L / nc
    q = np.stack([cell % nc, (cell // nc) % nc, cell // (nc * nc)], 1)
    # the cell of a particle contains it (up to one rounding of x * nc / L)
    lo = q * side
    hi = (q + 1) * side
    assert np.all(xw >= lo - 1e-12 * L) and np.all(xw < hi + 1e-12 * L)
    # cell_start is the exclusive prefix sum of the counts
    counts = np.bincount(cell, minlength=nc ** 3)
    assert cs[0] == 0 and cs[-1] == n
    assert np.array_equal(np.diff(cs), counts)
    # order is ascending (cell, id)
    assert sorted(order.tolist()) == list(range(n))
    keys = cell[order].astype(np.int64) * n + order
    assert np.all(np.diff(keys) > 0)


def brute_pairs(xw, t, L, thr_tab):
    """Independent list: j in list(i) iff min-image r^2 < (rc+skin)^2, with
    the pairs whose r^2 lies within 1e-12 of the threshold reported apart."""
    d = xw[None, :, :] - xw[:, None, :]
    d -= L * np.round(d / L)
    r2 = np.einsum("ijk,ijk->ij", d, d)
    thr = thr_tab[t[:, None], t[None, :]]
    inside = r2 < thr
    np.fill_diagonal(inside, False)
    band = np.abs(r2 - thr) <= 1e-12 * thr
    return inside, band


@pytest.mark.parametrize("n,seed,shift", [(256, 21, 0.0), (500, 22, 0.0), (864, 23, 0.25),
                                          (2048, 24, 0.0), (1372, 25, -0.6)])
def test_cells_and_lists_vs_definition(oracle_lib, n, seed, shift):
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=0.3)
    x, t, L = jittered(n, seed, T=1.0)
    x = x + shift  # some coordinates fall outside [0, L): one wrap brings them back
    xw, img, cell, cs, order, nc = o.build_cells(p, x, L)
    assert np.array_equal(xw + img * L, x) or np.allclose(xw + img * L, x, atol=1e-12 * L)
    check_cells(xw, cell, cs, order, L, nc)
    count, ids = o.build_nlist(p, xw, t, L, cell, cs, order, nc)
    thr_tab = np.array([[(rc[a][b] + 0.3) ** 2 for b in range(2)] for a in range(2)])
    inside, band = brute_pairs(xw, t, L, thr_tab)
    for i in range(n):
        got = np.zeros(n, bool)
        got[ids[i, :count[i]]] = True
        assert len(set(ids[i, :count[i]].tolist())) == count[i]
        diff = got ^ inside[i]
        assert not np.any(diff & ~band[i]), f"particle {i}"
    # the list is symmetric
    pairs = {(i, j) for i in range(n) for j in ids[i, :count[i]]}
    assert all((j, i) in pairs for (i, j) in pairs)
    # forces: brute force == list == cells
    Fb, peb, wb = o.forces_brute(p, xw, t, L)
    Fl, pel, wl = o.forces_list(p, xw, t, L, count, ids)
    Fc, pec, wc = o.forces_cells(p, xw, t, L)
    assert floored_err(Fl, Fb) <= 1e-13
    assert floored_err(Fc, Fb) <= 1e-13
    assert pel == pytest.approx(peb, rel=1e-13)
    assert pec.sum() == pytest.approx(peb, rel=1e-12)
    assert wl == pytest.approx(wb, rel=1e-13)
    assert wc.sum() == pytest.approx(wb, rel=1e-12)


def test_list_symmetric_at_the_threshold_across_a_face(oracle_lib):
    """Two particles on opposite faces of the box, with the cut-off placed
    strictly between the two values that a shift-first displacement
    ((x_j + s L) - x_i) takes in the two directions.  The list must still be
    symmetric, as the third-law halving of the pair count presumes (section
    "Grid-search method"), and agree with d = (x_j - x_i) + s L, whose
    exchange negates every rounding step exactly."""
    o = oracle_lib
    L = 29.3
    rng = np.random.default_rng(7)
    for _ in range(200000):
        a, b = rng.uniform(0.2, 1.1, size=2)
        xa, xb = L - a, b
        if not (xa < L):
            continue
        fwd = ((xb + L) - xa) ** 2   # home xa, partner xb seen at xb + L
        bwd = ((xa - L) - xb) ** 2   # home xb, partner xa seen at xa - L
        lo, hi = min(fwd, bwd), max(fwd, bwd)
        # a cut-off rc with lo < rc * rc < hi (skin 0: the threshold is rc^2)
        rc = math.sqrt(0.5 * (lo + hi))
        for _ in range(8):
            if rc * rc <= lo:
                rc = np.nextafter(rc, np.inf)
            elif rc * rc >= hi:
                rc = np.nextafter(rc, 0.0)
        if lo < rc * rc < hi:
            break
    else:
        pytest.fail("no pair with a threshold between the two shift-first values")
    p = o.make_params([[1.0]], [[0.3]], [[rc]], [1.0], skin=0.0)
    x = np.array([[xa, 5.0, 5.0], [xb, 5.0, 5.0]])
    t = np.zeros(2, np.int32)
    xw, img, cell, cs, order, nc = o.build_cells(p, x, L)
    assert nc >= 3 and np.array_equal(xw, x)
    count, ids = o.build_nlist(p, xw, t, L, cell, cs, order, nc)
    want = ((xb - xa) + L) ** 2 < rc * rc
    assert ((xa - xb) - L) ** 2 == ((xb - xa) + L) ** 2
    assert count.tolist() == [int(want), int(want)]


def test_small_box_single_cell(oracle_lib):
    """L < 3 (rc + skin): one cell, the list falls back to the minimum image."""
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=0.3)
    x, t, L = jittered(200, 31)
    assert L < 3 * 2.8
    xw, img, cell, cs, order, nc = o.build_cells(p, x, L)
    assert nc == 1 and np.all(cell == 0)
    count, ids = o.build_nlist(p, xw, t, L, cell, cs, order, nc)
    thr_tab = np.array([[(rc[a][b] + 0.3) ** 2 for b in range(2)] for a in range(2)])
    inside, band = brute_pairs(xw, t, L, thr_tab)
    for i in range(len(x)):
        got = np.zeros(len(x), bool)
        got[ids[i, :count[i]]] = True
        assert not np.any((got ^ inside[i]) & ~band[i])
    Fb, peb, _ = o.forces_brute(p, xw, t, L)
    Fl, pel, _ = o.forces_list(p, xw, t, L, count, ids)
    assert floored_err(Fl, Fb) <= 1e-13


def test_boundary_placements(oracle_lib):
    """Particles exactly on cell faces, at 0, at L - ulp and at -tiny."""
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=0.3)
    x, t, L = jittered(1372, 32)
    nc, inv = o.cell_grid(p, L)
    side = L / nc
    x = x.copy()
    x[0] = [0.0, 0.0, 0.0]
    x[1] = [np.nextafter(L, 0), np.nextafter(L, 0), 1.0]
    x[2] = [side, 2 * side, 3 * side]
    x[3] = [-1e-18, 5.0, 5.0]          # -tiny + L rounds to L: wraps to 0
    x[4] = [L, 1.0, 1.0]               # exactly L wraps to 0
    x[5] = [-0.1, L + 0.1, 2.0]
    xw, img, cell, cs, order, nc = o.build_cells(p, x, L)
    check_cells(xw, cell, cs, order, L, nc)
    assert xw[3, 0] == 0.0 and img[3, 0] == 0
    assert xw[4, 0] == 0.0 and img[4, 0] == 1
    assert img[5, 0] == -1 and img[5, 1] == 1
    count, ids = o.build_nlist(p, xw, t, L, cell, cs, order, nc)
    thr_tab = np.array([[(rc[a][b] + 0.3) ** 2 for b in range(2)] for a in range(2)])
    inside, band = brute_pairs(xw, t, L, thr_tab)
    for i in range(len(x)):
        got = np.zeros(len(x), bool)
        got[ids[i, :count[i]]] = True
        assert not np.any((got ^ inside[i]) & ~band[i])
