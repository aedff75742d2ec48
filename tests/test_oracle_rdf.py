"""Pins of the oracle's radial distribution function (glass section):
g(r) = 2V/N^2 <sum_{i<j} delta(r - r_ij)>, estimated as a histogram.

* a perfect FCC crystal: the running coordination number
  n(r) = (2/N) * (pairs with r_ij < r) = rho * sum_b g_b * shell_b
  steps by the textbook FCC shell counts 12, 6, 24, 12, 24, 8 at the shell
  radii a/sqrt2, a, a sqrt(3/2), a sqrt2, a sqrt(5/2), a sqrt3;
* an ideal gas (uniform positions): g = 1 - 1/N in expectation at every r;
* two particles: a single count in the bin of their minimum-image distance,
  also across the periodic boundary.
"""
import math

import numpy as np

import oracle
from initconf import fcc_system, uniform_positions

RHO = 1.2


def _counts(g, n, L, rmax, nbins):
    dr = rmax / nbins
    r0 = np.arange(nbins) * dr
    r1 = r0 + dr
    shell = 4.0 / 3.0 * math.pi * (r1 ** 3 - r0 ** 3)
    return g * n * n * shell / (2.0 * L ** 3), r1


def test_rdf_fcc_shell_counts():
    m = 4
    n = 4 * m ** 3
    s = fcc_system(n, rho=RHO, jitter=0.0, seed=3)
    L = s["L"]
    a = L / m
    rmax, nbins = 0.49 * L, 490
    g = oracle.rdf(s["x"], L, rmax, nbins)
    pairs, r1 = _counts(g, n, L, rmax, nbins)
    np.testing.assert_allclose(pairs, np.round(pairs), atol=1e-6)
    running = 2.0 * np.cumsum(np.round(pairs)) / n
    shells = a * np.sqrt([0.5, 1.0, 1.5, 2.0, 2.5, 3.0])
    cum = [12, 18, 42, 54, 78, 86]
    for k, rs in enumerate(shells):
        # a bin edge between this shell and the next
        nxt = shells[k + 1] if k + 1 < len(shells) else a * math.sqrt(3.5)
        b = int(np.searchsorted(r1, 0.5 * (rs + nxt)))
        assert running[b] == cum[k], (k, running[b])
    # nothing inside the nearest-neighbour shell
    assert running[int(np.searchsorted(r1, 0.9 * shells[0]))] == 0


def test_rdf_ideal_gas_is_one():
    n = 3000
    L = (n / RHO) ** (1.0 / 3.0)
    x = uniform_positions(n, L, seed=77)
    rmax, nbins = 0.5 * L, 50
    g = oracle.rdf(x, L, rmax, nbins)
    # bins from r = 1.5 on hold thousands of pairs each
    sel = (np.arange(nbins) + 0.5) * rmax / nbins > 1.5
    assert abs(g[sel].mean() - (1 - 1 / n)) < 0.01
    assert np.all(np.abs(g[sel] - 1) < 0.1)


def test_rdf_two_particles_across_boundary():
    L = 10.0
    x = np.array([[0.25, 5.0, 5.0], [9.5, 5.0, 5.0]])  # distance 0.75 through the wall
    rmax, nbins = 5.0, 50
    g = oracle.rdf(x, L, rmax, nbins)
    pairs, _ = _counts(g, 2, L, rmax, nbins)
    want = np.zeros(nbins)
    want[7] = 1.0  # 0.75 lies in [0.7, 0.8)
    np.testing.assert_allclose(pairs, want, atol=1e-9)
