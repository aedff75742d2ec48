"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import initconf  # noqa: E402
import oracle  # noqa: E402

SKIN = 0.3


def tables():
    return initconf.mixture_tables()


def oracle_params(skin=SKIN, potential=0, trunc=0):
    eps, sig, rc, mass = tables()
    return oracle.make_params(eps, sig, rc, mass, skin=skin, potential=potential, trunc=trunc)


def lib_params(precision=0, skin=SKIN, dt=0.005, **kw):
    from paper_1105_5613_amd import make_params
    eps, sig, rc, mass = tables()
    return make_params(eps, sig, rc, mass, skin=skin, dt=dt, precision=precision, **kw)


def floored_err(Fa, Fb):
    """max_i |Fa_i - Fb_i| / max(|Fb_i|, F_rms)."""
    nb = np.linalg.norm(Fb, axis=1)
    frms = math.sqrt(float(np.mean(nb ** 2)))
    d = np.linalg.norm(np.asarray(Fa, dtype=np.float64) - Fb, axis=1)
    return float(np.max(d / np.maximum(nb, frms)))


def force_error_report(Fa, Fb, cond=None):
    """The other error norms reported beside the floored e: the raw per-particle
    ratio |dF_i| / |F_i| (p50, p99.9, max), the global |dF| / |F| and, given
    cond_i = sum_j |F_ij|, the condition-normalised max_i |dF_i| / cond_i."""
    d = np.linalg.norm(np.asarray(Fa, dtype=np.float64) - Fb, axis=1)
    nb = np.linalg.norm(Fb, axis=1)
    raw = d / np.maximum(nb, np.finfo(np.float64).tiny)
    out = {"raw_p50": float(np.percentile(raw, 50)), "raw_p999": float(np.percentile(raw, 99.9)),
           "raw_max": float(raw.max()),
           "global": float(np.linalg.norm(d) / np.linalg.norm(nb))}
    if cond is not None:
        out["cond_max"] = float(np.max(d / cond))
    return out


def pair_force_sums(eps, sig, rc, types, xw, L, count, ids):
    """cond_i = sum over the list of |f(r_ij)| for pairs within r_c (shifted-force LJ,
    Eq. (3)), for the condition-normalised error (a report, not a pin)."""
    eps, sig, rc = (np.asarray(a, dtype=np.float64) for a in (eps, sig, rc))
    n, cap = ids.shape
    i = np.repeat(np.arange(n), cap)
    j = ids.reshape(-1)
    m = (np.arange(cap)[None, :] < count[:, None]).reshape(-1)
    i, j = i[m], j[m]
    d = xw[i] - xw[j]
    d -= L * np.rint(d / L)
    r = np.linalg.norm(d, axis=1)
    a, b = types[i], types[j]
    e, s, c = eps[a, b], sig[a, b], rc[a, b]

    def dv(x):
        sr6 = (s / x) ** 6
        return -(24.0 * e / x) * (2.0 * sr6 * sr6 - sr6)
    f = np.where(r < c, np.abs(-dv(r) + dv(c)), 0.0)
    out = np.zeros(n)
    np.add.at(out, i, f)
    return out


def pair_abs_sums(eps, sig, rc, types, xw, L, count, ids):
    """Condition numbers of the energy and virial sums: sum over the pairs
    within r_c (each once) of |V*(r)| and |r f(r)| (shifted-force LJ,
    Eq. (3)).  A sum of rounded terms errs by at most about n u times the sum
    of their magnitudes; when the signed total is close to zero (a compressed
    lattice whose pair energies cancel) these replace it in a relative bar."""
    eps, sig, rc = (np.asarray(a, dtype=np.float64) for a in (eps, sig, rc))
    n, cap = ids.shape
    i = np.repeat(np.arange(n), cap)
    j = ids.reshape(-1)
    m = (np.arange(cap)[None, :] < count[:, None]).reshape(-1)
    i, j = i[m], j[m]
    d = xw[i] - xw[j]
    d -= L * np.rint(d / L)
    r = np.linalg.norm(d, axis=1)
    a, b = types[i], types[j]
    e, s, c = eps[a, b], sig[a, b], rc[a, b]

    def v(x):
        sr6 = (s / x) ** 6
        return 4.0 * e * (sr6 * sr6 - sr6)

    def dv(x):
        sr6 = (s / x) ** 6
        return -(24.0 * e / x) * (2.0 * sr6 * sr6 - sr6)
    inside = r < c
    vs = np.where(inside, v(r) - v(c) - (r - c) * dv(c), 0.0)
    f = np.where(inside, -dv(r) + dv(c), 0.0)
    return 0.5 * float(np.sum(np.abs(vs))), 0.5 * float(np.sum(np.abs(r * f)))


def canonical(count, ids):
    """Rows of ids sorted ascending, padding with a large value past count."""
    n, cap = ids.shape
    m = np.arange(cap)[None, :] < count[:, None]
    a = np.where(m, ids, np.iinfo(np.int32).max)
    return np.sort(a, axis=1)


def oracle_cells_lists(p, x, types, L):
    xw, img, cell, cs, order, nc = oracle.build_cells(p, x, L)
    count, ids = oracle.build_nlist(p, xw, types, L, cell, cs, order, nc)
    return xw, cs, order, count, ids, nc


def drift_slope(E, n, burn=100):
    e = np.asarray(E, dtype=np.float64)[burn:] / n
    k = np.arange(len(e), dtype=np.float64)
    return abs(np.polyfit(k, e, 1)[0]) * 1000.0
