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
