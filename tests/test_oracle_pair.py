"""Pins of the oracle's pair functions against exact closed forms.

Eq. (1) (Lennard-Jones), Eq. (2) (soft sphere) and the truncated
shifted-force form Eq. (3) of the "Interaction potential" section are
evaluated here in exact rational arithmetic (``fractions.Fraction``) at
rational separations, which is an independent computation of the same
mathematics; a dropped term, a wrong sign or a wrong power in the oracle
fails these tests.
"""
from fractions import Fraction as Q
import math
import random

import pytest

import initconf

EPS_M = 2.0 ** -52


def exact_v(eps, sig, r, soft=False):
    s = Q(sig) / Q(r)
    s6 = s ** 6
    if soft:
        return 4 * Q(eps) * s6 * s6
    return 4 * Q(eps) * (s6 * s6 - s6)


def exact_dv(eps, sig, r, soft=False):
    s = Q(sig) / Q(r)
    s6 = s ** 6
    if soft:
        return -48 * Q(eps) * s6 * s6 / Q(r)
    return -4 * Q(eps) * (12 * s6 * s6 - 6 * s6) / Q(r)


def exact_pair(eps, sig, rc, r, soft=False, trunc=0):
    if not (r < rc):
        return Q(0), Q(0)
    vr, dvr = exact_v(eps, sig, r, soft), exact_dv(eps, sig, r, soft)
    vc, dvc = exact_v(eps, sig, rc, soft), exact_dv(eps, sig, rc, soft)
    if trunc == 0:
        return vr - vc - (Q(r) - Q(rc)) * dvc, -dvr + dvc
    return vr - vc, -dvr


def test_cutoff_constants_closed_form(oracle_lib, mix_params):
    """V(rc) and V'(rc) of Eq. (1) at rc = 2.5 sigma_ab for the three pairs.

    The decimal values are the exact closed forms
    4 eps [(sig/rc)^12 - (sig/rc)^6] and -(24 eps / rc)[2 (sig/rc)^12 - (sig/rc)^6]
    (AA: sig/rc = 0.4 exactly).  AB/BB use the binary values of 0.8 / 0.88.
    """
    o = oracle_lib
    # AA: exact decimals
    assert o.v(mix_params, 0, 0, 2.5) == pytest.approx(-0.016316891136, rel=4 * EPS_M)
    assert o.dv(mix_params, 0, 0, 2.5) == pytest.approx(0.0389994774528, rel=4 * EPS_M)
    eps, sig, rc, _ = initconf.mixture_tables()
    for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        r = rc[a][b]
        ev = float(exact_v(eps[a][b], sig[a][b], r))
        edv = float(exact_dv(eps[a][b], sig[a][b], r))
        assert o.v(mix_params, a, b, r) == pytest.approx(ev, rel=16 * EPS_M)
        assert o.dv(mix_params, a, b, r) == pytest.approx(edv, rel=16 * EPS_M)
    # AB printed values (rc = 2.0, sig = 0.8, eps = 1.5)
    assert o.v(mix_params, 0, 1, 2.0) == pytest.approx(-0.024475336704, rel=1e-12)
    assert o.dv(mix_params, 0, 1, 2.0) == pytest.approx(0.073124020224, rel=1e-12)


def test_special_points(oracle_lib, mix_params):
    o = oracle_lib
    # V(sigma) = 0, minimum at 2^(1/6) sigma with depth -eps
    for a, b, s, e in [(0, 0, 1.0, 1.0), (0, 1, 0.8, 1.5), (1, 1, 0.88, 0.5)]:
        assert abs(o.v(mix_params, a, b, s)) <= 8 * EPS_M * 4 * e
        rmin = 2.0 ** (1.0 / 6.0) * s
        assert o.v(mix_params, a, b, rmin) == pytest.approx(-e, rel=1e-14)
        assert abs(o.dv(mix_params, a, b, rmin)) <= 1e-13 * 24 * e / rmin
    # Eq. (3): V* and f vanish at (and beyond) the cutoff, continuously
    eps, sig, rc, _ = initconf.mixture_tables()
    for a, b in [(0, 0), (0, 1), (1, 1)]:
        vs, f = o.pair(mix_params, a, b, rc[a][b])
        assert vs == 0.0 and f == 0.0
        vs, f = o.pair(mix_params, a, b, rc[a][b] * (1 - 1e-9))
        assert abs(vs) < 1e-15 and abs(f) < 1e-8
        vs, f = o.pair(mix_params, a, b, rc[a][b] * 1.5)
        assert vs == 0.0 and f == 0.0


@pytest.mark.parametrize("soft,trunc", [(False, 0), (False, 1), (True, 0), (True, 1)])
def test_pair_exact_rationals(oracle_lib, soft, trunc):
    """V*(r) and f(r) of Eq. (3) against exact rational evaluation."""
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, skin=0.3, potential=1 if soft else 0, trunc=trunc)
    rng = random.Random(7)
    for a, b in [(0, 0), (0, 1), (1, 1)]:
        for _ in range(60):
            r = rng.uniform(0.75 * sig[a][b], rc[a][b] * 1.02)
            vs, f = o.pair(p, a, b, r)
            ev, ef = exact_pair(eps[a][b], sig[a][b], rc[a][b], r, soft, trunc)
            # rounding scale: magnitude of the terms that are combined
            # (sum of absolute values of the terms, incl. the r^-12 / r^-6 parts)
            s6 = (Q(sig[a][b]) / Q(r)) ** 6
            e4 = 4 * Q(eps[a][b])
            vr = e4 * (s6 * s6 + s6)
            dvr = e4 * (12 * s6 * s6 + 6 * s6) / Q(r)
            vc = abs(exact_v(eps[a][b], sig[a][b], rc[a][b], soft))
            dvc = abs(exact_dv(eps[a][b], sig[a][b], rc[a][b], soft))
            scale_v = float(vr + vc + abs(Q(r) - Q(rc[a][b])) * dvc)
            scale_f = float(dvr + dvc)
            assert abs(vs - float(ev)) <= 32 * EPS_M * scale_v + 1e-300
            assert abs(f - float(ef)) <= 32 * EPS_M * scale_f + 1e-300


def test_force_is_minus_derivative(oracle_lib, mix_params):
    """f(r) = -dV*/dr by a central difference of the oracle's own V*."""
    o = oracle_lib
    for a, b, lo, hi in [(0, 0, 0.9, 2.45), (0, 1, 0.7, 1.95), (1, 1, 0.8, 2.15)]:
        for r in [lo + (hi - lo) * k / 9 for k in range(10)]:
            h = 1e-5 * r
            vp, _ = o.pair(mix_params, a, b, r + h)
            vm, _ = o.pair(mix_params, a, b, r - h)
            _, f = o.pair(mix_params, a, b, r)
            fd = -(vp - vm) / (2 * h)
            assert fd == pytest.approx(f, rel=1e-7, abs=1e-9)


def test_soft_sphere_reduces_to_r12(oracle_lib):
    """Eq. (2) is Eq. (1) without the r^-6 term."""
    o = oracle_lib
    eps, sig, rc, mass = initconf.mixture_tables()
    p = o.make_params(eps, sig, rc, mass, potential=1)
    for r in [0.9, 1.0, 1.3, 2.0]:
        assert o.v(p, 0, 0, r) == pytest.approx(4.0 * r ** -12, rel=1e-14)
        assert o.dv(p, 0, 0, r) == pytest.approx(-48.0 * r ** -13, rel=1e-14)
    assert math.isclose(o.v(p, 0, 1, 1.0), 4 * 1.5 * 0.8 ** 12, rel_tol=1e-14)
