"""Property-based checks (hypothesis) of the kernels' per-pair arithmetic, CPU build.

Adversarial inputs for the exact decisions: endpoints with small dyadic coordinates (so
heights, slopes and s^2 are often exactly zero or tied), latitudes drawn from the endpoint
heights, the great circle's top and simple dyadic values, and their binary64 neighbours.
For every drawn pair the EFT evaluation's count, roots and flags equal the exact oracle's,
and its points equal the oracle's AccuX replica; for arc pairs, the arc x arc evaluation's
count and flags equal the exact orientation rule.
"""

import math

import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

from oracle import arcarc as AA, batch as OB, geometry as G

import test_hostcheck as TH
import test_hostcheck_arcarc as TA

dyadic = st.integers(min_value=-8, max_value=8).map(lambda k: k / 4.0)
point = st.tuples(dyadic, dyadic, dyadic).filter(lambda p: any(p))


def _latitudes(x1, x2):
    out = [0.0, 0.5, -0.5, 1.0 / 3.0]
    for x in (x1, x2):
        h = x[2] / math.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
        out += [h, math.nextafter(h, 2.0), math.nextafter(h, -2.0)]
    t = G.exact_terms(x1, x2, 0.0)
    if t["S3"] > 0:
        zmax = math.sqrt(t["S2"] / t["S3"])
        out += [zmax, -zmax, math.nextafter(zmax, 2.0), math.nextafter(zmax, -2.0)]
    return out


_LIB = {}


def _hc():
    if "lat" not in _LIB:
        import ctypes
        lib = ctypes.CDLL(TH.LIBPATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.sphint_hostcheck_eval.argtypes = ([ctypes.c_int, ctypes.c_int64] + [dp] * 7 +
                                              [ip] * 4 + [dp] * 4)
        lib.sphint_hostcheck_arcarc.argtypes = [ctypes.c_int, ctypes.c_int64,
                                                ctypes.POINTER(dp), ctypes.POINTER(dp),
                                                dp, dp, dp, ip, ip]
        _LIB["lat"] = lib
    return _LIB["lat"]


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(point, point)
def test_eft_decisions_on_dyadic_arcs(x1, x2):
    lats = _latitudes(x1, x2)
    n = len(lats)
    soa = [np.full(n, x1[0]), np.full(n, x1[1]), np.full(n, x1[2]),
           np.full(n, x2[0]), np.full(n, x2[1]), np.full(n, x2[2]), np.array(lats)]
    count, flags, r0, r1, px0, py0, px1, py1 = TH.run(_hc(), 1, soa)
    ex = OB.exact(*soa, workers=1)
    assert np.array_equal(count, ex.count)
    assert np.array_equal(flags & TH.FLAG_MASK, ex.flags)
    rep = OB.accux_points(*soa, ex.roots, workers=1)
    for i in range(n):
        got = [(r0[i], px0[i], py0[i]), (r1[i], px1[i], py1[i])][:count[i]]
        assert tuple(int(g[0]) for g in got) == ex.roots[i]
        for j, (_, x, y) in enumerate(got):
            assert (x, y) == rep[i][j]


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(point, point, point, point)
def test_arcarc_decisions_on_dyadic_arcs(a1, a2, b1, b2):
    A, B = TA.soa([(a1, a2, b1, b2)])
    count, flags, *_ = TA.run(_hc(), 1, A, B)
    c, _, fl = AA.classify(a1, a2, b1, b2)
    assert (int(count[0]), int(flags[0]) & TA.MASK) == (c, fl)
