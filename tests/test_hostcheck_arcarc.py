"""The arc x arc per-pair arithmetic, compiled for the CPU, against the oracle.

libsphint_hostcheck.so compiles the header the GPU kernel uses, so these CPU tests pin its
operation sequence before any GPU run:

* EFT mode: counts and flags equal the exact oracle (integer orientations); points equal the
  oracle's binary64 replica (AccuDOP pairs, CompDot, SumOfSquares) bit for bit and lie within
  4 * 2^-53 of the exact points;
* naive mode: everything equals the oracle's plain binary64 replica bit for bit;
* the exact orientation equals the sign of the integer determinant, ties included.
"""

import ctypes
import math
import os
from decimal import Decimal

import numpy as np
import pytest

from oracle import arcarc as AA
from oracle.geometry import scaled_ints
from paper_2510_09892_amd import inputs

U = 2.0 ** -53
# SPHINT_HOSTCHECK_LIB selects another build of the same sources (e.g. the sanitizer build)
LIBPATH = os.environ.get("SPHINT_HOSTCHECK_LIB") or os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2510_09892_amd",
    "libsphint_hostcheck.so")
MASK = AA.HIT | AA.DEGEN | AA.COPLANAR | AA.NONFINITE
EXACT = 32


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIBPATH):
        pytest.fail("libsphint_hostcheck.so is not built (python -m paper_2510_09892_amd.build)")
    lib = ctypes.CDLL(LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    dpp = ctypes.POINTER(dp)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_arcarc.argtypes = [ctypes.c_int, ctypes.c_int64, dpp, dpp, dp, dp, dp,
                                            ip, ip]
    lib.sphint_hostcheck_orient.argtypes = [dp, dp, dp]
    lib.sphint_hostcheck_orient.restype = ctypes.c_int
    return lib


def run(hc, mode, A, B):
    """A, B: six arrays each (x1, y1, z1, x2, y2, z2)."""
    A = [np.ascontiguousarray(v, dtype=np.float64) for v in A]
    B = [np.ascontiguousarray(v, dtype=np.float64) for v in B]
    n = len(A[0])
    dp = ctypes.POINTER(ctypes.c_double)
    pa = (dp * 6)(*[v.ctypes.data_as(dp) for v in A])
    pb = (dp * 6)(*[v.ctypes.data_as(dp) for v in B])
    px, py, pz = (np.zeros(n) for _ in range(3))
    count, flags = np.zeros(n, np.int32), np.zeros(n, np.int32)
    ip = ctypes.POINTER(ctypes.c_int32)
    hc.sphint_hostcheck_arcarc(mode, n, pa, pb, px.ctypes.data_as(dp), py.ctypes.data_as(dp),
                               pz.ctypes.data_as(dp), count.ctypes.data_as(ip),
                               flags.ctypes.data_as(ip))
    return count, flags, px, py, pz


def soa(pairs):
    a = [np.array([p[k][c] for p in pairs]) for k in (0, 1) for c in range(3)]
    b = [np.array([p[k][c] for p in pairs]) for k in (2, 3) for c in range(3)]
    return a, b


def as_tuples(P: inputs.ArcPairs):
    return [tuple(tuple(float(x) for x in v[i]) for v in (P.a1, P.a2, P.b1, P.b2))
            for i in range(len(P))]


def special_pairs():
    e = (1.0, 0.0, 0.0)
    f = (0.0, 1.0, 0.0)
    out = [
        (e, f, (1.0, 1.0, -1.0), (1.0, 1.0, 1.0)),       # equator x meridian: +p
        (f, e, (1.0, 1.0, -1.0), (1.0, 1.0, 1.0)),       # A reversed: -p
        (e, f, (1.0, 1.0, 1.0), (1.0, 1.0, -1.0)),       # B reversed
        (e, f, (-1.0, -1.0, -1.0), (-1.0, -1.0, 1.0)),   # the far side: miss
        (e, f, (1.0, 1.0, 0.5), (1.0, 1.0, 1.0)),        # north only: miss
        (e, f, (1.0, 1.0, 0.0), (1.0, 1.0, 1.0)),        # T-junction
        (e, f, f, (0.0, 0.0, 1.0)),                      # shared vertex
        (e, f, (0.0, 2.0, 0.0), (0.0, 0.0, 5.0)),        # scaled endpoints
        (e, f, (0.0, 0.0, 1.0), f),                      # shared vertex, B reversed
        (e, e, e, f),                                    # degenerate A
        (e, (-2.0, 0.0, 0.0), e, f),                     # antipodal A
        (e, f, (1.0, 1.0, 0.0), (-1.0, 1.0, 0.0)),       # one great circle
        (e, f, (0.0, 0.0, 1.0), (math.nan, 0.0, 1.0)),   # non-finite
        (e, f, (0.0, 0.0, 1.0), (math.inf, 0.0, 1.0)),
        ((0.6, 0.8, 0.0), (0.0, 0.6, 0.8), (0.8, 0.0, 0.6), (0.0, 0.8, -0.6)),
        ((1.0, 2.0 ** -40, 0.0), (1.0, 0.0, 2.0 ** -40), (1.0, 2.0 ** -41, 2.0 ** -41),
         (1.0, 0.0, 0.0)),  # a tiny triangle: every orientation near the filters' floor
    ]
    return out


def oracle_compare(pairs, eft, naive, eft_tol=4.0):
    """eft, naive: (count, flags, x, y, z) arrays of one evaluation each, against the oracle.
    Returns (hits, pairs that took the exact orientation path)."""
    ce, fe, xe, ye, ze = eft
    cn, fn, xn, yn, zn = naive
    worst = 0.0
    n_hits = n_exact = 0
    for k, (a1, a2, b1, b2) in enumerate(pairs):
        c, sg, fl = AA.classify(a1, a2, b1, b2)
        assert (int(ce[k]), int(fe[k]) & MASK) == (c, fl), (k, pairs[k], ce[k], fe[k])
        n_exact += bool(fe[k] & EXACT)
        assert not fe[k] & 64, (k, pairs[k])
        if c:
            n_hits += 1
            got = (float(xe[k]), float(ye[k]), float(ze[k]))
            want = AA.eft_point(a1, a2, b1, b2, sg)
            assert all(g == w or (math.isnan(g) and math.isnan(w)) for g, w in zip(got, want)), \
                (k, pairs[k], got, want)
            p = AA.point(a1, a2, b1, b2, sg)
            err = max(abs(Decimal(v) - w) for v, w in zip(got, p)) / Decimal(U)
            worst = max(worst, float(err))
        else:
            assert (xe[k], ye[k], ze[k]) == (0.0, 0.0, 0.0)
        # naive: the binary64 decisions and point
        c2, sg2, fl2 = AA.naive_classify(a1, a2, b1, b2)
        assert (int(cn[k]), int(fn[k])) == (c2, fl2), (k, pairs[k])
        if c2:
            got = (float(xn[k]), float(yn[k]), float(zn[k]))
            try:
                want = AA.naive_point(a1, a2, b1, b2, sg2)
            except ZeroDivisionError:  # the rounded cross products are parallel: 0/0
                assert all(math.isnan(v) for v in got)
                continue
            assert got == want, (k, pairs[k])
        else:
            assert (xn[k], yn[k], zn[k]) == (0.0, 0.0, 0.0)
    assert worst <= eft_tol, worst
    return n_hits, n_exact


def check(hc, pairs, eft_tol=4.0):
    a, b = soa(pairs)
    return oracle_compare(pairs, run(hc, 1, a, b), run(hc, 0, a, b), eft_tol)


def test_special_pairs(hc):
    n_hits, n_exact = check(hc, special_pairs())
    assert n_hits >= 8 and n_exact >= 3


@pytest.mark.parametrize("part", [0, 1, 2, 3])
def test_generated_parts(hc, part):
    P = inputs.arc_pairs(1200, seed_tag=50 + part)
    P = P.take(np.nonzero(P.part == part)[0])
    n_hits, n_exact = check(hc, as_tuples(P))
    assert n_hits > 0
    if part == 3:  # a shared vertex zeroes two orientations; the equal-endpoint rule decides them
        assert n_hits == len(P) and n_exact == 0


def test_integer_arcs_exhaustive_signs(hc):
    import itertools
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0, 2.0), repeat=3) if any(v)]
    g = np.random.Generator(np.random.PCG64(92))
    pairs = [tuple(verts[int(i)] for i in g.integers(0, len(verts), 4)) for _ in range(3000)]
    n_hits, n_exact = check(hc, pairs)
    assert n_hits > 300 and n_exact > 800


def test_exact_orient_against_integers(hc):
    g = np.random.Generator(np.random.PCG64(93))
    dp = ctypes.POINTER(ctypes.c_double)
    cases = []
    for _ in range(400):
        u, v = g.standard_normal(3), g.standard_normal(3)
        s, t = g.standard_normal(2)
        w = s * u + t * v  # nearly coplanar: the rounded w is off the plane by ~1e-16
        cases.append((u, v, w))
        cases.append((u, v, g.standard_normal(3)))
        cases.append((u, v, u.copy()))  # exactly zero
        cases.append((u * 2.0 ** 60, v * 2.0 ** -40, w))
    zeros = 0
    for u, v, w in cases:
        ints, _ = scaled_ints((*u, *v, *w))
        U_, V_, W_ = ints[0:3], ints[3:6], ints[6:9]
        det = (U_[0] * (V_[1] * W_[2] - V_[2] * W_[1]) + U_[1] * (V_[2] * W_[0] - V_[0] * W_[2])
               + U_[2] * (V_[0] * W_[1] - V_[1] * W_[0]))
        want = (det > 0) - (det < 0)
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (u, v, w)]
        got = hc.sphint_hostcheck_orient(*[x.ctypes.data_as(dp) for x in arrs])
        assert got == want, (u, v, w)
        zeros += want == 0
    assert zeros >= 400


def test_reversal_and_swap_invariance(hc):
    """Reversing either arc or swapping the two arcs negates n_A x n_B and the decision sign
    together, so the reported point is the same; the EFT arithmetic is antisymmetric exactly
    (TwoSum and TwoProduct commute with negation), so the outputs agree bit for bit, and the
    exact oracle agrees on the counts."""
    pairs = special_pairs()[:9] + as_tuples(inputs.arc_pairs(800, seed_tag=63))
    a, b = soa(pairs)
    base = run(hc, 1, a, b)
    variants = {
        "reverse A": (a[3:] + a[:3], b),
        "reverse B": (a, b[3:] + b[:3]),
        "swap": (b, a),
    }
    base_naive = run(hc, 0, a, b)
    for name, (va, vb) in variants.items():
        for mode, ref in ((1, base), (0, base_naive)):
            got = run(hc, mode, va, vb)
            for g_, r_ in zip(got, ref):
                assert np.array_equal(g_, r_, equal_nan=True), (name, mode)
    for a1, a2, b1, b2 in pairs[:200]:
        assert AA.classify(a2, a1, b1, b2)[0] == AA.classify(a1, a2, b1, b2)[0]
        assert AA.classify(b1, b2, a1, a2)[0] == AA.classify(a1, a2, b1, b2)[0]
