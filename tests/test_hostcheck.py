"""The kernels' per-pair arithmetic, compiled for the CPU, against the oracle.

libsphint_hostcheck.so is built from the same header the GPU kernels use (only the way
undecided exact predicates are scheduled differs), so these CPU tests pin the operation
sequence before any GPU run:

* EFT mode: hit counts, roots and flags equal the exact oracle; points equal the oracle's
  binary64 AccuX replica bit for bit and lie within 4 * 2^-53 of the exact points.
* naive mode: everything equals the oracle's binary64 Eq. (2.2) replica bit for bit.
* the exact expansion predicates equal the oracle's integer predicates, including exact
  ties and values far below any filter's reach.
"""

import ctypes
import itertools
import math
import os
from decimal import Decimal

import numpy as np
import pytest

from oracle import batch as OB, geometry as G, naive as ON
from paper_2510_09892_amd import inputs

U = 2.0 ** -53
# SPHINT_HOSTCHECK_LIB selects another build of the same sources (e.g. the sanitizer build)
LIBPATH = os.environ.get("SPHINT_HOSTCHECK_LIB") or os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2510_09892_amd",
    "libsphint_hostcheck.so")
FLAG_MASK = 31  # EXISTS | TANGENT | DEGEN_N | HORIZ | NONFINITE (diagnostic bits excluded)


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIBPATH):
        pytest.fail("libsphint_hostcheck.so is not built (python -m paper_2510_09892_amd.build)")
    lib = ctypes.CDLL(LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_eval.argtypes = [ctypes.c_int, ctypes.c_int64] + [dp] * 7 + [ip] * 4 + [dp] * 4
    lib.sphint_hostcheck_exact_sign.argtypes = [ctypes.c_int] + [ctypes.c_double] * 7
    lib.sphint_hostcheck_exact_sign.restype = ctypes.c_int
    return lib


def run(hc, mode, soa):
    soa = [np.ascontiguousarray(a, dtype=np.float64) for a in soa]
    n = len(soa[0])
    ints = [np.zeros(n, np.int32) for _ in range(4)]
    dbl = [np.zeros(n, np.float64) for _ in range(4)]
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    hc.sphint_hostcheck_eval(mode, n, *[dp(a) for a in soa], *[ip(a) for a in ints],
                             *[dp(a) for a in dbl])
    count, flags, r0, r1 = ints
    px0, py0, px1, py1 = dbl
    return count, flags, r0, r1, px0, py0, px1, py1


def compare_eft(hc, soa, check_points=True):
    count, flags, r0, r1, px0, py0, px1, py1 = run(hc, 1, soa)
    ex = OB.exact(*soa)
    np.testing.assert_array_equal(count, ex.count)
    np.testing.assert_array_equal(flags & FLAG_MASK, ex.flags)
    worst = 0.0
    if not check_points:
        return worst
    rep = OB.accux_points(*soa, ex.roots)
    k = 0
    for i in range(len(count)):
        roots = ex.roots[i]
        got = [(r0[i], px0[i], py0[i]), (r1[i], px1[i], py1[i])][:count[i]]
        assert tuple(g[0] for g in got) == roots, i
        for j, (r, x, y) in enumerate(got):
            assert (x, y) == rep[i][j], (i, j, (x, y), rep[i][j])
            e = max(abs(Decimal(x) - ex.hit_x[k]), abs(Decimal(y) - ex.hit_y[k])) / Decimal(U)
            worst = max(worst, float(e))
            k += 1
    return worst


def compare_naive(hc, soa):
    count, flags, r0, r1, px0, py0, px1, py1 = run(hc, 0, soa)
    ref = OB.naive_fp64(*soa)
    np.testing.assert_array_equal(count, ref.count)
    np.testing.assert_array_equal(flags, ref.flags)
    k = 0
    for i in range(len(count)):
        got = [(r0[i], px0[i], py0[i]), (r1[i], px1[i], py1[i])][:count[i]]
        for r, x, y in got:
            assert r == ref.hit_root[k] and x == ref.hit_x[k] and y == ref.hit_y[k], i
            k += 1


# ----------------------------------------------------------------- workloads

def test_eft_uniform_arcs(hc):
    P = inputs.uniform_arcs(3000, seed_tag=40)
    assert compare_eft(hc, P.soa()) <= 4.0


def test_eft_ill_conditioned(hc):
    P = inputs.ill_conditioned(3000, seed_tag=41)
    assert compare_eft(hc, P.soa()) <= 4.0


def test_naive_bit_exact(hc):
    compare_naive(hc, inputs.uniform_arcs(2000, seed_tag=42).soa())
    compare_naive(hc, inputs.ill_conditioned(2000, seed_tag=43).soa())


# ----------------------------------------------------------------- exact decisions

def _integer_cases():
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0), repeat=3) if any(v)]
    rows = []
    for x1 in verts:
        for x2 in verts:
            for z0 in (-1.0, -0.5, 0.0, 0.375, 1.0, 0.7071067811865476):
                rows.append((*x1, *x2, z0))
    a = np.array(rows)
    return [a[:, k].copy() for k in range(7)]


def test_eft_exact_ties_integer_arcs(hc):
    """Endpoint ties, pole tangencies, apex endpoints, DEGEN/HORIZ: exact decisions."""
    soa = _integer_cases()
    compare_eft(hc, soa)
    compare_naive(hc, soa)
    count, flags, *_ = run(hc, 1, soa)
    assert np.any(flags & 32)       # some decisions needed the exact expansions
    assert np.any(flags & 2)        # tangencies exist in this set


def test_eft_special_values(hc):
    rows = [
        (1.0, 0.0, 0.0, 0.0, 1.0, 1.0, math.nan),
        (math.inf, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0),
        (0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0),
        (1.0, 2.0, 3.0, 2.0, 4.0, 6.0, 0.5),
        (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0),
        (1.0, 0.0, -1.0, 0.0, 1.0, 1.0, 1.5),
        (1.0, 0.0, 3.0, -1.0, 0.0, 2.0, 1.0),
        (1e-3, 2e-3, 1.0, -1e-3, 1e-3, 1.0, 1.0),
    ]
    a = np.array(rows)
    soa = [a[:, k].copy() for k in range(7)]
    compare_eft(hc, soa)
    compare_naive(hc, soa)


def test_eft_near_ties(hc):
    """Latitudes one ulp around exact endpoint heights and around the apex: the filters
    must hand undecidable cases to the expansions, never certify a wrong sign."""
    g = np.random.Generator(np.random.PCG64(44))
    rows = []
    for _ in range(300):
        # an endpoint with a power-of-two-scaled exact unit direction: height exactly 0.6
        k = 2.0 ** int(g.integers(-3, 4))
        c, s = math.cos(g.uniform(0, 2 * math.pi)), math.sin(g.uniform(0, 2 * math.pi))
        x1 = (0.8 * k * c, 0.8 * k * s, 0.6 * k)
        x2 = tuple(float(v) for v in g.standard_normal(3))
        zh = x1[2] / math.sqrt(x1[0] ** 2 + x1[1] ** 2 + x1[2] ** 2)
        for z0 in (zh, math.nextafter(zh, 2), math.nextafter(zh, -2), 0.6):
            rows.append((*x1, *x2, z0))
    P = inputs.ill_conditioned(600, seed_tag=45)
    for i in np.flatnonzero(P.part == 1):
        t = G.exact_terms(tuple(P.p1[i]), tuple(P.p2[i]), float(P.z0[i]))
        zmax = math.sqrt(t["S2"] / t["S3"])
        for z0 in (zmax, math.nextafter(zmax, 2), math.nextafter(zmax, -2)):
            rows.append((*P.p1[i], *P.p2[i], math.copysign(z0, P.z0[i])))
    a = np.array(rows)
    soa = [a[:, k].copy() for k in range(7)]
    compare_eft(hc, soa, check_points=True)


def test_exact_sign_matches_oracle(hc):
    """exact_sign (expansion arithmetic) equals the integer predicates, near zero too."""
    g = np.random.Generator(np.random.PCG64(46))
    P = inputs.ill_conditioned(300, seed_tag=47)
    cases = []
    for i in range(len(P)):
        cases.append((*map(float, P.p1[i]), *map(float, P.p2[i]), float(P.z0[i])))
    for _ in range(200):
        v = [float(x) for x in g.standard_normal(7)]
        v[6] = float(g.uniform(-1, 1))
        cases.append(tuple(v))
    cases += [tuple(r) for r in np.array(_integer_cases()).T[::7]]
    for v in cases:
        x1, x2, z0 = v[:3], v[3:6], v[6]
        t = G.exact_terms(x1, x2, z0)
        K = t["K"]
        sg = lambda q: (q > 0) - (q < 0)
        assert hc.sphint_hostcheck_exact_sign(0, *v) == sg(t["s2"]), v
        assert hc.sphint_hostcheck_exact_sign(1, *v) == sg(t["Nx"] * t["Y1"] - t["Ny"] * t["X1"]), v
        assert hc.sphint_hostcheck_exact_sign(2, *v) == sg(t["Nx"] * t["Y2"] - t["Ny"] * t["X2"]), v
        for which, (X, Y, Z) in ((3, ("X1", "Y1", "Z1")), (4, ("X2", "Y2", "Z2"))):
            Xv, Yv, Zv = t[X], t[Y], t[Z]
            want = sg(t["Z0"] ** 2 * (Xv * Xv + Yv * Yv + Zv * Zv) - (Zv * Zv << (2 * K)))
            assert hc.sphint_hostcheck_exact_sign(which, *v) == want, (which, v)


def test_eft_heights_near_pole_within_ulps(hc):
    """Latitudes a few ulps from an endpoint's height near a pole: the first height filter
    leaves these open and the second must decide them correctly (or hand them on)."""
    P = inputs.ill_conditioned(3000, seed_tag=48)
    rows = []
    for i in np.flatnonzero(P.part == 2)[:300]:
        x1 = tuple(float(v) for v in P.p1[i])
        zh = x1[2] / math.sqrt(x1[0] ** 2 + x1[1] ** 2 + x1[2] ** 2)
        z0 = zh
        for _ in range(4):
            z0 = math.nextafter(z0, -2.0)
        for _ in range(9):
            rows.append((*x1, *P.p2[i], z0))
            z0 = math.nextafter(z0, 2.0)
    a = np.array(rows)
    soa = [a[:, k].copy() for k in range(7)]
    compare_eft(hc, soa)


@pytest.mark.parametrize("mode", [1, 0])
def test_metamorphic_relations_bit_exact(hc, mode):
    """Swapping the endpoints reverses the hits and exchanges their labels; mirroring z
    exchanges the labels in place; scaling an endpoint by 8 changes nothing (EFT only: the
    naive mode compares z0 with raw endpoint heights).  Points agree bit for bit: the
    arithmetic commutes with negation and with scaling by powers of two.  A tangency's double
    root may carry either label."""
    for P in (inputs.ill_conditioned(20000, seed_tag=31), inputs.uniform_arcs(20000, seed_tag=32)):
        x1, y1, z1, x2, y2, z2, z0 = P.soa()
        cnt, fl, r0, r1, px0, py0, px1, py1 = run(hc, mode, (x1, y1, z1, x2, y2, z2, z0))
        nt = (fl & 2) == 0
        one, two, hit = cnt == 1, cnt == 2, cnt > 0
        c2, f2, s0, s1, qx0, qy0, qx1, qy1 = run(hc, mode, (x2, y2, z2, x1, y1, z1, z0))
        assert np.array_equal(cnt, c2) and np.array_equal(fl, f2)
        assert np.array_equal(px0[one], qx0[one]) and np.array_equal(py0[one], qy0[one])
        assert np.array_equal(r0[one & nt], 1 - s0[one & nt])
        assert np.array_equal(px0[two], qx1[two]) and np.array_equal(px1[two], qx0[two])
        assert np.array_equal(py0[two], qy1[two]) and np.array_equal(py1[two], qy0[two])
        assert np.array_equal(r0[two], 1 - s1[two]) and np.array_equal(r1[two], 1 - s0[two])
        c3, f3, m0, m1, mx0, my0, mx1, my1 = run(hc, mode, (x1, y1, -z1, x2, y2, -z2, -z0))
        assert np.array_equal(cnt, c3) and np.array_equal(fl, f3)
        assert np.array_equal(px0[hit], mx0[hit]) and np.array_equal(py0[hit], my0[hit])
        assert np.array_equal(px1[two], mx1[two]) and np.array_equal(py1[two], my1[two])
        assert np.array_equal(r0[hit & nt], 1 - m0[hit & nt])
        assert np.array_equal(r1[two], 1 - m1[two])
        if mode == 1:
            # from a factor 8 to factors that move |n_xy|^2 by 2^-600 and 2^600 (nothing
            # underflows or overflows on this workload)
            for k1, k2 in ((3, 0), (-80, -80), (-200, -100), (150, 150), (-120, 60)):
                s1, s2 = 2.0 ** k1, 2.0 ** k2
                scaled = run(hc, mode, (s1 * x1, s1 * y1, s1 * z1, s2 * x2, s2 * y2, s2 * z2, z0))
                for u, v in zip((cnt, fl, r0, r1, px0, py0, px1, py1), scaled):
                    assert np.array_equal(u, v), (k1, k2)
