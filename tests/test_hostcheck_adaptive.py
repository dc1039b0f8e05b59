"""The adaptive evaluation's per-pair arithmetic, compiled for the CPU, against the oracle.

Pass 1 (the direct binary64 evaluation with a running error bound) either accepts a pair or
leaves it to the EFT evaluation.  For every pair:

* counts, roots and flags equal the exact oracle (the certified decisions are the exact
  ones, and the EFT evaluation decides exactly);
* an accepted pair's points equal the oracle's binary64 Eq. 2.2 replica for the same roots
  bit for bit, and lie within tol * 2^-53 (max-norm) of the exact points: the bound is sound;
* a recomputed pair's points equal the oracle's AccuX replica bit for bit (within 4 * 2^-53).
"""

import ctypes
import math
from decimal import Decimal

import numpy as np
import pytest

from oracle import batch as OB, geometry as G, naive as ON
from paper_2510_09892_amd import inputs

import test_hostcheck as TH

U = 2.0 ** -53
FLAG_MASK = 31


@pytest.fixture(scope="module")
def hc():
    lib = ctypes.CDLL(TH.LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_adaptive.argtypes = ([ctypes.c_int64] + [dp] * 7 + [ctypes.c_double] +
                                              [ip] * 4 + [dp] * 4 + [ip])
    return lib


def run_adaptive(hc, soa, tol):
    soa = [np.ascontiguousarray(a, dtype=np.float64) for a in soa]
    n = len(soa[0])
    ints = [np.zeros(n, np.int32) for _ in range(4)]
    dbl = [np.zeros(n, np.float64) for _ in range(4)]
    cert = np.zeros(n, np.int32)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    hc.sphint_hostcheck_adaptive(n, *[dp(a) for a in soa], float(tol), *[ip(a) for a in ints],
                                 *[dp(a) for a in dbl], ip(cert))
    return (*ints, *dbl, cert)


def check_adaptive(soa, res, tol):
    """Compares one adaptive result with the oracle; returns (accepted pairs with hits,
    pairs with hits, worst accepted error in u, worst recomputed error in u)."""
    count, flags, r0, r1, px0, py0, px1, py1, cert = res
    ex = OB.exact(*soa)
    np.testing.assert_array_equal(count, ex.count)
    np.testing.assert_array_equal(flags & FLAG_MASK, ex.flags)
    rep = OB.accux_points(*soa, ex.roots)
    worst_acc = worst_rec = 0.0
    acc = tot = 0
    k = 0
    for i in range(len(count)):
        roots = ex.roots[i]
        got = [(r0[i], px0[i], py0[i]), (r1[i], px1[i], py1[i])][:count[i]]
        assert tuple(int(g[0]) for g in got) == roots, i
        if count[i]:
            tot += 1
            acc += bool(cert[i])
        x1 = (soa[0][i], soa[1][i], soa[2][i])
        x2 = (soa[3][i], soa[4][i], soa[5][i])
        for j, (r, x, y) in enumerate(got):
            e = max(abs(Decimal(float(x)) - ex.hit_x[k]),
                    abs(Decimal(float(y)) - ex.hit_y[k])) / Decimal(U)
            if cert[i]:
                assert (x, y) == ON.point(x1, x2, float(soa[6][i]), int(r)), (i, j)
                assert float(e) <= tol, (i, j, float(e), tol)
                worst_acc = max(worst_acc, float(e))
            else:
                assert (x, y) == rep[i][j], (i, j)
                assert float(e) <= 4.0, (i, j, float(e))
                worst_rec = max(worst_rec, float(e))
            k += 1
    return acc, tot, worst_acc, worst_rec


@pytest.mark.parametrize("tol", [4.0, 16.0, 64.0, 1024.0])
def test_uniform_arcs(hc, tol):
    """The bound is worst-case (20-250x the actual error on these arcs), so pass 1 accepts
    few pairs at the EFT's own 4 u and most at 1024 u."""
    soa = inputs.uniform_arcs(3000, seed_tag=46).soa()
    acc, tot, wa, wr = check_adaptive(soa, run_adaptive(hc, soa, tol), tol)
    want = {4.0: 0.0, 16.0: 0.01, 64.0: 0.3, 1024.0: 0.8}[tol]
    assert acc >= want * tot, (acc, tot)


def test_ill_conditioned(hc):
    soa = inputs.ill_conditioned(3000, seed_tag=47).soa()
    check_adaptive(soa, run_adaptive(hc, soa, 16.0), 16.0)


def test_exact_ties_and_special_values(hc):
    """Endpoint ties, pole tangencies, apex endpoints and degenerate arcs are never
    certified by pass 1 unless their decisions are clear."""
    soa = TH._integer_cases()
    res = run_adaptive(hc, soa, 64.0)
    check_adaptive(soa, res, 64.0)
    rows = [
        (1.0, 0.0, 0.0, 0.0, 1.0, 1.0, math.nan),
        (math.inf, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0),
        (0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0),
        (1.0, 2.0, 3.0, 2.0, 4.0, 6.0, 0.5),
        (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0),
        (1.0, 0.0, -1.0, 0.0, 1.0, 1.0, 1.5),
        (1.0, 0.0, 3.0, -1.0, 0.0, 2.0, 1.0),
        (1e-3, 2e-3, 1.0, -1e-3, 1e-3, 1.0, 1.0),
        (1e40, 1e40, 1.0, -1e40, 1e40, 1.0, 0.5),
    ]
    a = np.array(rows)
    soa = [a[:, k].copy() for k in range(7)]
    check_adaptive(soa, run_adaptive(hc, soa, 64.0), 64.0)


def test_near_ties_and_near_tangency(hc):
    """Latitudes one ulp around endpoint heights and around the great circle's top, where
    the direct evaluation's decisions are least reliable."""
    g = np.random.Generator(np.random.PCG64(48))
    rows = []
    for _ in range(200):
        k = 2.0 ** int(g.integers(-3, 4))
        c, s = math.cos(g.uniform(0, 2 * math.pi)), math.sin(g.uniform(0, 2 * math.pi))
        x1 = (0.8 * k * c, 0.8 * k * s, 0.6 * k)
        x2 = tuple(float(v) for v in g.standard_normal(3))
        zh = x1[2] / math.sqrt(x1[0] ** 2 + x1[1] ** 2 + x1[2] ** 2)
        for z0 in (zh, math.nextafter(zh, 2), math.nextafter(zh, -2), 0.6):
            rows.append((*x1, *x2, z0))
    P = inputs.uniform_arcs(400, seed_tag=49)
    for i in range(len(P)):
        t = G.exact_terms(tuple(P.p1[i]), tuple(P.p2[i]), float(P.z0[i]))
        zmax = math.sqrt(t["S2"] / t["S3"])
        for z0 in (zmax, zmax * (1 - 1e-9), zmax * (1 - 1e-6), zmax * (1 - 1e-3)):
            rows.append((*P.p1[i], *P.p2[i], z0))
    a = np.array(rows)
    soa = [a[:, k].copy() for k in range(7)]
    for tol in (4.0, 64.0):
        check_adaptive(soa, run_adaptive(hc, soa, tol), tol)


def test_zero_tolerance_recomputes_every_hit(hc):
    soa = inputs.uniform_arcs(500, seed_tag=50).soa()
    res = run_adaptive(hc, soa, 0.0)
    acc, tot, _, _ = check_adaptive(soa, res, 0.0)
    assert acc == 0 and tot > 0
