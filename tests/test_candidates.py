"""Candidate latitude lists (the step before the intersection path), host build of the rule.

The rule (sphint_cand.hpp, compiled for the CPU here) must return, for every arc, a range
of the ascending latitude table that
* contains every latitude the arc meets, by the exact oracle (the classification of Sec. 2
  evaluated in integers): no intersection is lost before the intersection step;
* reaches no further than the slack beyond the arc's exact height range, computed from the
  exact slope signs and 100-digit heights.
The GPU kernels are compared with this host build in tests/test_gpu_candidates.py.
"""

import ctypes
import math
import os
from decimal import Decimal, localcontext

import numpy as np
import pytest

from oracle import batch as OB, geometry as G
from paper_2510_09892_amd import inputs

# SPHINT_HOSTCHECK_LIB selects another build of the same sources (e.g. the sanitizer build)
LIBPATH = os.environ.get("SPHINT_HOSTCHECK_LIB") or os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2510_09892_amd",
    "libsphint_hostcheck.so")
SLACK = 2.0 ** -46


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIBPATH):
        pytest.fail("libsphint_hostcheck.so is not built (python -m paper_2510_09892_amd.build)")
    lib = ctypes.CDLL(LIBPATH)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_candidates.argtypes = ([ctypes.c_int64] + [dp] * 6 + [dp, ctypes.c_int32,
                                                ctypes.c_double, ip, ip])
    return lib


def host_candidates(hc, p1, p2, lat_z, pad=0.0):
    soa = [np.ascontiguousarray(a, dtype=np.float64) for a in
           (p1[:, 0], p1[:, 1], p1[:, 2], p2[:, 0], p2[:, 1], p2[:, 2])]
    lz = np.ascontiguousarray(lat_z, dtype=np.float64)
    n = len(p1)
    first = np.zeros(n, np.int32)
    count = np.zeros(n, np.int32)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    hc.sphint_hostcheck_candidates(n, *[dp(a) for a in soa], dp(lz), len(lz), pad, ip(first),
                                   ip(count))
    return first, count


def exact_range(x1, x2):
    """The arc's exact height range [lo, hi] (Decimal): endpoint heights, extended to the top
    (bottom) of the great circle when the exact slope signs put it inside the arc."""
    t = G.exact_terms(tuple(x1), tuple(x2), 0.0)
    with localcontext() as ctx:
        ctx.prec = 60
        h = []
        for X, Y, Z in ((t["X1"], t["Y1"], t["Z1"]), (t["X2"], t["Y2"], t["Z2"])):
            h.append(Decimal(Z) / (Decimal(X * X + Y * Y + Z * Z)).sqrt())
        lo, hi = min(h), max(h)
        if t["S2"] > 0:
            sg = lambda v: (v > 0) - (v < 0)
            d1 = sg(t["Nx"] * t["Y1"] - t["Ny"] * t["X1"])
            d2 = sg(t["Nx"] * t["Y2"] - t["Ny"] * t["X2"])
            zmax = (Decimal(t["S2"]) / Decimal(t["S3"])).sqrt()
            if d1 > 0 > d2:
                hi = zmax
            if d1 < 0 < d2:
                lo = -zmax
    return lo, hi


def workload():
    g = inputs.rng(60)
    parts = [inputs.uniform_arcs(40, seed_tag=61), inputs.ill_conditioned(60, seed_tag=62)]
    p1 = np.concatenate([P.p1 for P in parts])
    p2 = np.concatenate([P.p2 for P in parts])
    lat = list(np.sin(np.deg2rad(np.linspace(-89.9, 89.9, 160))))
    # latitudes exactly at (rounded) endpoint heights and great-circle tops, and 1 ulp around
    for i in range(len(p1)):
        lo, hi = exact_range(p1[i], p2[i])
        for v in (float(lo), float(hi)):
            lat += [v, math.nextafter(v, 2.0), math.nextafter(v, -2.0)]
    lat = np.unique(np.array([v for v in lat if -1.0 <= v <= 1.0]))
    return p1, p2, lat


def test_candidates_contain_every_intersection(hc):
    p1, p2, lat = workload()
    first, count = host_candidates(hc, p1, p2, lat)
    n, L = len(p1), len(lat)
    a = np.repeat(np.arange(n), L)
    k = np.tile(np.arange(L), n)
    ex = OB.exact(p1[a, 0], p1[a, 1], p1[a, 2], p2[a, 0], p2[a, 1], p2[a, 2], lat[k])
    hit = ex.count.reshape(n, L) > 0
    inside = (np.arange(L)[None, :] >= first[:, None]) & (np.arange(L)[None, :] < (first + count)[:, None])
    missed = hit & ~inside
    assert not missed.any(), np.argwhere(missed)[:5]
    assert hit.sum() > 100  # the workload does intersect


def test_candidates_stay_within_the_slack(hc):
    p1, p2, lat = workload()
    pad = 1e-9
    first, count = host_candidates(hc, p1, p2, lat, pad)
    tol = Decimal(pad + SLACK) + Decimal(1e-15)
    for i in range(len(p1)):
        lo, hi = exact_range(p1[i], p2[i])
        for k in range(first[i], first[i] + count[i]):
            z = Decimal(float(lat[k]))
            assert lo - tol <= z <= hi + tol, (i, k)


def test_candidates_degenerate_and_nonfinite(hc):
    p1 = np.array([[1.0, 0.0, 0.0], [np.nan, 0.0, 1.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    p2 = np.array([[2.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]])
    lat = np.array([-0.5, 0.0, 0.5, 1.0])
    first, count = host_candidates(hc, p1, p2, lat)
    assert count[1] == 0                          # non-finite: no candidates
    assert list(range(first[0], first[0] + count[0])) == [1]   # coincident points at z = 0
    assert list(range(first[2], first[2] + count[2])) == [3]   # both endpoints at the pole
    assert list(range(first[3], first[3] + count[3])) == [1]   # an arc on the equator
