"""CSR lists evaluated with the arc part shared (the batched kernels' shared path),
compiled for the CPU, against the per-pair evaluation of the same pairs.

Everything of Alg. 8 before the latitude enters, and the slope signs of the containment
rule (Sec. 2), depends on the arc alone; the shared path computes it once per arc and
evaluates every candidate from that record.  The results must equal the per-pair
evaluation (itself pinned to the oracle in test_hostcheck.py) bit for bit, counts, roots,
points and every flag bit, including the exact fallback's diagnostic bit: on random meshes,
on arcs whose slope or height decisions are exact ties (integer endpoints, apex endpoints,
latitudes one ulp around endpoint heights and great-circle tops), on degenerate and
non-finite arcs, on latitude indices outside the table, and on arcs without candidates.
"""

import ctypes
import itertools
import math

import numpy as np
import pytest

from paper_2510_09892_amd import inputs
import test_hostcheck as TH

dp = ctypes.POINTER(ctypes.c_double)
ip = ctypes.POINTER(ctypes.c_int32)
lp = ctypes.POINTER(ctypes.c_int64)


@pytest.fixture(scope="module")
def hc():
    lib = ctypes.CDLL(TH.LIBPATH)
    lib.sphint_hostcheck_eval.argtypes = [ctypes.c_int, ctypes.c_int64] + [dp] * 7 + [ip] * 4 + [dp] * 4
    lib.sphint_hostcheck_eval_shared.argtypes = ([ctypes.c_int64] + [dp] * 6 + [dp, ctypes.c_int64, lp, ip]
                                                 + [ip] * 4 + [dp] * 4 + [lp])
    return lib


def run_shared(hc, ends, lat_z, off, idx):
    ends = [np.ascontiguousarray(a, dtype=np.float64) for a in ends]
    lat_z = np.ascontiguousarray(lat_z, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    nnz = int(off[-1])
    ints = [np.zeros(nnz, np.int32) for _ in range(4)]
    dbl = [np.zeros(nnz, np.float64) for _ in range(4)]
    opened = np.zeros(1, np.int64)
    hc.sphint_hostcheck_eval_shared(len(ends[0]), *[a.ctypes.data_as(dp) for a in ends],
                                    lat_z.ctypes.data_as(dp), len(lat_z), off.ctypes.data_as(lp),
                                    idx.ctypes.data_as(ip), *[a.ctypes.data_as(ip) for a in ints],
                                    *[a.ctypes.data_as(dp) for a in dbl], opened.ctypes.data_as(lp))
    return (*ints, *dbl), int(opened[0])


def expand(ends, lat_z, off, idx):
    arc = np.repeat(np.arange(len(ends[0])), np.diff(off))
    ok = (idx >= 0) & (idx < len(lat_z))
    z0 = np.where(ok, lat_z[np.where(ok, idx, 0)], np.nan)
    return [np.asarray(e, np.float64)[arc] for e in ends] + [z0]


def check_same(hc, ends, lat_z, off, idx):
    got, opened = run_shared(hc, ends, lat_z, off, idx)
    want = TH.run(hc, 1, expand(ends, lat_z, off, idx))
    names = ("count", "flags", "r0", "r1", "px0", "py0", "px1", "py1")
    for n, g, w in zip(names, got, want):
        assert np.array_equal(np.asarray(g).view(np.uint8), np.asarray(w).view(np.uint8)), n
    return got, opened


def mesh_arrays(m):
    return m.soa(), m.lat_z, m.lat_offsets, m.lat_idx


def test_random_meshes_equal_per_pair(hc):
    for k, (n_arcs, n_lat) in enumerate([(500, 40), (2000, 400), (300, 3000)]):
        m = inputs.random_mesh(inputs.rng(90, k), n_arcs, n_lat)
        got, _ = check_same(hc, *mesh_arrays(m))
        assert got[0].sum() > 0


def _csr(arcs, lats_per_arc):
    """arcs: list of (x1, y1, z1, x2, y2, z2); lats_per_arc: list of latitude lists (may be
    empty).  One shared latitude table; indices point into it."""
    table = sorted({float(z) for zs in lats_per_arc for z in zs if not math.isnan(z)})
    pos = {z: i for i, z in enumerate(table)}
    off = [0]
    idx = []
    for zs in lats_per_arc:
        for z in zs:
            idx.append(-1 if math.isnan(z) else pos[float(z)])
        off.append(len(idx))
    a = np.array(arcs, np.float64).reshape(-1, 6)
    return [a[:, k].copy() for k in range(6)], np.array(table), np.array(off), np.array(idx, np.int32)


def test_exact_ties_equal_per_pair(hc):
    """Integer endpoints (slope ties at apex endpoints, endpoint-height ties, tangencies,
    DEGEN / HORIZ arcs) with latitudes at the tie values and one ulp around them."""
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0), repeat=3) if any(v)]
    zs = []
    for z in (-1.0, -0.5, 0.0, 0.375, 1.0, 0.7071067811865476, 0.5773502691896258):
        zs += [z, math.nextafter(z, 2.0), math.nextafter(z, -2.0)]
    arcs, lats = [], []
    for x1 in verts:
        for x2 in verts:
            arcs.append((*x1, *x2))
            lats.append(zs)
    got, opened = check_same(hc, *_csr(arcs, lats))
    assert opened > 0                   # some slope filters were open (exact signs per arc)
    assert np.any(got[1] & 32)          # some pairs took the exact fallback
    assert np.any(got[1] & 2)           # tangencies
    assert np.any(got[1] & 4) and np.any(got[1] & 8)  # degenerate and horizontal arcs


def test_near_ties_and_special_values_equal_per_pair(hc):
    """Endpoint heights exactly 0.6 with latitudes one ulp around them, great-circle tops
    one ulp around, near-pole arcs a few ulps around their endpoint heights, non-finite
    endpoints, latitude indices outside the table, and arcs without candidates."""
    g = np.random.Generator(np.random.PCG64(91))
    arcs, lats = [], []
    for _ in range(200):
        k = 2.0 ** int(g.integers(-3, 4))
        c, s = math.cos(g.uniform(0, 2 * math.pi)), math.sin(g.uniform(0, 2 * math.pi))
        x1 = (0.8 * k * c, 0.8 * k * s, 0.6 * k)
        x2 = tuple(float(v) for v in g.standard_normal(3))
        zh = x1[2] / math.sqrt(x1[0] ** 2 + x1[1] ** 2 + x1[2] ** 2)
        arcs.append((*x1, *x2))
        lats.append([zh, math.nextafter(zh, 2), math.nextafter(zh, -2), 0.6, 0.0, -0.3])
    P = inputs.ill_conditioned(900, seed_tag=92)
    from oracle import geometry as G
    for i in np.flatnonzero(P.part == 1)[:150]:
        t = G.exact_terms(tuple(P.p1[i]), tuple(P.p2[i]), float(P.z0[i]))
        zmax = math.copysign(math.sqrt(t["S2"] / t["S3"]), P.z0[i])
        arcs.append((*P.p1[i], *P.p2[i]))
        lats.append([zmax, math.nextafter(zmax, 2), math.nextafter(zmax, -2), float(P.z0[i])])
    for i in np.flatnonzero(P.part == 2)[:150]:
        x1 = tuple(float(v) for v in P.p1[i])
        zh = x1[2] / math.sqrt(x1[0] ** 2 + x1[1] ** 2 + x1[2] ** 2)
        z = zh
        for _ in range(4):
            z = math.nextafter(z, -2.0)
        zz = []
        for _ in range(9):
            zz.append(z)
            z = math.nextafter(z, 2.0)
        arcs.append((*x1, *P.p2[i]))
        lats.append(zz)
    # special arcs, arcs without candidates, invalid latitude indices
    arcs += [(math.inf, 0, 0, 0, 1, 1), (0, 0, 0, 0, 1, 1), (1, 2, 3, 2, 4, 6), (1, 0, 0, 0, 1, 0),
             (1e-3, 2e-3, 1.0, -1e-3, 1e-3, 1.0), (1, 0, -1, 0, 1, 1), (0.3, 0.2, 0.1, -0.2, 0.4, 0.3)]
    lats += [[0.0, 0.5], [0.0], [0.5], [0.0, 0.1], [1.0, 0.9999999], [], [0.2, math.nan, 0.25]]
    ends, table, off, idx = _csr(arcs, lats)
    idx = idx.copy()
    idx[idx == -1] = len(table) + 5     # outside the table: z0 = NaN
    got, _ = check_same(hc, ends, table, off, idx)
    assert np.any(got[1] & 16)          # non-finite inputs flagged
    assert np.any(got[0] == 2)          # two-hit pairs (both roots from the shared record)


def test_sparse_rows_equal_per_pair(hc):
    """Most arcs without candidates: rows span many arc ids (the shared path's own-arc
    case on the GPU; the arithmetic is the same)."""
    m = inputs.random_mesh(inputs.rng(93), 5000, 12, d_hi=0.01)
    got, _ = check_same(hc, *mesh_arrays(m))
    assert (np.diff(m.lat_offsets) == 0).mean() > 0.5
