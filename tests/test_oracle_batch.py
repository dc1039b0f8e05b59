"""The oracle's array drivers agree with its per-pair functions (ordering, compaction)."""

import numpy as np

from oracle import batch, geometry as G, naive, eft
from paper_2510_09892_amd import inputs


def test_batch_matches_per_pair():
    P = inputs.uniform_arcs(400, seed_tag=31)
    soa = P.soa()
    ex = batch.exact(*soa, workers=2)
    nv = batch.naive_fp64(*soa, workers=1)
    k = 0
    for i in range(len(P)):
        x1, x2, z0 = tuple(map(float, P.p1[i])), tuple(map(float, P.p2[i])), float(P.z0[i])
        c, pts = G.intersect(x1, x2, z0)
        assert ex.count[i] == c.count and ex.flags[i] == c.flags and ex.roots[i] == c.roots
        for r, p in zip(c.roots, pts):
            assert ex.hit_pair[k] == i and ex.hit_root[k] == r and (ex.hit_x[k], ex.hit_y[k]) == p
            k += 1
        cnt, roots, flags, npts = naive.intersect(x1, x2, z0)
        assert nv.count[i] == cnt and nv.flags[i] == flags
    assert k == ex.total
    pts = batch.accux_points(*soa, ex.roots, workers=2)
    for i in range(0, len(P), 37):
        for r, p in zip(ex.roots[i], pts[i]):
            assert p == eft.accux(tuple(P.p1[i]), tuple(P.p2[i]), float(P.z0[i]),
                                  1 if r == G.PLUS else -1)
