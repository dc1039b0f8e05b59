"""Array drivers over the oracle (test infrastructure only).

Arrays are SoA binary64 numpy arrays: p1 = (x1, y1, z1), p2 = (x2, y2, z2), one z0 per
pair.  Outputs follow the library's order: per pair, hits in along-arc order; compacted
hits are listed by pair index then along-arc order.  Work is spread over host processes
with ``multiprocessing`` (pure functions, no shared state).
"""

from __future__ import annotations

import os
from multiprocessing import get_context

import numpy as np

from . import geometry, eft, naive


def default_workers() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def _rows(x1, y1, z1, x2, y2, z2, z0):
    cols = [np.asarray(a, dtype=np.float64).tolist() for a in (x1, y1, z1, x2, y2, z2, z0)]
    return list(zip(*cols))


def _exact_chunk(rows):
    out = []
    for (a, b, c, d, e, f, z) in rows:
        cl, pts = geometry.intersect((a, b, c), (d, e, f), z)
        out.append((cl.count, cl.roots, cl.flags, pts))
    return out


def _naive_chunk(rows):
    out = []
    for (a, b, c, d, e, f, z) in rows:
        out.append(naive.intersect((a, b, c), (d, e, f), z))
    return out


def _eft_chunk(jobs):
    out = []
    for (a, b, c, d, e, f, z, roots) in jobs:
        if not roots:
            out.append([])
            continue
        q = eft.accux_parts((a, b, c), (d, e, f), z)
        pts = []
        for r in roots:
            x, y = eft.accux_numerators(q, z, 1 if r == geometry.PLUS else -1)
            pts.append((-(x / q["S2"]), -(y / q["S2"])))
        out.append(pts)
    return out


def _map(fn, items, workers, chunk=256):
    if workers is None:
        workers = default_workers()
    chunks = [items[i:i + chunk] for i in range(0, len(items), chunk)]
    if workers <= 1 or len(chunks) <= 1:
        res = [fn(c) for c in chunks]
    else:
        with get_context("fork").Pool(workers) as pool:
            res = pool.map(fn, chunks)
    return [r for part in res for r in part]


class Result:
    """Per-pair counts/flags plus compacted hits (pair, root, Px, Py)."""

    def __init__(self, n, per_pair):
        self.count = np.zeros(n, dtype=np.uint8)
        self.flags = np.zeros(n, dtype=np.uint8)
        self.roots = []
        self.hit_pair, self.hit_root, self.hit_x, self.hit_y = [], [], [], []
        for i, (cnt, roots, flg, pts) in enumerate(per_pair):
            self.count[i] = cnt
            self.flags[i] = flg
            self.roots.append(roots)
            for r, (px, py) in zip(roots, pts):
                self.hit_pair.append(i)
                self.hit_root.append(r)
                self.hit_x.append(px)
                self.hit_y.append(py)

    @property
    def total(self):
        return len(self.hit_pair)


def exact(x1, y1, z1, x2, y2, z2, z0, workers=None) -> Result:
    """Exact hit counts, flags and 100-digit points for every pair."""
    rows = _rows(x1, y1, z1, x2, y2, z2, z0)
    return Result(len(rows), _map(_exact_chunk, rows, workers))


def naive_fp64(x1, y1, z1, x2, y2, z2, z0, workers=None) -> Result:
    """The direct binary64 evaluation (counts, flags, float points) for every pair."""
    rows = _rows(x1, y1, z1, x2, y2, z2, z0)
    return Result(len(rows), _map(_naive_chunk, rows, workers))


def accux_points(x1, y1, z1, x2, y2, z2, z0, roots_per_pair, workers=None):
    """Alg. 8 binary64 points for the given root labels of each pair (list of lists)."""
    rows = _rows(x1, y1, z1, x2, y2, z2, z0)
    jobs = [r + (tuple(rt),) for r, rt in zip(rows, roots_per_pair)]
    return _map(_eft_chunk, jobs, workers)


# ------------------------------------------------------------------ arc x arc

def _arcarc_chunk(rows):
    from . import arcarc
    out = []
    for (a1, a2, b1, b2) in rows:
        count, flags, p = arcarc.intersect(a1, a2, b1, b2)
        out.append((count, flags, p))
    return out


def arcarc_exact(a1, a2, b1, b2, workers=None):
    """The arc x arc oracle over (n, 3) endpoint arrays: [(count, flags, point or None)]."""
    rows = list(zip(*(map(tuple, np.asarray(v, dtype=np.float64).tolist())
                      for v in (a1, a2, b1, b2))))
    return _map(_arcarc_chunk, rows, workers)
