"""GPU: metamorphic relations of the main path at 1e6 pairs, exact to the bit.

The EFT arithmetic commutes with negation and with scaling by powers of two (TwoSum,
TwoProduct and every rounding do), so, pair by pair:

* swapping an arc's endpoints negates n: the same points come back in the reverse order
  with the root labels exchanged (away from tangency, where the double root's label is a
  convention), bit for bit, and the same count and flags;
* scaling an endpoint by 8 changes nothing at all;
* mirroring z -> -z (and z0 -> -z0) keeps (x, y), keeps the order and exchanges the labels.

These hold at any size without the oracle, so they check the full-size launches
configuration by configuration (dense ill-conditioned and uniform inputs, both modes where
the relation is exact for the mode's arithmetic).
"""

import os
import sys

import numpy as np
import pytest

from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import gpu_dense  # noqa: E402


def note(msg):
    print(f"[gpu-metamorphic] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def per_pair(res):
    """(first hit offset, count) per pair from the compacted output."""
    c = res["count"].astype(np.int64)
    off = np.zeros(len(c), np.int64)
    np.cumsum(c[:-1], out=off[1:])
    return off, c


def same_per_pair(a, b, reverse, swap_labels):
    oa, ca = per_pair(a)
    ob, cb = per_pair(b)
    assert np.array_equal(ca, cb)
    assert np.array_equal(a["flags"], b["flags"])
    one = ca == 1
    two = ca == 2
    for sel, ia, ib in ((one, oa[one], ob[one]),
                        (two, oa[two], (ob[two] + 1) if reverse else ob[two]),
                        (two, oa[two] + 1, ob[two] if reverse else ob[two] + 1)):
        assert np.array_equal(a["x"][ia], b["x"][ib])
        assert np.array_equal(a["y"][ia], b["y"][ib])
        # a tangency's double root carries either label (a convention of the rule), so the
        # label relation is checked away from tangency
        keep = (a["flags"][sel] & 2) == 0
        ra, rb = a["root"][ia][keep], b["root"][ib][keep]
        assert np.array_equal(ra, (1 - rb) if swap_labels else rb)


@pytest.mark.parametrize("workload", ["ill", "uniform"])
def test_endpoint_swap_scale_and_mirror(torch_cuda, workload):
    P = (inputs.ill_conditioned(1_000_000, seed_tag=31) if workload == "ill"
         else inputs.uniform_arcs(1_000_000, seed_tag=32))
    x1, y1, z1, x2, y2, z2, z0 = P.soa()
    for mode in ("eft", "naive"):
        note(f"{workload} {mode}: base, swapped, scaled, mirrored")
        base = gpu_dense(torch_cuda, (x1, y1, z1, x2, y2, z2, z0), mode)
        swapped = gpu_dense(torch_cuda, (x2, y2, z2, x1, y1, z1, z0), mode)
        if mode == "eft":  # the naive mode compares z0 with the raw endpoint heights, so a
            # scaled endpoint changes its decisions; swapping and mirroring are exact for both
            scaled = gpu_dense(torch_cuda, (8 * x1, 8 * y1, 8 * z1, x2, y2, z2, z0), mode)
            same_per_pair(base, scaled, reverse=False, swap_labels=False)
        mirrored = gpu_dense(torch_cuda, (x1, y1, -z1, x2, y2, -z2, -z0), mode)
        same_per_pair(base, swapped, reverse=True, swap_labels=True)
        same_per_pair(base, mirrored, reverse=False, swap_labels=True)
