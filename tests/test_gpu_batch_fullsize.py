"""GPU: the batched launch at the full 64-mesh size, against per-mesh calls and the oracle.

64 meshes with log-uniform 1e3..1e7 arcs (arc length U[1e-3, 0.05] rad) and U{10..3600}
uniformly spaced latitudes, as the batch benchmark draws them, about 8e8 candidate pairs.
The arcs are drawn on the device (torch's seeded generator) and the CSR lists are built by
the library's own candidate kernels, so the whole set is ready in seconds; the benchmark's
host-built lists differ only by extra edge candidates.  Checks, in the benchmark's launch
configuration (one autotuned persistent graph launch):

* every mesh's output equals that mesh's single call bit for bit (compared on the device),
  and in EFT mode also the per-pair schedule's (the autotuned launch and the single calls
  share arc records on dense candidate lists);
* 400 pairs sampled across the meshes match the exact oracle (counts, roots, flags) and the
  AccuX replica (points, within 4 * 2^-53).
"""

from decimal import Decimal

import numpy as np
import pytest

from oracle import batch as OB
from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def note(msg):
    print(f"[gpu-batch-full] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


@pytest.fixture(scope="module")
def meshes(torch_cuda):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    out = inputs.device_mesh_arcs(torch, 64, seed_tag=3)
    for m in out:
        m["lat_offsets"], m["lat_idx"] = sphint.candidates(m["p1"], m["p2"], m["lat_z"])
        m["out"] = sphint.Output(len(m["lat_idx"]))
    torch.cuda.synchronize()
    note(f"64 meshes: {sum(len(m['p1'][0]) for m in out)} arcs, "
         f"{sum(len(m['lat_idx']) for m in out)} pairs")
    return out


@pytest.mark.parametrize("mode", ["eft", "naive"])
def test_full_batch_equals_per_mesh_and_sampled_oracle(torch_cuda, meshes, mode):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    plan = sphint.BatchPlan(meshes, mode=mode)
    try:
        plan.autotune()
        note(f"{mode}: autotuned params {plan.params()}, look-back {plan.lookback()}")
        plan.launch()
        torch.cuda.synchronize()
        plan.check()
    finally:
        plan.close()
    biggest = max(len(m["lat_idx"]) for m in meshes)
    scratch = sphint.Output(biggest)
    g = np.random.Generator(np.random.PCG64(33))
    picks = []
    for k, m in enumerate(meshes):
        nnz = len(m["lat_idx"])
        o = m["out"]
        ref = sphint.Output(nnz) if nnz != biggest else scratch
        sphint.arc_constlat(m["p1"], m["p2"], m["lat_z"], m["lat_offsets"], m["lat_idx"],
                            mode=mode, out=ref)
        torch.cuda.synchronize()
        t = ref.check()
        assert int(o.total.item()) == t, k
        assert torch.equal(o.count, ref.count) and torch.equal(o.flags, ref.flags), k
        for a, b in ((o.x, ref.x), (o.y, ref.y), (o.pair, ref.pair), (o.root, ref.root)):
            assert torch.equal(a[:t], b[:t]), k
        if mode == "eft" and nnz:
            picks += [(k, int(q)) for q in g.integers(0, nnz, 7)]
    note(f"{mode}: every mesh equals its single call")
    if mode != "eft":
        return
    # the per-pair schedule (every pair from its own endpoints) into a second set of outputs:
    # the autotuned launch and the single calls share arc records on dense lists
    scratch = None  # the single calls' outputs are freed before the second set is allocated
    second = [dict(m, out=sphint.Output(len(m["lat_idx"]))) for m in meshes]
    plan = sphint.BatchPlan(second, mode="eft")
    try:
        plan.set_share(False)
        plan.set_lookback(False)
        plan.set_params(3, 0)
        plan.launch()
        torch.cuda.synchronize()
        plan.check()
    finally:
        plan.close()
    for k, (m, s2) in enumerate(zip(meshes, second)):
        o, r = m["out"], s2["out"]
        t = int(o.total.item())
        assert int(r.total.item()) == t, k
        assert torch.equal(o.count, r.count) and torch.equal(o.flags, r.flags), k
        for a, b in ((o.x, r.x), (o.y, r.y), (o.pair, r.pair), (o.root, r.root)):
            assert torch.equal(a[:t], b[:t]), k
    del second
    note("eft: every mesh equals the per-pair schedule")
    # sampled pairs against the oracle
    rows, hits = [], []
    for k, q in picks[:400]:
        m = meshes[k]
        qt = torch.tensor([q], dtype=torch.int64, device="cuda")
        arc = int(torch.searchsorted(m["lat_offsets"], qt, right=True).item()) - 1
        lat = int(m["lat_idx"][q].item())
        x1 = tuple(float(c[arc].item()) for c in m["p1"])
        x2 = tuple(float(c[arc].item()) for c in m["p2"])
        z0 = float(m["lat_z"][lat].item())
        o = m["out"]
        first = int(o.count[:q].sum().item())
        c = int(o.count[q].item())
        hits.append((c, int(o.flags[q].item()), o.x[first:first + c].cpu().numpy(),
                     o.y[first:first + c].cpu().numpy(), o.root[first:first + c].cpu().numpy()))
        rows.append((*x1, *x2, z0))
    soa = [np.array([r[i] for r in rows]) for i in range(7)]
    ex = OB.exact(*soa, workers=1)
    rep = OB.accux_points(*soa, ex.roots, workers=1)
    k = 0
    for i, (c, fl, xs, ys, rs) in enumerate(hits):
        assert c == ex.count[i] and (fl & 31) == ex.flags[i], i
        assert tuple(int(r) for r in rs) == ex.roots[i], i
        for j in range(c):
            assert (xs[j], ys[j]) == rep[i][j], (i, j)
            e = max(abs(Decimal(float(xs[j])) - ex.hit_x[k]),
                    abs(Decimal(float(ys[j])) - ex.hit_y[k])) / Decimal(U)
            assert e <= 4, (i, j, float(e))
            k += 1
    note(f"{len(hits)} sampled pairs match the oracle")
