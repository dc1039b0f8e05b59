"""GPU: the batched persistent launch (sphint_batch_*) over many uneven meshes.

* One graph-replayed launch over all meshes gives, for every mesh, the bytes of a
  per-mesh sphint_arc_constlat call (counts, flags, hits), in both modes.
* Every tile/schedule parameter choice the autotuner may pick (pairs per lane, workgroups
  per CU, scanner or decoupled look-back, and for EFT arc records shared by a tile's rows)
  gives the same bytes, also on meshes with exact ties, degenerate and non-finite arcs,
  out-of-range latitude indices and mostly empty candidate lists.
* Graph replays, with eager work and synchronisations between them, all give the same
  bytes; the autotuner's cache file is written and read back.
* One small mesh against the oracle.
* Meshes without flags arrays: every schedule gives the per-mesh counts and hits.
* The one-shot batched launch (sphint_batch_run, no plan) over 1, 7 and 16 meshes (CSR
  with an empty mesh among them, and dense), reusing one workspace on one stream: every
  mesh equals its single call, in both modes.
"""

import os
import sys

import numpy as np
import pytest

from oracle import batch as OB
from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

FLAG_MASK = 31


def note(msg):
    print(f"[gpu-batch] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def make_meshes(n=7, seed_tag=40):
    g = inputs.rng(seed_tag)
    out = []
    for k in range(n):
        arcs = int(np.exp(g.uniform(np.log(200), np.log(60_000))))
        lats = int(g.integers(10, 900))
        out.append(inputs.random_mesh(inputs.rng(seed_tag, k + 1), arcs, lats))
    return out


def to_dev(torch, m):
    from paper_2510_09892_amd import sphint
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()]
    return dict(p1=tuple(d[:3]), p2=tuple(d[3:]), lat_z=torch.from_numpy(m.lat_z).cuda(),
                lat_offsets=torch.from_numpy(m.lat_offsets).cuda(),
                lat_idx=torch.from_numpy(m.lat_idx).cuda(), out=sphint.Output(m.nnz))


def read(out):
    t = int(out.total.item())
    return dict(total=t, count=out.count.cpu().numpy().copy(), flags=out.flags.cpu().numpy().copy(),
                x=out.x[:t].cpu().numpy().copy(), y=out.y[:t].cpu().numpy().copy(),
                pair=out.pair[:t].cpu().numpy().copy(), root=out.root[:t].cpu().numpy().copy())


def same(a, b):
    return a["total"] == b["total"] and all(
        np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8))
        for k in ("count", "flags", "x", "y", "pair", "root"))


def per_mesh(torch, devs, mode):
    from paper_2510_09892_amd import sphint
    res = []
    for d in devs:
        o = sphint.Output(d["out"].nnz)
        sphint.arc_constlat(d["p1"], d["p2"], d["lat_z"], d["lat_offsets"], d["lat_idx"],
                            mode=mode, out=o)
        torch.cuda.synchronize()
        o.check()
        res.append(read(o))
    return res


def scrub(torch, devs):
    for d in devs:
        o = d["out"]
        for t in (o.x, o.y):
            t.fill_(float("nan"))
        o.pair.fill_(-1)
        o.root.fill_(255)
        o.count.fill_(255)
        o.flags.fill_(255)
        o.total.fill_(-1)
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["eft", "naive"])
def test_batch_equals_per_mesh(torch_cuda, mode, tmp_path):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    meshes = make_meshes()
    note(f"{mode}: {len(meshes)} meshes, nnz {[m.nnz for m in meshes]}")
    devs = [to_dev(torch, m) for m in meshes]
    ref = per_mesh(torch, devs, mode)
    plan = sphint.BatchPlan(devs, mode=mode)
    try:
        for lb in (False, True):
            plan.set_lookback(lb)
            assert plan.lookback() == lb
            for ppt in (1, 2, 3, 4):
                for wg in (0, 1, 2):
                    note(f"{mode}: params ppt={ppt} wg_per_cu={wg} lookback={lb}")
                    plan.set_params(ppt, wg)
                    scrub(torch, devs)
                    plan.launch()
                    torch.cuda.synchronize()
                    plan.check()
                    for d, r in zip(devs, ref):
                        assert same(read(d["out"]), r), (ppt, wg, lb)
        cache = os.path.join(str(tmp_path), "tune.txt")
        note(f"{mode}: autotune")
        plan.autotune(cache)
        chosen = plan.params(), plan.lookback(), plan.share()
        assert chosen[0][0] in (1, 2, 3, 4) and chosen[0][1] >= 0
        assert mode == "eft" or not chosen[2]
        note(f"{mode}: autotuner chose {chosen}")
        assert os.path.exists(cache) and open(cache).read().strip()
        plan.set_params(1, 1)
        plan.set_lookback(not chosen[1])
        if mode == "eft":
            plan.set_share(not chosen[2])
        plan.autotune(cache)  # read back from the cache
        assert (plan.params(), plan.lookback(), plan.share()) == chosen
        for rep in range(4):  # graph replays with eager work in between
            note(f"{mode}: replay {rep}")
            scrub(torch, devs)
            eager = torch.arange(1000, device="cuda", dtype=torch.float64).sum()
            plan.launch()
            torch.cuda.synchronize()
            assert float(eager.item()) == 499500.0
            plan.check()
            for d, r in zip(devs, ref):
                assert same(read(d["out"]), r), rep
    finally:
        plan.close()


def test_batch_small_mesh_against_oracle(torch_cuda):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    meshes = [inputs.random_mesh(inputs.rng(41, k), 400 + 300 * k, 60 + 40 * k) for k in range(3)]
    devs = [to_dev(torch, m) for m in meshes]
    plan = sphint.BatchPlan(devs, mode="eft")
    try:
        plan.launch()
        torch.cuda.synchronize()
        plan.check()
        for m, d in zip(meshes, devs):
            r = read(d["out"])
            ex = OB.exact(*m.expand().soa(), workers=1)
            np.testing.assert_array_equal(r["count"], ex.count)
            np.testing.assert_array_equal(r["flags"] & FLAG_MASK, ex.flags)
            np.testing.assert_array_equal(r["pair"], np.array(ex.hit_pair, dtype=np.int64))
    finally:
        plan.close()


def test_batch_dense_meshes(torch_cuda):
    """Dense (1:1) meshes in one plan equal per-mesh dense calls."""
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    sets = [inputs.ill_conditioned(n, seed_tag=42 + k) for k, n in enumerate((700, 20_000, 5_001))]
    devs = []
    for P in sets:
        d = [torch.from_numpy(a).cuda() for a in P.soa()]
        devs.append(dict(p1=tuple(d[:3]), p2=tuple(d[3:6]), lat_z=d[6], out=sphint.Output(len(P))))
    ref = []
    for d in devs:
        o = sphint.Output(d["out"].nnz)
        sphint.arc_constlat(d["p1"], d["p2"], d["lat_z"], mode="eft", out=o)
        torch.cuda.synchronize()
        o.check()
        ref.append(read(o))
    plan = sphint.BatchPlan(devs, mode="eft")
    try:
        for ppt in (1, 3, 4):
            note(f"dense batch ppt={ppt}")
            plan.set_params(ppt, 0)
            scrub(torch, devs)
            plan.launch()
            torch.cuda.synchronize()
            plan.check()
            for d, r in zip(devs, ref):
                assert same(read(d["out"]), r), ppt
    finally:
        plan.close()


@pytest.mark.parametrize("mode", ["eft", "naive"])
def test_batch_run_equals_single_calls(torch_cuda, mode):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    csr = make_meshes(16, seed_tag=47)
    empty = inputs.random_mesh(inputs.rng(47, 99), 50, 3)
    empty.lat_offsets[:] = 0
    empty.lat_idx = empty.lat_idx[:0]
    csr[5] = empty
    dense = [inputs.ill_conditioned(n, seed_tag=48 + k) for k, n in enumerate((1, 640, 5_000, 70_001))]
    ref = {}
    for k, m in enumerate(csr):
        d = to_dev(torch, m)
        sphint.arc_constlat(d["p1"], d["p2"], d["lat_z"], d["lat_offsets"], d["lat_idx"],
                            mode=mode, out=d["out"])
        torch.cuda.synchronize()
        d["out"].check()
        ref[("csr", k)] = read(d["out"])
    for k, P in enumerate(dense):
        t = [torch.from_numpy(a).cuda() for a in P.soa()]
        out = sphint.Output(len(P))
        sphint.arc_constlat(tuple(t[:3]), tuple(t[3:6]), t[6], mode=mode, out=out)
        torch.cuda.synchronize()
        out.check()
        ref[("dense", k)] = read(out)
    ws = torch.empty(sphint.batch_run_workspace_size(16, sum(m.nnz for m in csr)),
                     dtype=torch.uint8, device="cuda")
    for sel in ([3], list(range(7)), list(range(16))):
        devs = [to_dev(torch, csr[k]) for k in sel]
        note(f"batch_run {mode}: {len(sel)} CSR meshes, {sum(csr[k].nnz for k in sel)} pairs")
        sphint.batch_run(devs, mode=mode, workspace=ws)
        torch.cuda.synchronize()
        assert sphint.load().sphint_check(ws.data_ptr(), 0, 0) == sphint.OK
        for k, d in zip(sel, devs):
            got = read(d["out"])
            for key, v in ref[("csr", k)].items():
                assert np.array_equal(np.asarray(got[key]), np.asarray(v)), (k, key)
    devs = []
    for P in dense:
        t = [torch.from_numpy(a).cuda() for a in P.soa()]
        devs.append(dict(p1=tuple(t[:3]), p2=tuple(t[3:6]), lat_z=t[6], out=sphint.Output(len(P))))
    note(f"batch_run {mode}: {len(dense)} dense meshes")
    sphint.batch_run(devs, mode=mode, workspace=ws)
    torch.cuda.synchronize()
    for k, d in enumerate(devs):
        got = read(d["out"])
        for key, v in ref[("dense", k)].items():
            assert np.array_equal(np.asarray(got[key]), np.asarray(v)), (k, key)


class _Mesh:
    """A CSR mesh from explicit arrays (the shape inputs.CsrMesh has)."""

    def __init__(self, ends, lat_z, off, idx):
        self.ends = [np.ascontiguousarray(a, dtype=np.float64) for a in ends]
        self.lat_z = np.ascontiguousarray(lat_z, dtype=np.float64)
        self.lat_offsets = np.ascontiguousarray(off, dtype=np.int64)
        self.lat_idx = np.ascontiguousarray(idx, dtype=np.int32)
        self.nnz = int(self.lat_offsets[-1])

    def soa(self):
        return self.ends


def shared_arc_meshes():
    """Meshes for the shared-arc schedules: uneven random meshes; one with many candidates
    per arc (windows reused over many rows); one with most arcs without candidates (rows
    spanning more than 64 arc ids: every lane computes its own arc); integer arcs with
    latitudes at exact ties (open slope filters, the exact fallback); degenerate and
    non-finite arcs with out-of-range latitude indices."""
    import itertools
    import math
    import test_hostcheck_shared as TS
    meshes = make_meshes(5, seed_tag=44)
    meshes.append(inputs.random_mesh(inputs.rng(44, 50), 30_000, 3000))
    meshes.append(inputs.random_mesh(inputs.rng(44, 51), 40_000, 12, d_hi=0.01))
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0), repeat=3) if any(v)]
    zs = []
    for z in (-1.0, -0.5, 0.0, 0.375, 1.0, 0.7071067811865476, 0.5773502691896258):
        zs += [z, math.nextafter(z, 2.0), math.nextafter(z, -2.0)]
    arcs = [(*a, *b) for a in verts for b in verts]
    meshes.append(_Mesh(*TS._csr(arcs, [zs] * len(arcs))))
    m = inputs.random_mesh(inputs.rng(44, 52), 3000, 200)
    x1 = m.soa()[0].copy()
    x1[::97] = np.inf
    ends = [x1] + list(m.soa()[1:])
    ends[3] = ends[3].copy()
    ends[3][5::89] = ends[0][5::89]       # some arcs with equal endpoints (degenerate)
    ends[4] = ends[4].copy()
    ends[4][5::89] = ends[1][5::89]
    ends[5] = ends[5].copy()
    ends[5][5::89] = ends[2][5::89]
    idx = m.lat_idx.copy()
    idx[::11] = 10_000                    # out of range: NONFINITE, never an out-of-bounds read
    meshes.append(_Mesh(ends, m.lat_z, m.lat_offsets, idx))
    return meshes


@pytest.mark.parametrize("mode", ["eft", "naive"])
def test_batch_without_flags_arrays(torch_cuda, mode):
    """Meshes without flags arrays (their flags go to the count bytes first, then the
    counts): every schedule gives the per-mesh calls' counts and hits."""
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    meshes = make_meshes(4, seed_tag=47)
    devs = [to_dev(torch, m) for m in meshes]
    ref = per_mesh(torch, devs, mode)
    for d in devs:
        d["out"] = sphint.Output(d["out"].nnz, flags=False)
    plan = sphint.BatchPlan(devs, mode=mode)
    shares = (False, True) if mode == "eft" else (False,)
    try:
        for share in shares:
            if mode == "eft":
                plan.set_share(share)
            for lb in (False, True):
                plan.set_lookback(lb)
                for ppt in ((1, 2, 3, 4, 5) if share else (1, 2, 3, 4)):
                    note(f"{mode} without flags: ppt={ppt} lookback={lb} share={share}")
                    plan.set_params(ppt, 0)
                    for d in devs:
                        d["out"].count.fill_(255)
                        d["out"].total.fill_(-1)
                    plan.launch()
                    torch.cuda.synchronize()
                    plan.check()
                    for d, r in zip(devs, ref):
                        o = d["out"]
                        t = int(o.total.item())
                        assert t == r["total"], (ppt, lb, share)
                        assert np.array_equal(o.count.cpu().numpy(), r["count"])
                        for key, a in (("x", o.x), ("y", o.y), ("pair", o.pair), ("root", o.root)):
                            assert np.array_equal(a[:t].cpu().numpy().view(np.uint8),
                                                  r[key].view(np.uint8)), (key, ppt, lb, share)
    finally:
        plan.close()


def test_batch_shared_arcs_equal_per_mesh(torch_cuda):
    """EFT plans over CSR lists with arc records shared by a tile's rows: every schedule
    (pairs per lane x scanner or look-back x workgroups per CU), and every single call, gives
    for every mesh the bytes of the per-pair schedule; naive and dense plans refuse the
    option."""
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    meshes = shared_arc_meshes()
    note(f"shared arcs: {len(meshes)} meshes, nnz {[m.nnz for m in meshes]}")
    devs = [to_dev(torch, m) for m in meshes]
    plan = sphint.BatchPlan(devs, mode="eft")
    try:
        assert not plan.share()
        # the reference: every pair evaluated from its own endpoints (per-pair schedule)
        plan.set_params(3, 0)
        scrub(torch, devs)
        plan.launch()
        torch.cuda.synchronize()
        plan.check()
        ref = [read(d["out"]) for d in devs]
        assert any(np.any(r["flags"] & 32) for r in ref)  # the exact fallback occurs
        # single calls (which share arc records on meshes with >= 2.5 candidates per arc)
        for k, (r, s) in enumerate(zip(ref, per_mesh(torch, devs, "eft"))):
            assert same(s, r), k
        plan.set_share(True)
        assert plan.share()
        for lb in (False, True):
            plan.set_lookback(lb)
            for ppt in (1, 2, 3, 4, 5):
                for wg in (0, 1):
                    note(f"shared arcs: ppt={ppt} wg_per_cu={wg} lookback={lb}")
                    plan.set_params(ppt, wg)
                    scrub(torch, devs)
                    plan.launch()
                    torch.cuda.synchronize()
                    plan.check()
                    for k, (d, r) in enumerate(zip(devs, ref)):
                        assert same(read(d["out"]), r), (k, ppt, wg, lb)
        for rep in range(3):  # graph replays
            note(f"shared arcs: replay {rep}")
            scrub(torch, devs)
            plan.launch()
            torch.cuda.synchronize()
            plan.check()
            for k, (d, r) in enumerate(zip(devs, ref)):
                assert same(read(d["out"]), r), (k, rep)
        with pytest.raises(sphint.SphintError):
            plan.set_share(False)  # five pairs per lane exist with shared records only
        plan.set_params(4, 0)
        plan.set_share(False)
        with pytest.raises(sphint.SphintError):
            plan.set_params(5, 0)
    finally:
        plan.close()
    naive = sphint.BatchPlan(devs[:2], mode="naive")
    try:
        with pytest.raises(sphint.SphintError):
            naive.set_share(True)
    finally:
        naive.close()


def test_batch_run_shared_arcs_equal_per_pair(torch_cuda):
    """The one-shot batched launch over dense candidate lists (>= 2.5 candidates per arc in
    all: arc records shared, EFT) equals the per-pair schedule of a plan, bit for bit, on
    random meshes and the exact-tie mesh."""
    import itertools
    import math
    import test_hostcheck_shared as TS
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    meshes = [inputs.random_mesh(inputs.rng(49, k), 2000 + 700 * k, 2500) for k in range(4)]
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0), repeat=3) if any(v)]
    zs = []
    for z in (-1.0, -0.5, 0.0, 0.375, 1.0, 0.7071067811865476):
        zs += [z, math.nextafter(z, 2.0), math.nextafter(z, -2.0)]
    meshes.append(_Mesh(*TS._csr([(*a, *b) for a in verts for b in verts],
                                 [zs] * (len(verts) ** 2))))
    assert 2 * sum(m.nnz for m in meshes) >= 5 * sum(len(m.lat_offsets) - 1 for m in meshes)
    devs = [to_dev(torch, m) for m in meshes]
    plan = sphint.BatchPlan(devs, mode="eft")
    try:
        plan.set_params(3, 0)  # per-pair schedule (sharing off by default)
        plan.launch()
        torch.cuda.synchronize()
        plan.check()
        ref = [read(d["out"]) for d in devs]
    finally:
        plan.close()
    assert any(np.any(r["flags"] & 32) for r in ref)
    ws = torch.empty(sphint.batch_run_workspace_size(len(devs), sum(m.nnz for m in meshes)),
                     dtype=torch.uint8, device="cuda")
    for rep in range(2):
        note(f"batch_run shared arcs, {len(devs)} meshes, round {rep}")
        scrub(torch, devs)
        sphint.batch_run(devs, mode="eft", workspace=ws)
        torch.cuda.synchronize()
        assert sphint.load().sphint_check(ws.data_ptr(), 0, 0) == sphint.OK
        for k, (d, r) in enumerate(zip(devs, ref)):
            assert same(read(d["out"]), r), (k, rep)
