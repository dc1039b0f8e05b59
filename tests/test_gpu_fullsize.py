"""GPU parity at full size, in the launch configuration bench.py times.

The 1e7-pair ill-conditioned workload (dense) and the ne = 1024 cubed sphere x 1800
latitudes (CSR, 6.0e6 candidate pairs) run exactly as the benchmark runs them (one
sphint_arc_constlat call on the default stream).  Then:

* properties that hold at any size: the hit total is the sum of the counts, hits are in
  pair order, every pair index appears `count` times, roots are labels 0/1 and differ
  within a pair, EXISTS is set wherever a pair has hits;
* every pair of both modes equals the host build of the kernel arithmetic (the same
  headers compiled for the CPU, run on all host threads) bit for bit: counts, flags, and
  the compacted hits (pair, root, x, y) in order;
* the exact oracle on 10^6 stratified pairs of the 1e7 workload (a third per part): EFT
  counts, roots and flags exactly equal, every EFT point within 4 * 2^-53 of the exact
  one (>= 3 * 10^5 points per part);
* a smaller stratified sample of pairs is recomputed by the binary64 replicas one by one:
  EFT points bit-identical to the binary64 AccuX replica; naive everything bit-identical
  to the binary64 Eq. (2.2) replica;
* log2 histograms of the point errors (err / 2^-53) of both modes on the 10^6 sample, per
  part, are printed (naive mismatches in count are reported, not required to vanish).
"""

import ctypes
import math
import os
import sys
import threading
from decimal import Decimal

import numpy as np
import pytest

from oracle import batch as OB
from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
FLAG_MASK = 31
WORKERS = max(1, min(os.cpu_count() or 1, 16))
HOSTCHECK = os.environ.get("SPHINT_HOSTCHECK_LIB") or os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2510_09892_amd",
    "libsphint_hostcheck.so")


def note(msg):
    print(f"[gpu-full] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


@pytest.fixture(scope="module")
def ill(torch_cuda):
    note("generating 1e7 ill-conditioned pairs")
    P = inputs.ill_conditioned(10_000_000, seed_tag=1)
    dev = [torch_cuda.from_numpy(a).cuda() for a in P.soa()]
    return P, dev


@pytest.fixture(scope="module")
def cubed(torch_cuda):
    note("generating the ne=1024 cubed sphere x 1800 latitudes")
    m = inputs.cubed_sphere(1024)
    t = torch_cuda
    dev = dict(p=[t.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()],
               lat_z=t.from_numpy(m.lat_z).cuda(), off=t.from_numpy(m.lat_offsets).cuda(),
               idx=t.from_numpy(m.lat_idx).cuda())
    return m, dev


def fetch(torch, out):
    torch.cuda.synchronize()
    t = out.check()
    return dict(total=t, count=out.count.cpu().numpy(), flags=out.flags.cpu().numpy(),
                x=out.x[:t].cpu().numpy(), y=out.y[:t].cpu().numpy(),
                pair=out.pair[:t].cpu().numpy(), root=out.root[:t].cpu().numpy())


def host_eval(mode, soa, threads=WORKERS):
    """The host build of the kernel arithmetic on every pair, on `threads` host threads
    (ctypes releases the GIL): per-pair count, flags, roots and both points."""
    lib = ctypes.CDLL(HOSTCHECK)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_eval.argtypes = [ctypes.c_int, ctypes.c_int64] + [dp] * 7 + [ip] * 4 + [dp] * 4
    soa = [np.ascontiguousarray(a, dtype=np.float64) for a in soa]
    n = len(soa[0])
    ints = [np.zeros(n, np.int32) for _ in range(4)]
    dbl = [np.zeros(n, np.float64) for _ in range(4)]
    bounds = np.linspace(0, n, threads + 1).astype(np.int64)

    def work(lo, hi):
        ptr = lambda a: a[lo:hi].ctypes.data_as(dp if a.dtype == np.float64 else ip)  # noqa: E731
        lib.sphint_hostcheck_eval(mode, int(hi - lo), *[ptr(a) for a in soa],
                                  *[ptr(a) for a in ints], *[ptr(a) for a in dbl])
    ts = [threading.Thread(target=work, args=(bounds[k], bounds[k + 1])) for k in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    count, flags, r0, r1 = ints
    px0, py0, px1, py1 = dbl
    return dict(count=count, flags=flags, r0=r0, r1=r1, px0=px0, py0=py0, px1=px1, py1=py1)


def compact(h):
    """Per-pair host results in the library's output order: pair index, then along-arc."""
    c = h["count"].astype(np.int64)
    pair = np.repeat(np.arange(len(c), dtype=np.int64), c)
    start = np.concatenate([[0], np.cumsum(c)])[:-1]
    second = np.zeros(len(pair), bool)
    two = np.flatnonzero(c == 2)
    second[start[two] + 1] = True
    pick = lambda a, b: np.where(second, b[pair], a[pair])  # noqa: E731
    return dict(total=int(c.sum()), pair=pair, root=pick(h["r0"], h["r1"]).astype(np.uint8),
                x=pick(h["px0"], h["px1"]), y=pick(h["py0"], h["py1"]))


def check_equals_host(r, soa, mode):
    h = host_eval(1 if mode == "eft" else 0, soa)
    np.testing.assert_array_equal(r["count"], h["count"].astype(np.uint8))
    np.testing.assert_array_equal(r["flags"], h["flags"].astype(np.uint8))
    e = compact(h)
    assert r["total"] == e["total"]
    for k in ("pair", "root", "x", "y"):
        np.testing.assert_array_equal(r[k], e[k], err_msg=k)


def exact_errors_u(x, y, hit_x, hit_y):
    """Max-norm distance (in units of 2^-53) of binary64 points from 100-digit exact ones:
    each exact coordinate is split into a binary64 head and tail; the GPU value minus the
    head is exact (they agree to a few ulps), so the error carries a relative rounding of
    2^-53 at most, far below the 4 * 2^-53 bar."""
    def split(vals):
        hi = np.array([float(v) for v in vals])
        lo = np.array([float(v - Decimal(float(h))) for v, h in zip(vals, hi)])
        return hi, lo
    hx, lx = split(hit_x)
    hy, ly = split(hit_y)
    ex = np.abs((np.asarray(x) - hx) - lx)
    ey = np.abs((np.asarray(y) - hy) - ly)
    return np.maximum(ex, ey) / U


def run_dense(torch, dev, mode):
    from paper_2510_09892_amd import sphint
    out = sphint.Output(len(dev[6]))
    sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode=mode, out=out)
    return fetch(torch, out)


def run_csr(torch, dev, mode):
    from paper_2510_09892_amd import sphint
    p = dev["p"]
    out = sphint.Output(len(dev["idx"]))
    sphint.arc_constlat(tuple(p[:3]), tuple(p[3:]), dev["lat_z"], dev["off"], dev["idx"],
                        mode=mode, out=out)
    return fetch(torch, out)


def check_properties(r, n):
    c = r["count"].astype(np.int64)
    assert r["total"] == int(c.sum())
    assert np.all(np.diff(r["pair"]) >= 0)
    assert np.array_equal(np.bincount(r["pair"], minlength=n), c)
    assert np.all(r["root"] <= 1)
    start = np.concatenate([[0], np.cumsum(c)])[:-1]
    two = np.flatnonzero(c == 2)
    assert np.all(r["root"][start[two]] != r["root"][start[two] + 1])
    assert np.all(r["flags"][c > 0] & 1)
    return start


def err_u(x, y, px, py):
    return float(max(abs(Decimal(float(x)) - px), abs(Decimal(float(y)) - py)) / Decimal(U))


def check_sample_eft(r, start, soa, idx):
    sub = [a[idx] for a in soa]
    ex = OB.exact(*sub, workers=1)
    np.testing.assert_array_equal(r["count"][idx], ex.count)
    np.testing.assert_array_equal(r["flags"][idx] & FLAG_MASK, ex.flags)
    rep = OB.accux_points(*sub, ex.roots, workers=1)
    k = 0
    errs = []
    for j, i in enumerate(idx):
        s = start[i]
        for h, root in enumerate(ex.roots[j]):
            assert r["pair"][s + h] == i and r["root"][s + h] == root
            x, y = r["x"][s + h], r["y"][s + h]
            assert (x, y) == rep[j][h], (i, h)
            e = err_u(x, y, ex.hit_x[k], ex.hit_y[k])
            assert e <= 4.0, (i, h, e)
            errs.append(e)
            k += 1
    return ex, errs


def check_sample_naive(r, start, soa, idx):
    sub = [a[idx] for a in soa]
    nv = OB.naive_fp64(*sub, workers=1)
    np.testing.assert_array_equal(r["count"][idx], nv.count)
    np.testing.assert_array_equal(r["flags"][idx], nv.flags)
    k = 0
    for j, i in enumerate(idx):
        s = start[i]
        for h in range(int(nv.count[j])):
            assert r["root"][s + h] == nv.hit_root[k]
            assert r["x"][s + h] == nv.hit_x[k] and r["y"][s + h] == nv.hit_y[k]
            k += 1


def log2_hist(errs):
    h = {}
    for e in np.asarray(errs, dtype=np.float64).tolist():
        b = "0" if e == 0 else f"2^{math.ceil(math.log2(e))}"
        h[b] = h.get(b, 0) + 1
    return dict(sorted(h.items(), key=lambda kv: (kv[0] != "0", len(kv[0]), kv[0])))


@pytest.fixture(scope="module")
def ill_runs(torch_cuda, ill):
    P, dev = ill
    n = len(P)
    runs = {}
    for mode in ("eft", "naive"):
        note(f"{mode} launch at 1e7")
        r = run_dense(torch_cuda, dev, mode)
        r["start"] = check_properties(r, n)
        runs[mode] = r
    return runs


def test_ill1e7_every_pair_equals_host_build(ill, ill_runs):
    P, _ = ill
    for mode in ("eft", "naive"):
        note(f"host build ({WORKERS} threads) on all 1e7 pairs, {mode}")
        check_equals_host(ill_runs[mode], P.soa(), mode)


def test_ill1e7_oracle_million_and_error_histograms(ill, ill_runs):
    P, _ = ill
    soa = P.soa()
    re, rn = ill_runs["eft"], ill_runs["naive"]
    se, sn = re["start"], rn["start"]
    idx = inputs.stratified_sample(P, 333_334, seed=5)
    note(f"exact oracle on {len(idx)} stratified pairs ({WORKERS} workers)")
    sub = [a[idx] for a in soa]
    ex = OB.exact(*sub, workers=WORKERS)
    np.testing.assert_array_equal(re["count"][idx], ex.count)
    np.testing.assert_array_equal(re["flags"][idx] & FLAG_MASK, ex.flags)
    # the sampled pairs' hits, in the oracle's order, from the GPU output
    cnt = ex.count.astype(np.int64)
    rows = np.repeat(np.arange(len(idx)), cnt)
    h = np.arange(len(rows)) - np.repeat(np.concatenate([[0], np.cumsum(cnt)])[:-1], cnt)
    pos = se[idx][rows] + h
    assert np.array_equal(re["pair"][pos], idx[rows])
    assert np.array_equal(re["root"][pos], np.array(ex.hit_root, np.uint8))
    err = exact_errors_u(re["x"][pos], re["y"][pos], ex.hit_x, ex.hit_y)
    part = P.part[idx][rows]
    names = {0: "short arcs", 1: "near-tangent", 2: "near-pole"}
    for k in (0, 1, 2):
        note(f"part {names[k]}: {int((part == k).sum())} EFT points, max {err[part == k].max():.3g} u")
        assert (part == k).sum() >= 300_000
    assert err.max() <= 4.0, err.max()
    # naive: the same pairs; root/count mismatches are reported, errors where roots agree
    ncnt = rn["count"][idx].astype(np.int64)
    nroots_ok = np.zeros(len(idx), bool)
    for j in range(len(idx)):
        i = idx[j]
        nroots_ok[j] = (ncnt[j] == cnt[j] and
                        tuple(rn["root"][sn[i]:sn[i] + ncnt[j]]) == tuple(ex.roots[j]))
    ok_rows = nroots_ok[rows]
    npos = sn[idx][rows[ok_rows]] + h[ok_rows]
    hx = [v for v, o in zip(ex.hit_x, ok_rows) if o]
    hy = [v for v, o in zip(ex.hit_y, ok_rows) if o]
    nerr = exact_errors_u(rn["x"][npos], rn["y"][npos], hx, hy)
    npart = part[ok_rows]
    ppart = P.part[idx]
    for k in (0, 1, 2):
        note(f"part {names[k]}: naive hit/root mismatches {int((~nroots_ok[ppart == k]).sum())} "
             f"of {int((ppart == k).sum())} pairs")
        note(f"  eft   max {err[part == k].max():.3g} u  histogram {log2_hist(err[part == k])}")
        e = nerr[npart == k]
        note(f"  naive max {e.max() if len(e) else 0:.3g} u  histogram {log2_hist(e)}")


def test_ill1e7_sample_equals_binary64_replicas(ill, ill_runs):
    P, _ = ill
    soa = P.soa()
    idx = inputs.stratified_sample(P, 1500, seed=5)
    note(f"binary64 replicas on {len(idx)} sampled pairs")
    check_sample_eft(ill_runs["eft"], ill_runs["eft"]["start"], soa, idx)
    check_sample_naive(ill_runs["naive"], ill_runs["naive"]["start"], soa, idx)


def test_cubed1024_every_pair_and_sampled(torch_cuda, cubed):
    torch = torch_cuda
    m, dev = cubed
    assert m.nnz == len(m.lat_idx) and m.nnz > 5_000_000
    pairs = m.expand()
    soa = pairs.soa()
    g = np.random.Generator(np.random.PCG64(6))
    idx = np.sort(g.choice(m.nnz, 3000, replace=False))
    for mode in ("eft", "naive"):
        note(f"cubed sphere {mode} launch, nnz {m.nnz}")
        r = run_csr(torch, dev, mode)
        start = check_properties(r, m.nnz)
        note(f"host build ({WORKERS} threads) on all {m.nnz} pairs ({mode})")
        check_equals_host(r, soa, mode)
        note(f"oracle on {len(idx)} sampled pairs ({mode})")
        if mode == "eft":
            check_sample_eft(r, start, soa, idx)
        else:
            check_sample_naive(r, start, soa, idx)
