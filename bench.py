#!/usr/bin/env python3
"""Throughput of arc x constant-latitude intersections on one MI355X.

A step is one sphint_arc_constlat call over the whole workload (every pair evaluated,
counts/flags written, hits compacted), inputs already resident in HBM.  Default workload:
10^7 ill-conditioned arcs in three equal parts (1e-10..1e-6 rad arcs; latitudes within
1e-12 of an arc's apex or nadir; arcs within 1e-6 rad of a pole), one latitude per arc.
The EFT step is the headline; the naive binary64 step runs on the same inputs beside it.

Prints one JSON line.  Extra lines go to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))

METRIC = "arc-latitude intersections/s (EFT vs naive FP64, ≤4·2^-53 err); p99 latency"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
ALU_PEAK = 256 * 64 * 2.4e9  # binary64 lane operations/s: 256 CUs x 64 lanes x 2.4 GHz
BYTES_PER_PAIR = 7 * 8 + 2   # x1, y1, z1, x2, y2, z2, z0 read; count + flags written
BYTES_PER_HIT = 8 + 8 + 8 + 1  # x, y, pair, root
# Algorithmic binary64 operations (add, sub, mul, FMA, and each sqrt or division, count 1),
# counted on the operations the method defines (EFT: Alg. 8 with the normal renormalised,
# plus the first stage of each exact-decision filter; naive: Eq. 2.2 and its predicates).
EFT_OPS_PER_ARC = 146            # normal, norms, F pairs, filter inputs (z0-free)
EFT_OPS_PER_PAIR = EFT_OPS_PER_ARC + 79  # per arc part + per pair
EFT_OPS_PER_HITPAIR = 16         # AccSqrt and the root-independent z0 products
EFT_OPS_PER_HIT = 100            # two six-term CompDots and two divisions per root
NAIVE_OPS_PER_PAIR = 25
NAIVE_OPS_PER_HITPAIR = 15       # sqrt, six products, both roots' sums and divisions


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest():
    """sha256 over the kernel sources, the public header and the build flags."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_09892_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)
                   if f.endswith((".hip", ".hpp")))
    files += [os.path.join(ROOT, "include", "sphint.h"),
              os.path.join(ROOT, "paper_2510_09892_amd", "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel_tag, digest):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
    this kernel, or None when the summary is absent or was taken from other sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    got = dict(re.findall(r"^- (\w+): `([^`]+)`", txt, re.M))
    if got.get("source_sha256") != digest:
        return None
    try:
        return {"fetch_bytes": float(got["fetch_bytes_per_launch"]),
                "write_bytes": float(got["write_bytes_per_launch"]),
                "bytes": float(got["fetch_bytes_per_launch"]) + float(got["write_bytes_per_launch"]),
                "source": os.path.relpath(path, ROOT)}
    except (KeyError, ValueError):
        return None


def measured_valu(kernel_tag, digest):
    """VALU instructions per 64-pair wavefront row from the committed rocprofv3 SQ counter
    summary of this kernel, or None when absent or taken from other sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_sq.md")
    if not os.path.exists(path):
        return None
    got = dict(re.findall(r"^- (\w+): `([^`]+)`", open(path).read(), re.M))
    if got.get("source_sha256") != digest:
        return None
    try:
        return {"valu_per_row": float(got["valu_insts_per_row"]),
                "fp64_per_row": float(got["fp64_insts_per_row"]),
                "source": os.path.relpath(path, ROOT)}
    except (KeyError, ValueError):
        return None


def settle(torch, call, out, mode, seconds):
    """Untimed calls of the mode for `seconds` of wall time, before the warm-up steps.  Under
    sustained binary64 load the GPU's clock settles over the first ~0.1 s: the first calls
    of a fresh process run up to ~20% slower than the steady state that the timed steps are
    meant to measure.  Returns the number of calls made."""
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            call(out, mode)
        torch.cuda.synchronize()
        n += 10
    return n


def run_mode(torch, sphint, call, nnz, mode, steps, warmup, settle_s=0.0):
    """Times `steps` calls of call(out, mode) (one sphint_arc_constlat each), after
    settle_s seconds of untimed calls and `warmup` untimed steps."""
    out = sphint.Output(nnz)
    settled = settle(torch, call, out, mode, settle_s) if settle_s > 0 else 0
    for _ in range(warmup):
        call(out, mode)
    total = out.check()
    timer = sphint.KernelTimer(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        timer.arm(k)
        call(out, mode)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timer.disarm()
    kms = timer.durations_ms()
    timer.close()
    total2 = out.check()
    assert total2 == total
    hitpairs = int((out.count > 0).sum().item())  # accounting only, after the timed region
    return dict(wall_s=t1 - t0, kernel_ms=kms, total=total, hitpairs=hitpairs, out=out,
                settle_calls=settled)


def csr_main_bytes(arcs_used, nnz, n_lat, hits):
    """Algorithmic bytes of one CSR main-kernel launch: the endpoints of every arc that has a
    candidate (48 B, read once; arcs without one need not be read), per pair its latitude
    index (4 B), its arc id (4 B, from the pair-to-arc table) and its count and flags (2 B),
    the latitude table, and 25 B per hit (x, y, pair, root)."""
    return 48 * arcs_used + 10 * nnz + 8 * n_lat + BYTES_PER_HIT * hits


def roofline(mode, r, pairs, bytes_launch, kernel, tag, shared_arcs=None):
    """Binding roof of the dominant kernel from its mean duration (HIP events).  With
    shared_arcs (the number of arcs with candidates, when arc records are shared) the EFT
    z0-free part counts once per arc instead of once per pair."""
    kms = statistics.mean(r["kernel_ms"])
    hits = r["total"]
    if mode == "eft":
        per_arc = EFT_OPS_PER_ARC * (pairs if shared_arcs is None else shared_arcs)
        ops_launch = (per_arc + (EFT_OPS_PER_PAIR - EFT_OPS_PER_ARC) * pairs
                      + EFT_OPS_PER_HITPAIR * r["hitpairs"] + EFT_OPS_PER_HIT * hits)
    else:
        ops_launch = NAIVE_OPS_PER_PAIR * pairs + NAIVE_OPS_PER_HITPAIR * r["hitpairs"]
    bw = bytes_launch / (kms * 1e-3)
    ops = ops_launch / (kms * 1e-3)
    hbm = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
           "frac": bw / HBM_PEAK}
    alu = {"bound": "alu", "achieved": ops / 1e12, "peak": ALU_PEAK / 1e12,
           "unit": "Tlane-op/s (binary64)", "frac": ops / ALU_PEAK}
    roof = dict(hbm if hbm["frac"] >= alu["frac"] else alu)
    other = alu if roof["bound"] == "hbm" else hbm
    tr = measured_traffic(tag, source_digest()) if tag else None
    roof["traffic"] = tr["bytes"] if tr else None
    if tr:
        roof["traffic_detail"] = tr
    va = measured_valu(tag, source_digest()) if tag else None
    if va:  # the measured issue roof: wavefront VALU instructions x 64 lanes per launch
        lane_instr = va["valu_per_row"] * 64 * (pairs / 64)
        rate = lane_instr / (kms * 1e-3)
        roof["valu_issue"] = {"achieved": rate / 1e12, "peak": ALU_PEAK / 1e12,
                              "unit": "Tlane-instr/s", "frac": rate / ALU_PEAK,
                              "valu_instr_per_pair": va["valu_per_row"],
                              "fp64_instr_per_pair": va["fp64_per_row"], "source": va["source"]}
    roof["kernel"] = kernel
    roof["kernel_ms"] = kms
    roof["kernel_ms_p10_p50_p90"] = pctl(r["kernel_ms"])
    roof["algorithmic_bytes"] = bytes_launch
    roof["algorithmic_ops"] = ops_launch
    roof["other_bound"] = {k: other[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    return roof


def copy_calibration(torch, nbytes):
    """A plain device copy of known size, for scaling the profiler's byte counters."""
    if not nbytes:
        return
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {nbytes} bytes x3")


def pctl(v):
    v = sorted(v)
    return [v[int(q * (len(v) - 1))] for q in (0.1, 0.5, 0.9)]


def latency_small(torch, sphint, inputs, reps=1000):
    """The 1e5-arc uniform workload (EFT): per-call latency, host enqueue to completion, and
    the throughput of back-to-back replays of the call captured in a hipGraph (a one-mesh
    batched plan)."""
    P = inputs.uniform_arcs(100_000, seed_tag=0)
    dev = [torch.from_numpy(a).cuda() for a in P.soa()]
    out = sphint.Output(len(P))
    lat = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for r in range(reps + 10):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if r >= 10:
            ev[r - 10][0].record()
        sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode="eft", out=out)
        if r >= 10:
            ev[r - 10][1].record()
        torch.cuda.synchronize()
        if r >= 10:
            lat.append((time.perf_counter() - t0) * 1e6)
    lat.sort()
    # device time of each call: HIP events on the call's stream around its launches
    dev_us = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
    plan = sphint.BatchPlan([dict(p1=tuple(dev[:3]), p2=tuple(dev[3:6]), lat_z=dev[6], out=out)],
                            mode="eft")
    for _ in range(10):
        plan.launch()
    torch.cuda.synchronize()
    n_rep = 200
    t0 = time.perf_counter()
    for _ in range(n_rep):
        plan.launch()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n_rep
    plan.check()
    plan.close()
    return dict(device_p50_us=dev_us[len(dev_us) // 2], device_p10_p90_us=[
                    dev_us[int(0.1 * (len(dev_us) - 1))], dev_us[int(0.9 * (len(dev_us) - 1))]],
                device_p99_us=dev_us[int(len(dev_us) * 0.99) - 1],
                p50_us=lat[len(lat) // 2], p99_us=lat[int(len(lat) * 0.99) - 1], calls=reps,
                graph_replay_us=dt * 1e6, graph_replay_pairs_per_s=len(P) / dt,
                note="device_*: HIP events around each call on its stream (init and main "
                     "launch); p50_us/p99_us: host enqueue to completion")


def serving(torch, args, log):
    """The serving loop on Poisson arrivals (both modes, same arrivals and payloads)."""
    from paper_2510_09892_amd import inputs, serve
    log(f"[bench] serving: building {args.serve_pool} request payloads")
    pool = serve.request_pool(args.serve_pool)
    arrivals, _ = inputs.request_stream(rate_hz=args.serve_rate, duration_s=args.serve_seconds,
                                        seed_tag=4)
    n = len(arrivals)
    out = {"workload": f"Poisson arrivals at {args.serve_rate:g}/s for {args.serve_seconds:g} s "
                       f"({n} requests); request k uses payload k mod {len(pool)} of a pool drawn "
                       "from log-uniform 1e3..1e6 arcs x log-uniform 1..1000 latitudes (CSR "
                       "candidates); 64 GiB device budget; continuous batching: up to 16 "
                       "requests per persistent launch, 2 launches in flight, 32 request slots",
           "pool_pairs_mean": sum(p.nnz for p in pool) / len(pool)}
    for mode in ("eft", "naive"):
        srv = serve.Server(mode=mode, budget_bytes=64 << 30, slots=32)
        srv.run(arrivals[:64] * 0.0, lambda i: pool[i % len(pool)])  # warm-up: arenas, code
        log(f"[bench] serving {mode}: {n} requests")
        rep = srv.run(arrivals, lambda i: pool[i % len(pool)])
        srv.close()
        log(f"[bench] serving {mode}: {rep['req_per_s']:.0f} req/s, p50 {rep['latency_ms']['p50']:.3f} ms, "
            f"p99 {rep['latency_ms']['p99']:.3f} ms, {rep['launches']} launches, "
            f"{rep['requests_per_launch_mean']:.2f} requests per launch")
        out[mode] = rep
    return out


def candidate_timing(torch, sphint, inputs, mesh, dp, lz, reps=10):
    """CSR candidate lists of the mesh built on the GPU (sphint_candidates_count + _fill,
    including the host read of nnz between them) against the host generator."""
    t0 = time.perf_counter()
    off_h, idx_h = inputs.candidates(mesh.p1, mesh.p2, mesh.lat_z)
    host_s = time.perf_counter() - t0
    for _ in range(2):
        sphint.candidates(tuple(dp[:3]), tuple(dp[3:]), lz, 1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        off, idx = sphint.candidates(tuple(dp[:3]), tuple(dp[3:]), lz, 1e-12)
    torch.cuda.synchronize()
    gpu_s = (time.perf_counter() - t0) / reps
    return {"gpu_ms": gpu_s * 1e3, "host_numpy_s": host_s, "arcs": len(mesh.p1),
            "candidates_gpu": int(len(idx)), "candidates_host": int(len(idx_h)),
            "arcs_per_s_gpu": len(mesh.p1) / gpu_s}


def cubed_subresult(torch, np, sphint, inputs, steps, warmup, settle_s=0.0):
    """The regridding-shaped workload (ne = 1024 cubed sphere x 1800 latitudes, CSR) in both
    modes: wall time per call, main-kernel time (HIP events) and its roofline."""
    log("[bench] cubed sphere ne=1024 x 1800 latitudes: generating")
    mesh = inputs.cubed_sphere(1024)
    n = mesh.nnz
    dp = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in mesh.soa()]
    lz, off, idx = (torch.from_numpy(a).cuda() for a in (mesh.lat_z, mesh.lat_offsets, mesh.lat_idx))

    def call(out, mode):
        sphint.arc_constlat(tuple(dp[:3]), tuple(dp[3:]), lz, off, idx, mode=mode, out=out)
    arcs_used = int(np.count_nonzero(np.diff(mesh.lat_offsets)))
    res = {"workload": "cubed sphere ne=1024: 12,582,912 unique great-circle edges x 1800 "
                       "latitude lines (-89.95 deg + 0.1 deg k), CSR candidates from z-range "
                       "overlap", "pairs": n, "arcs": mesh.n_arcs, "arcs_with_candidates": arcs_used}
    for mode in ("eft", "naive"):
        r = run_mode(torch, sphint, call, n, mode, steps, warmup, settle_s)
        byts = csr_main_bytes(arcs_used, n, len(mesh.lat_z), r["total"])
        shared = mode == "eft" and 2 * n >= 5 * mesh.n_arcs  # the rule sphint_arc_constlat applies
        kern = (f"sphint::k_intersect_w<{1 if mode == 'eft' else 0},{3 if mode == 'eft' else 4},"
                f"true,{'true' if shared else 'false'}>")
        roof = roofline(mode, r, n, byts, kern, f"k_intersect_w_{mode}_cubed1024")
        if roof.get("traffic"):
            roof["traffic_over_algorithmic"] = roof["traffic"] / byts
        res[mode] = {"value": n * steps / r["wall_s"], "ms_per_step": r["wall_s"] / steps * 1e3,
                     "kernel_ms": statistics.mean(r["kernel_ms"]), "hits": r["total"],
                     "roofline": roof}
        log(f"[bench] cubed {mode}: {res[mode]['ms_per_step']:.4f} ms per call, kernel "
            f"{res[mode]['kernel_ms']:.4f} ms, {roof['bound']} frac {roof['frac']:.3f}")
        del r["out"]
    res["eft_over_naive"] = res["eft"]["value"] / res["naive"]["value"]
    return res


def batch_measure(torch, sphint, devs, stats, modes, steps, warmup):
    """One autotuned persistent graph launch over all meshes against one sphint_arc_constlat
    call per mesh; `stats` per mesh: (arcs, arcs with candidates, pairs, latitudes)."""
    nnz = sum(st[2] for st in stats)
    res = {}
    for mode in modes:
        def per_mesh():
            for d in devs:
                sphint.arc_constlat(d["p1"], d["p2"], d["lat_z"], d["lat_offsets"], d["lat_idx"],
                                    mode=mode, out=d["out"])
        for _ in range(warmup):
            per_mesh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            per_mesh()
        torch.cuda.synchronize()
        t_per = (time.perf_counter() - t0) / steps
        plan = sphint.BatchPlan(devs, mode=mode)
        t1 = time.perf_counter()
        plan.autotune()
        t_tune = time.perf_counter() - t1
        for _ in range(warmup):
            plan.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.launch()
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / steps
        # device time of each graph launch (HIP events on the launch stream around it)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for e0, e1 in ev:
            e0.record()
            plan.launch()
            e1.record()
        torch.cuda.synchronize()
        dms = [e0.elapsed_time(e1) for e0, e1 in ev]
        plan.check()
        hits = sum(int(d["out"].total.item()) for d in devs)
        hitpairs = sum(int((d["out"].count > 0).sum().item()) for d in devs)
        # algorithmic bytes of one launch: the endpoints of arcs with candidates and the
        # offsets, per pair its latitude index and its count and flags, the latitude tables,
        # and the hits; the binding roof (HBM or binary64 ALU) of the whole graph launch,
        # whose batched kernel dominates it
        byts = sum(48 * st[1] + 8 * (st[0] + 1) + 6 * st[2] + 8 * st[3] for st in stats) \
            + BYTES_PER_HIT * hits
        lb = plan.lookback()
        share = plan.share()
        kname = (f"graph launch: k_batch<{1 if mode == 'eft' else 0},{plan.params()[0]},true,"
                 f"{'true' if lb else 'false'},{'true' if share else 'false'}> with its init "
                 f"launch (tile states, pair-to-arc tables)")
        roof = roofline(mode, {"kernel_ms": dms, "total": hits, "hitpairs": hitpairs}, nnz, byts,
                        kname, None, sum(st[1] for st in stats) if share else None)
        if share:
            roof["ops_note"] = ("arc records shared: the z0-free part of the EFT evaluation "
                                "counts once per arc with candidates")
        res[mode] = dict(ms_per_step=t_batch * 1e3, device_ms=statistics.mean(dms),
                         per_mesh_ms=t_per * 1e3, speedup_vs_per_mesh=t_per / t_batch,
                         params=plan.params(), lookback=lb, share_arcs=share,
                         autotune_s=t_tune, hits=hits,
                         value=nnz / t_batch, roofline=roof)
        plan.close()
        log(f"[bench] batch {mode}: {t_batch * 1e3:.2f} ms (per-mesh launches {t_per * 1e3:.2f} ms), "
            f"params {res[mode]['params']}, look-back {lb}, shared arcs {share}")
    return res


def batch_subresult(torch, sphint, inputs, steps, warmup):
    """The 64-mesh batch with arcs drawn on the device and CSR lists built by the library's
    candidate kernels (the host generator would take minutes for 7e7 arcs)."""
    log("[bench] 64-mesh batch: drawing arcs and candidate lists on the device")
    devs = inputs.device_mesh_arcs(torch, 64, seed_tag=3)
    stats = []
    for d in devs:
        d["lat_offsets"], d["lat_idx"] = sphint.candidates(d["p1"], d["p2"], d["lat_z"])
        d["out"] = sphint.Output(len(d["lat_idx"]))
        n_arcs = len(d["p1"][0])
        used = int((d["lat_offsets"][1:] > d["lat_offsets"][:-1]).sum().item())
        stats.append((n_arcs, used, len(d["lat_idx"]), len(d["lat_z"])))
    torch.cuda.synchronize()
    nnz = sum(st[2] for st in stats)
    log(f"[bench] batch: 64 meshes, {sum(st[0] for st in stats)} arcs, {nnz} pairs")
    res = batch_measure(torch, sphint, devs, stats, ("eft", "naive"), steps, warmup)
    out = {"workload": "64 meshes, log-uniform 1e3..1e7 arcs (d ~ U[1e-3, 0.05] rad, drawn on "
                       "the device) x U{10..3600} latitudes, CSR lists from the GPU candidate "
                       "kernels; one autotuned persistent hipGraph launch against 64 per-mesh calls",
           "meshes": 64, "arcs": sum(st[0] for st in stats), "pairs": nnz}
    out.update(res)
    out["eft_over_naive"] = res["eft"]["value"] / res["naive"]["value"]
    for d in devs:
        d.clear()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(P, inputs, sample):
    """The oracle (exact predicates + 100-digit points) on a stratified sample, all workers,
    plus one in-process worker on a tenth of it."""
    from oracle import batch as OB
    idx = inputs.stratified_sample(P, sample // 3, seed=11)
    S = P.take(idx)
    workers = OB.default_workers()
    t0 = time.perf_counter()
    OB.exact(*S.soa(), workers=workers)
    dt = time.perf_counter() - t0
    S1 = P.take(idx[::10])
    t1 = time.perf_counter()
    OB.exact(*S1.soa(), workers=1)
    d1 = time.perf_counter() - t1
    return {"value": len(S) / dt, "unit": "intersections/s", "cores": workers, "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{len(S)} pairs, stratified over the 3 parts of the same workload "
                      f"(exact integer predicates + 100-digit decimal points), {dt:.1f} s wall",
            "single_core_value": len(S1) / d1, "cpu_model": cpu_model()}


def cpu_baseline_dense(P, sample, what):
    """The oracle on the first `sample` pairs of a dense workload, all workers."""
    from oracle import batch as OB
    S = P.take(slice(0, sample))
    workers = OB.default_workers()
    t0 = time.perf_counter()
    OB.exact(*S.soa(), workers=workers)
    dt = time.perf_counter() - t0
    return {"value": len(S) / dt, "unit": "intersections/s", "cores": workers, "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{len(S)} pairs, {what} (exact integer predicates + 100-digit decimal "
                      f"points), {dt:.1f} s wall", "cpu_model": cpu_model()}


def cpu_replica(P, sample, threads):
    """Context only: the library's own per-pair arithmetic compiled for the host (the CPU
    check library, one evaluation per pair, exact fallbacks inline), on `threads` host
    threads (ctypes releases the GIL), over the first `sample` pairs of each part."""
    import ctypes
    import threading
    import numpy as np
    path = os.path.join(ROOT, "paper_2510_09892_amd", "libsphint_hostcheck.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_eval.argtypes = [ctypes.c_int, ctypes.c_int64] + [dp] * 7 + [ip] * 4 + [dp] * 4
    idx = np.concatenate([np.flatnonzero(P.part == k)[: sample // 3] for k in range(3)])
    soa = [np.ascontiguousarray(a[idx]) for a in P.soa()]
    n = len(idx)
    out = {"threads": threads, "pairs": n, "unit": "intersections/s", "cpu_model": cpu_model(),
           "kind": "host build of the kernel arithmetic (not the oracle)"}
    for mode, name in ((1, "eft"), (0, "naive")):
        ints = [np.zeros(n, np.int32) for _ in range(4)]
        dbl = [np.zeros(n, np.float64) for _ in range(4)]
        bounds = np.linspace(0, n, threads + 1).astype(np.int64)

        def work(lo, hi):
            off = lambda a: a[lo:hi].ctypes.data_as(ctypes.POINTER(
                ctypes.c_double if a.dtype == np.float64 else ctypes.c_int32))
            lib.sphint_hostcheck_eval(mode, int(hi - lo), *[off(a) for a in soa],
                                      *[off(a) for a in ints], *[off(a) for a in dbl])
        ts = [threading.Thread(target=work, args=(bounds[k], bounds[k + 1])) for k in range(threads)]
        t0 = time.perf_counter()
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        out[name] = n / (time.perf_counter() - t0)
    return out


def cpu_baseline_csr(meshes, inputs, sample):
    """The oracle on `sample` candidate pairs drawn uniformly from the meshes' CSR lists."""
    import numpy as np
    from oracle import batch as OB
    g = np.random.Generator(np.random.PCG64(12))
    nnz = np.array([m.nnz for m in meshes], dtype=np.float64)
    which = g.choice(len(meshes), size=sample, p=nnz / nnz.sum())
    rows = []
    for k in np.unique(which):
        m = meshes[k]
        ks = np.sort(g.choice(m.nnz, size=int((which == k).sum()), replace=m.nnz < (which == k).sum()))
        arc = np.searchsorted(m.lat_offsets, ks, side="right") - 1
        rows.append((m.p1[arc], m.p2[arc], m.lat_z[m.lat_idx[ks]]))
    p1 = np.concatenate([r[0] for r in rows])
    p2 = np.concatenate([r[1] for r in rows])
    z0 = np.concatenate([r[2] for r in rows])
    S = inputs.Pairs(p1, p2, z0)
    workers = OB.default_workers()
    t0 = time.perf_counter()
    OB.exact(*S.soa(), workers=workers)
    dt = time.perf_counter() - t0
    return {"value": len(S) / dt, "unit": "intersections/s", "cores": workers, "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{len(S)} candidate pairs drawn uniformly from the workload's CSR lists "
                      f"(exact integer predicates + 100-digit decimal points), {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle", type=float, default=0.2,
                    help="seconds of untimed calls per mode before the warm-up steps (the GPU "
                         "clock settles under sustained load)")
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--workload", default="ill1e7",
                    choices=["ill1e7", "cubed1024", "batch64", "arcarc1e7", "adaptive",
                             "ablation"],
                    help="ill1e7: the headline (1e7 ill-conditioned dense pairs); cubed1024: "
                         "regridding-shaped CSR; batch64: 64 uneven meshes in one launch; "
                         "arcarc1e7: 1e7 arc x arc pairs; adaptive: filtered direct/EFT "
                         "evaluation on 1e7 uniform and 1e7 ill-conditioned pairs; ablation: "
                         "the alternative point formulas")
    ap.add_argument("--modes", default="eft,naive")
    ap.add_argument("--cpu-sample", type=int, default=300_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-subresults", action="store_true",
                    help="skip the cubed-sphere and 64-mesh sub-results of the default line")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a torch copy of this many bytes (profiler calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for "
              f"--gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_09892_amd import inputs, sphint

    sphint.load()
    if args.workload == "batch64":
        return bench_batch(args, torch, np, inputs, sphint)
    if args.workload == "arcarc1e7":
        return bench_arcarc(args, torch, np, inputs, sphint)
    if args.workload == "adaptive":
        return bench_adaptive(args, torch, np, inputs, sphint)
    if args.workload == "ablation":
        return bench_ablation(args, torch, np, inputs, sphint)
    if args.workload == "cubed1024":
        log("[bench] generating the ne=1024 cubed sphere x 1800 latitudes")
        mesh = inputs.cubed_sphere(1024)
        n = mesh.nnz
        P = None
        workload = ("cubed sphere ne=1024: 12,582,912 unique great-circle edges x 1800 latitude "
                    "lines (-89.95 deg + 0.1 deg k), CSR candidates from z-range overlap, mode ")
    else:
        log(f"[bench] generating {args.n} ill-conditioned arcs")
        P = inputs.ill_conditioned(args.n, seed_tag=1)
        n = args.n
        workload = ("1e7 ill-conditioned arcs in three parts (short 1e-10..1e-6 rad; "
                    "near-tangent r<=1e-12; within 1e-6 rad of a pole), one latitude "
                    "per arc, dense 1:1, mode ")
    cpu = replica = None
    if not args.no_cpu_baseline:
        # before any GPU call: the oracle's worker processes are forked from this one
        log(f"[bench] cpu baseline: oracle on {args.cpu_sample} pairs")
        if P is not None:
            replica = cpu_replica(P, 3_000_000, min(os.cpu_count() or 1, 16))
            cpu = cpu_baseline(P, inputs, args.cpu_sample)
        else:
            cpu = cpu_baseline_csr([mesh], inputs, args.cpu_sample)
        log(f"[bench] cpu baseline {cpu['value']:.0f} pairs/s on {cpu['cores']} workers")
    if P is not None:
        dev = [torch.from_numpy(a).cuda() for a in P.soa()]

        def call(out, mode):
            sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode=mode, out=out)
        bytes_in = BYTES_PER_PAIR * n
        csr = False
    else:
        dp = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in mesh.soa()]
        lz, off, idx = (torch.from_numpy(a).cuda() for a in (mesh.lat_z, mesh.lat_offsets, mesh.lat_idx))

        def call(out, mode):
            sphint.arc_constlat(tuple(dp[:3]), tuple(dp[3:]), lz, off, idx, mode=mode, out=out)
        # what the main kernel reads and writes once (hits added below)
        bytes_in = csr_main_bytes(int(np.count_nonzero(np.diff(mesh.lat_offsets))), n,
                                  len(mesh.lat_z), 0)
        csr = True
    torch.cuda.synchronize()

    res = {}
    for mode in args.modes.split(","):
        log(f"[bench] mode={mode} settle={args.settle}s warmup={args.warmup} steps={args.steps}")
        res[mode] = run_mode(torch, sphint, call, n, mode, args.steps, args.warmup, args.settle)
        r = res[mode]
        log(f"[bench] mode={mode} wall={r['wall_s']:.4f}s kernel_mean={statistics.mean(r['kernel_ms']):.4f}ms "
            f"hits={r['total']} settle_calls={r['settle_calls']}")

    copy_calibration(torch, args.copy_calibration)

    head = "eft" if "eft" in res else next(iter(res))
    r = res[head]
    value = n * args.steps / r["wall_s"]
    hits = r["total"]
    kname = lambda m: (f"sphint::k_intersect_w<{1 if m == 'eft' else 0},{3 if m == 'eft' else 4},"
                       f"{'true' if csr else 'false'},"
                       f"{'true' if m == 'eft' and csr and 2 * n >= 5 * mesh.n_arcs else 'false'}>")
    kernel = kname(head)
    tag = f"k_intersect_w_{head}_{args.workload}"
    roof = roofline(head, r, n, bytes_in + BYTES_PER_HIT * hits, kernel, tag)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "intersections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"seconds": args.settle, "calls": r["settle_calls"],
                   "note": "untimed calls of the same mode before the warm-up steps"},
        "ms_per_step": r["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload + head, "pairs": n, "hits": hits},
        "roofline": roof,
    }
    if "naive" in res and head != "naive":
        rn = res["naive"]
        nv = n * args.steps / rn["wall_s"]
        line["naive"] = {"value": nv, "ms_per_step": rn["wall_s"] / args.steps * 1e3,
                         "kernel_ms": statistics.mean(rn["kernel_ms"]), "hits": rn["total"],
                         "roofline": roofline("naive", rn, n, bytes_in + BYTES_PER_HIT * rn["total"],
                                              kname("naive"),
                                              f"k_intersect_w_naive_{args.workload}")}
        line["eft_over_naive"] = value / nv
    if not args.no_latency and args.workload == "ill1e7":
        log("[bench] latency, 1e5 uniform arcs")
        line["latency_1e5"] = latency_small(torch, sphint, inputs)
    if not args.no_serve and args.workload == "ill1e7":
        line["serving"] = serving(torch, args, log)
    if not args.no_subresults and args.workload == "ill1e7":
        line["cubed_sphere"] = cubed_subresult(torch, np, sphint, inputs, 10, 3, args.settle)
        line["batch64"] = batch_subresult(torch, sphint, inputs, 5, 2)
    if args.workload == "cubed1024":
        log("[bench] candidate lists on the GPU and on the host")
        line["candidates"] = candidate_timing(torch, sphint, inputs, mesh, dp, lz)
    if replica is not None:
        line["cpu_replica"] = replica
    if cpu is not None:
        line["cpu_baseline"] = cpu
    if args.workload == "ill1e7":
        line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


# The paper's own timings (Sec. 7.2), as context for the EFT / naive ratio measured here: its
# text states ratios only (the timing plots carry no numbers in the text).
PAPER_CONTEXT = {
    "hardware": "AMD Ryzen 9 5950X, 16 cores, AVX2; gcc -O3 -ffp-contract=off; binary64",
    "workload": "1e9 random intersecting arc/latitude pairs, one root per pair",
    "accux_vs_naive_eq22_serial": "AccuX about 9x slower than the direct Eq. 2.2, one thread",
    "accux_vs_naive_parallel": "with SIMD and threads the gap closes: AccuX reaches the naive "
                               "rate once both are bound by memory bandwidth (AccuX scales to "
                               "8 threads, the naive code stops gaining beyond 2)",
    "absolute_rates": None,
    "note": "context only, not a target; this GPU's ratio is eft_over_naive above",
}


def bench_batch(args, torch, np, inputs, sphint):
    """64 uneven meshes: one autotuned persistent graph launch vs 64 per-mesh launches."""
    g = inputs.rng(3)
    sizes = np.floor(np.exp(g.uniform(np.log(1e3), np.log(1e7), 64))).astype(int)
    lats = g.integers(10, 3601, 64)
    meshes = []
    for m, (sz, L) in enumerate(zip(sizes, lats)):
        meshes.append(inputs.random_mesh(inputs.rng(3, 1 + m), int(sz), int(L)))
        log(f"[bench] mesh {m}: {sz} arcs x {L} latitudes, nnz {meshes[-1].nnz}")
    nnz = sum(m.nnz for m in meshes)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_csr(meshes, inputs, args.cpu_sample)
        log(f"[bench] cpu baseline {cpu['value']:.0f} pairs/s on {cpu['cores']} workers")
    devs = []
    for m in meshes:
        d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()]
        devs.append(dict(p1=tuple(d[:3]), p2=tuple(d[3:]), lat_z=torch.from_numpy(m.lat_z).cuda(),
                         lat_offsets=torch.from_numpy(m.lat_offsets).cuda(),
                         lat_idx=torch.from_numpy(m.lat_idx).cuda(), out=sphint.Output(m.nnz)))
    log(f"[bench] batch: 64 meshes, {sum(m.n_arcs for m in meshes)} arcs, {nnz} pairs on the device")
    stats = [(m.n_arcs, int(np.count_nonzero(np.diff(m.lat_offsets))), m.nnz, len(m.lat_z))
             for m in meshes]
    res = batch_measure(torch, sphint, devs, stats, args.modes.split(","), args.steps, args.warmup)
    head = "eft" if "eft" in res else next(iter(res))
    r = res[head]
    line = {
        "metric": METRIC, "value": r["value"], "unit": "intersections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "64 meshes, log-uniform 1e3..1e7 arcs (d <= 0.05 rad) x 10..3600 "
                               "latitudes, CSR; one autotuned persistent hipGraph launch, mode " + head,
                   "pairs": nnz, "hits": r["hits"]},
        "roofline": r["roofline"],
        "batch": res,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


# Arc x arc: per pair, four endpoints read (12 binary64) and the point, count and flags
# written.  Operations as counted for the latitude path: EFT normals (two AccuDOP cross
# products, TwoSum-renormalised: 114) and the first filter stage of four orientations (60)
# per pair; per hit three compensated cross-product components (AccuDOP on the leading parts
# plus four first-order products: 18 each), SumOfSquares, sqrt, three divisions and the sign
# (85).  Naive: two cross products and four dot products (38); per hit a cross
# product, the norm, sqrt and three divisions with the sign (21).
AA_BYTES_PER_PAIR = 12 * 8 + 3 * 8 + 2
AA_EFT_OPS_PER_PAIR, AA_EFT_OPS_PER_HIT = 174, 85
AA_NAIVE_OPS_PER_PAIR, AA_NAIVE_OPS_PER_HIT = 38, 21
AA_METRIC = "arc x arc intersections/s (EFT vs naive FP64)"


def cpu_baseline_arcarc(P, sample):
    """The arc x arc oracle (exact integer orientations + 100-digit points) on a stratified
    sample of the workload, all workers."""
    import numpy as np
    from oracle import batch as OB
    idx = np.concatenate([np.flatnonzero(P.part == k)[: sample // 4] for k in range(4)])
    S = P.take(idx)
    workers = OB.default_workers()
    t0 = time.perf_counter()
    OB.arcarc_exact(S.a1, S.a2, S.b1, S.b2, workers=workers)
    dt = time.perf_counter() - t0
    return {"value": len(S) / dt, "unit": "intersections/s", "cores": workers, "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{len(S)} pairs, the first {sample // 4} of each of the 4 parts of the same "
                      f"workload (exact integer orientations + 100-digit decimal points), "
                      f"{dt:.1f} s wall", "cpu_model": cpu_model()}


def cpu_replica_arcarc(P, sample, threads):
    """Context only: the kernel's per-pair arithmetic compiled for the host, `threads` host
    threads, over the first `sample` pairs."""
    import ctypes
    import threading
    import numpy as np
    path = os.path.join(ROOT, "paper_2510_09892_amd", "libsphint_hostcheck.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_arcarc.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(dp),
                                            ctypes.POINTER(dp), dp, dp, dp, ip, ip]
    S = P.take(np.arange(min(sample, len(P))))
    A, B = S.soa_a(), S.soa_b()
    n = len(S)
    out = {"threads": threads, "pairs": n, "unit": "intersections/s", "cpu_model": cpu_model(),
           "kind": "host build of the kernel arithmetic (not the oracle)"}
    for mode, name in ((1, "eft"), (0, "naive")):
        res = [np.zeros(n) for _ in range(3)] + [np.zeros(n, np.int32) for _ in range(2)]
        bounds = np.linspace(0, n, threads + 1).astype(np.int64)

        def work(lo, hi):
            pa = (dp * 6)(*[a[lo:hi].ctypes.data_as(dp) for a in A])
            pb = (dp * 6)(*[b[lo:hi].ctypes.data_as(dp) for b in B])
            lib.sphint_hostcheck_arcarc(mode, int(hi - lo), pa, pb,
                                        *[r[lo:hi].ctypes.data_as(dp) for r in res[:3]],
                                        *[r[lo:hi].ctypes.data_as(ip) for r in res[3:]])
        ts = [threading.Thread(target=work, args=(bounds[k], bounds[k + 1])) for k in range(threads)]
        t0 = time.perf_counter()
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        out[name] = n / (time.perf_counter() - t0)
    return out


def bench_arcarc(args, torch, np, inputs, sphint):
    """1e7 arc x arc pairs (crossing-shaped, short, nearly parallel, shared-vertex quarters),
    direct pairing; one sphint_arc_arc call (one kernel) per step."""
    log(f"[bench] generating {args.n} arc x arc pairs")
    P = inputs.arc_pairs(args.n)
    n = len(P)
    cpu = replica = None
    if not args.no_cpu_baseline:
        sample = max(args.cpu_sample, 1_000_000)
        log(f"[bench] cpu baseline: arc x arc oracle on {sample} pairs")
        replica = cpu_replica_arcarc(P, 4_000_000, min(os.cpu_count() or 1, 16))
        cpu = cpu_baseline_arcarc(P, sample)
        log(f"[bench] cpu baseline {cpu['value']:.0f} pairs/s on {cpu['cores']} workers")
    a = [torch.from_numpy(v).cuda() for v in P.soa_a()]
    b = [torch.from_numpy(v).cuda() for v in P.soa_b()]
    torch.cuda.synchronize()
    res = {}
    for mode in args.modes.split(","):
        out = sphint.ArcArcOutput(n)
        call = lambda: sphint.arc_arc(tuple(a[:3]), tuple(a[3:]), tuple(b[:3]), tuple(b[3:]),
                                      mode=mode, out=out)
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for e0, e1 in ev:  # events on the stream the kernel is launched on
            e0.record()
            call()
            e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [e0.elapsed_time(e1) for e0, e1 in ev]
        hits = int(out.count.sum().item())
        res[mode] = dict(wall_s=wall, kernel_ms=kms, hits=hits,
                         exact=int(((out.flags & sphint.AA_EXACT) > 0).sum().item()))
        log(f"[bench] arcarc {mode}: wall {wall / args.steps * 1e3:.4f} ms/step, kernel "
            f"{statistics.mean(kms):.4f} ms, hits {hits}")

    copy_calibration(torch, args.copy_calibration)

    def roof(mode):
        r = res[mode]
        kms = statistics.mean(r["kernel_ms"])
        byts = AA_BYTES_PER_PAIR * n
        if mode == "eft":
            ops = AA_EFT_OPS_PER_PAIR * n + AA_EFT_OPS_PER_HIT * r["hits"]
        else:
            ops = AA_NAIVE_OPS_PER_PAIR * n + AA_NAIVE_OPS_PER_HIT * r["hits"]
        bw, rate = byts / (kms * 1e-3), ops / (kms * 1e-3)
        hbm = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
               "frac": bw / HBM_PEAK}
        alu = {"bound": "alu", "achieved": rate / 1e12, "peak": ALU_PEAK / 1e12,
               "unit": "Tlane-op/s (binary64)", "frac": rate / ALU_PEAK}
        out = dict(hbm if hbm["frac"] >= alu["frac"] else alu)
        other = alu if out["bound"] == "hbm" else hbm
        tr = measured_traffic(f"k_arc_arc_{mode}_arcarc1e7", source_digest())
        out["traffic"] = tr["bytes"] if tr else None
        if tr:
            out["traffic_detail"] = tr
        out["kernel"] = f"k_arc_arc<{1 if mode == 'eft' else 0}, false>"
        out["kernel_ms"] = kms
        out["kernel_ms_p10_p50_p90"] = pctl(r["kernel_ms"])
        out["algorithmic_bytes"] = byts
        out["algorithmic_ops"] = ops
        out["other_bound"] = {k: other[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
        return out

    head = "eft" if "eft" in res else next(iter(res))
    r = res[head]
    value = n * args.steps / r["wall_s"]
    line = {
        "metric": AA_METRIC, "value": value, "unit": "intersections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["wall_s"] / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1e7 arc x arc pairs in four parts (crossing-shaped 0.05..1 rad; "
                               "short 1e-9..1e-6 rad; nearly parallel, tilt 1e-9..1e-3; shared "
                               "vertex), direct pairing, mode " + head,
                   "pairs": n, "hits": r["hits"], "exact_fallback_pairs": r["exact"]},
        "roofline": roof(head),
    }
    if "naive" in res and head != "naive":
        rn = res["naive"]
        nv = n * args.steps / rn["wall_s"]
        line["naive"] = {"value": nv, "ms_per_step": rn["wall_s"] / args.steps * 1e3,
                         "kernel_ms": statistics.mean(rn["kernel_ms"]), "hits": rn["hits"],
                         "roofline": roof("naive")}
        line["eft_over_naive"] = value / nv
    if replica is not None:
        line["cpu_replica"] = replica
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


ADAPTIVE_TOLS = (0.0, 4.0, 16.0, 64.0, 1024.0)


def bench_adaptive(args, torch, np, inputs, sphint):
    """Adaptive evaluation (direct binary64 with a running error bound, EFT for the rest) on
    1e7 uniform and 1e7 ill-conditioned dense pairs, at several tolerances, beside the EFT and
    naive calls of the main path on the same inputs."""
    sets = {}
    for name in ("uniform", "ill"):
        log(f"[bench] generating 1e7 {name} pairs")
        P = (inputs.uniform_arcs(args.n, seed_tag=0) if name == "uniform"
             else inputs.ill_conditioned(args.n, seed_tag=1))
        sets[name] = [torch.from_numpy(a).cuda() for a in P.soa()]
    torch.cuda.synchronize()

    def timed(call):
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record()
            call()
            e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall / args.steps * 1e3, statistics.mean(e0.elapsed_time(e1) for e0, e1 in ev)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on {args.cpu_sample} uniform pairs")
        cpu = cpu_baseline_dense(inputs.uniform_arcs(args.n, seed_tag=0), args.cpu_sample,
                                 "the first pairs of the 1e7 uniform workload")
    table = {}
    pass1 = {}
    for name, d in sets.items():
        n = len(d[6])
        row = {}
        for mode in ("eft", "naive"):
            out = sphint.Output(n)
            ms, dev_ms = timed(lambda: sphint.arc_constlat(tuple(d[:3]), tuple(d[3:6]), d[6],
                                                           mode=mode, out=out))
            row[mode] = {"ms_per_call": ms, "device_ms": dev_ms, "pairs_per_s": n / (ms * 1e-3)}
        out = sphint.AdaptiveOutput(n)
        for tol in ADAPTIVE_TOLS:
            ms, dev_ms = timed(lambda: sphint.arc_constlat_adaptive(tuple(d[:3]), tuple(d[3:6]),
                                                                    d[6], tol, out=out))
            rec = int(out.recomputed.item())
            timer = sphint.KernelTimer(args.steps)  # pass 1 alone (library events)
            for k in range(args.steps):
                timer.arm(k)
                sphint.arc_constlat_adaptive(tuple(d[:3]), tuple(d[3:6]), d[6], tol, out=out)
            torch.cuda.synchronize()
            timer.disarm()
            p1 = timer.durations_ms()
            timer.close()
            row[f"tol{tol:g}"] = {"ms_per_call": ms, "device_ms": dev_ms,
                                  "pass1_ms": statistics.mean(p1),
                                  "pairs_per_s": n / (ms * 1e-3), "recomputed": rec,
                                  "recomputed_frac": rec / n}
            pass1[(name, tol)] = (p1, rec)
            log(f"[bench] adaptive {name} tol={tol:g}: {ms:.4f} ms/call, recomputed {rec / n:.4f}")
        log(f"[bench] {name}: eft {row['eft']['ms_per_call']:.4f} ms, naive "
            f"{row['naive']['ms_per_call']:.4f} ms")
        table[name] = row
    # roofline of pass 1 (the kernel every pair goes through) at tol 64 on the uniform pairs:
    # 56 B read per pair, 36 B of dense output per accepted pair, a 4-byte queue entry per
    # queued pair
    p1, rec = pass1[("uniform", 64.0)]
    n = args.n
    byts = 56 * n + 36 * (n - rec) + 4 * rec
    kms = statistics.mean(p1)
    bw = byts / (kms * 1e-3)
    roof = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": bw / HBM_PEAK, "traffic": None, "kernel": "k_adapt_pass1", "kernel_ms": kms,
            "kernel_ms_p10_p50_p90": pctl(p1), "algorithmic_bytes": byts}
    head = table["uniform"]["tol64"]
    line = {
        "metric": "adaptive arc-latitude intersections/s (points within tol*2^-53, exact decisions)",
        "value": head["pairs_per_s"], "unit": "intersections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_call"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1e7 uniform pairs (d ~ U[1e-3, 0.2] rad), dense, adaptive "
                               "tol = 64 (value); the table adds tol 0/4/16/1024, the 1e7 "
                               "ill-conditioned workload, and the EFT and naive calls",
                   "pairs": args.n},
        "roofline": roof,
        "adaptive": table,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def bench_ablation(args, torch, np, inputs, sphint):
    """Throughput of each point formula (sphint_circle_points: both circle points per pair,
    no containment) on the 1e7 ill-conditioned pairs.  Their accuracy is measured against the
    exact points by the GPU tests (tests/test_gpu_ablation.py prints the table)."""
    log(f"[bench] generating {args.n} ill-conditioned arcs")
    P = inputs.ill_conditioned(args.n, seed_tag=1)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on {args.cpu_sample} pairs")
        cpu = cpu_baseline(P, inputs, args.cpu_sample)
    d = [torch.from_numpy(a).cuda() for a in P.soa()]
    n = len(P)
    rows = {}
    kmss = {}
    for name in sphint.FORMULAS:
        call = lambda: sphint.circle_points(tuple(d[:3]), tuple(d[3:6]), d[6], name)
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record()
            call()
            e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        kmss[name] = [e0.elapsed_time(e1) for e0, e1 in ev]
        kms = statistics.mean(kmss[name])
        # 56 B read, 32 B of points and 1 B written per pair
        rows[name] = {"ms_per_call": wall * 1e3, "device_ms": kms, "pairs_per_s": n / wall,
                      "hbm_frac": 89 * n / (kms * 1e-3) / HBM_PEAK}
        log(f"[bench] formula {name}: {kms:.4f} ms device, {n / wall:.3g} pairs/s")
    head = rows["accux"]
    byts = 89 * n
    bw = byts / (head["device_ms"] * 1e-3)
    roof = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": bw / HBM_PEAK, "traffic": None, "kernel": "k_circle<4>",
            "kernel_ms": head["device_ms"], "kernel_ms_p10_p50_p90": pctl(kmss["accux"]),
            "algorithmic_bytes": byts}
    line = {
        "metric": "circle-intersection point pairs/s by formula (accuracy in the GPU tests)",
        "value": head["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_call"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1e7 ill-conditioned pairs, both circle points per pair, "
                               "formula accux (value); the table adds eq22, eq21, eq71, kahan",
                   "pairs": n},
        "roofline": roof,
        "formulas": rows,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
