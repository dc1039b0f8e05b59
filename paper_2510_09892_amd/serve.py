"""Serving loop for arc x constant-latitude intersection requests on one GPU.

Each request is one mesh: arcs (binary64 SoA endpoints), a latitude table and CSR
candidate lists.  Requests arrive over time and are served by continuous batching:

* admission: a request is admitted when one of the request slots is free and its device
  arena (inputs, CSR lists, 2 nnz hit slots, counts and flags) fits the device-memory
  budget together with the other arenas and the launch workspace; its inputs then go from
  pinned host memory into the arena in 4 MiB chunks on the copy stream, the loop keeping only a
  few chunks in flight and always taking the next chunk from the request with the fewest
  bytes left (so a small request's copy does not wait behind a large one's: the copy engine
  serves one queue in order);
* batching: admitted requests whose copy has finished wait for the next launch; a launch
  takes up to SPHINT_BATCH_RUN_MAX of them (and at most a set number of pairs) and runs them
  in ONE
  persistent kernel (sphint_batch_run), whose tiles cover all its requests, so the work
  of co-resident requests shares the device instead of queueing whole-device launches;
* pipelining: up to `depth` launches are enqueued at once on the compute stream, so a
  launch formed from the requests that arrived during the previous one is already queued
  behind it when it ends;
* completion: after each launch the kernels' error word and every request's hit total are
  copied to pinned host memory; the loop checks both for every request when the launch has
  finished, records latencies and frees the slots.

Latency runs from a request's arrival to the completion of its launch on the device
(device timestamps mapped onto the host clock through one reference event), reported with
and without the request's own host-to-device copy time.

All computation runs in libsphint's kernels; this module moves bytes and keeps time.
"""

from __future__ import annotations

import collections
import time

import numpy as np

from . import inputs, sphint

ALIGN = 256

# The servers' streams, created once per device and shared by every Server of the process.
# Streams are spread over the device's few hardware queues in the order they are created;
# with fresh streams per server, a server built after another measured slower on the same
# requests (p50 latency 0.34 against 0.21 ms), and the same with these.
_STREAMS = {}


def _streams(torch, device):
    key = device.index if device.index is not None else torch.cuda.current_device()
    if key not in _STREAMS:
        # default priority for every stream: copy, compute, read-back
        _STREAMS[key] = tuple(torch.cuda.Stream(device=device) for _ in range(3))
    return _STREAMS[key]


def _align(n):
    return (n + ALIGN - 1) // ALIGN * ALIGN


class Payload:
    """One request's inputs packed into one pinned host buffer, and its arena layout."""

    def __init__(self, mesh: inputs.CsrMesh):
        import torch
        self.n_arcs = mesh.n_arcs
        self.n_lat = len(mesh.lat_z)
        self.nnz = mesh.nnz
        parts = list(mesh.soa()) + [mesh.lat_z, mesh.lat_offsets, mesh.lat_idx]
        offs, o = [], 0
        for a in parts:
            offs.append(o)
            o = _align(o + a.nbytes)
        self.in_bytes = o
        self.host = torch.empty(o, dtype=torch.uint8, pin_memory=True)
        view = self.host.numpy()
        for a, off in zip(parts, offs):
            view[off:off + a.nbytes] = np.ascontiguousarray(a).view(np.uint8)
        self.in_offs = offs
        # outputs after the inputs
        cap = 2 * self.nnz
        self.capacity = cap
        sizes = dict(count=self.nnz, flags=self.nnz, x=8 * cap, y=8 * cap, pair=8 * cap, root=cap)
        self.out_offs = {}
        for k, b in sizes.items():
            self.out_offs[k] = o
            o = _align(o + b)
        self.footprint = o

    def desc(self, base, total_addr):
        """The request's sphint_mesh_desc on the arena at device address ``base``, with its
        hit total written to ``total_addr``."""
        a = [base + off for off in self.in_offs]
        o = {k: base + v for k, v in self.out_offs.items()}
        return sphint.MeshDesc(
            self.n_arcs, self.n_lat, self.nnz, sphint.PtsSoA(a[0], a[1], a[2]),
            sphint.PtsSoA(a[3], a[4], a[5]), a[6], a[7], a[8],
            sphint.Hits(o["x"], o["y"], o["pair"], o["root"], self.capacity), o["count"],
            o["flags"], total_addr)


class _Slot:
    """A request's device arena (kept for later requests) and its copy events."""

    def __init__(self, torch):
        self.arena = None
        self.capacity = 0
        self.rid = None
        self.payload = None
        self.t_admit = 0.0
        self.copy_off = 0
        self.ev_h2d0 = torch.cuda.Event(enable_timing=True)
        self.ev_h2d1 = torch.cuda.Event(enable_timing=True)


class _Launch:
    """One batched launch in flight: its requests, events and result buffers."""

    def __init__(self, torch, device):
        n = sphint.BATCH_RUN_MAX
        self.totals = torch.zeros(n + 1, dtype=torch.int64, device=device)  # [0]: error word
        self.host = torch.zeros(n + 1, dtype=torch.int64, pin_memory=True)
        self.ev_done = torch.cuda.Event(enable_timing=True)
        self.ev_read = torch.cuda.Event()
        self.slots = []
        self.seq = -1


def _small_half(lat, sizes):
    """p50/p99 latency (ms) of the requests with at most the median number of pairs."""
    if not lat:
        return None
    lat, sizes = np.asarray(lat), np.asarray(sizes)
    sel = lat[sizes <= np.median(sizes)]
    return {"p50": 1e3 * _pct(sel, 50), "p99": 1e3 * _pct(sel, 99)}


def _pct(v, q):
    if not len(v):
        return None
    return float(np.percentile(np.asarray(v), q))


class Server:
    """Continuous batching: admission by device-memory budget, up to `max_batch` requests
    per persistent launch, `depth` launches in flight, latency accounting."""

    def __init__(self, mode="eft", budget_bytes=64 << 30, slots=32, max_batch=None, depth=2,
                 max_launch_pairs=1 << 25, copy_chunk=1 << 22, copy_inflight=2 << 22,
                 device="cuda"):
        import torch
        self.torch = torch
        self.mode = mode
        self.budget = int(budget_bytes)
        self.device = torch.device(device)
        self.slots = [_Slot(torch) for _ in range(slots)]
        self.max_batch = min(max_batch or sphint.BATCH_RUN_MAX, sphint.BATCH_RUN_MAX)
        self.depth = depth
        self.max_launch_pairs = int(max_launch_pairs)
        self.copy_stream, self.compute_stream, self.read_stream = _streams(torch, self.device)
        self.copy_chunk = int(copy_chunk)        # bytes per copy
        self.copy_inflight = int(copy_inflight)  # bytes of copies enqueued and not finished
        self.launches = [_Launch(torch, self.device) for _ in range(depth)]
        self.ws = None
        self.ws_pairs = -1
        self.reserved = 0  # bytes held by slot arenas and the launch workspace

    # -- launch workspace: sized once per run for the largest launch the loop forms
    def _workspace(self, pairs):
        if pairs > self.ws_pairs:
            if self.ws is not None:
                self.reserved -= self.ws.numel()
            self.torch.cuda.synchronize(self.device)
            self.ws = None
            need = sphint.batch_run_workspace_size(sphint.BATCH_RUN_MAX, pairs)
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
            self.ws_pairs = pairs
            self.reserved += need
        return self.ws

    # -- arena management (only free slots are touched: nothing of theirs is in flight)
    def _fit(self, free, need):
        """A free slot whose arena holds `need` bytes, growing one within the budget if
        necessary (releasing idle arenas of other free slots first); None if none can.
        Memory of a released arena stays in PyTorch's cache and serves the next arena."""
        ok = [s for s in free if s.capacity >= need]
        if ok:
            return min(ok, key=lambda s: s.capacity)
        s = max(free, key=lambda s: s.capacity)
        if self.reserved - s.capacity + need > self.budget:
            for o in sorted(free, key=lambda o: o.capacity):
                if o is s or self.reserved - s.capacity + need <= self.budget:
                    continue
                self.reserved -= o.capacity
                o.arena, o.capacity = None, 0
            if self.reserved - s.capacity + need > self.budget:
                return None
        self.reserved -= s.capacity
        s.arena = None
        # allocated on the device's default stream: a released arena's memory is reusable
        # by every slot (only idle slots' arenas are ever released or replaced)
        s.arena = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        s.capacity = need
        self.reserved += need
        return s

    def _admit(self, s, rid, p):
        s.rid, s.payload = rid, p
        s.copy_off = 0

    def _copy_chunk(self, s):
        """Enqueues the next chunk of s's inputs; returns (event, bytes, last chunk?)."""
        p = s.payload
        cs = self.copy_stream
        a, b = s.copy_off, min(s.copy_off + self.copy_chunk, p.in_bytes)
        with self.torch.cuda.stream(cs):
            if a == 0:
                s.ev_h2d0.record(cs)
            s.arena[a:b].copy_(p.host[a:b], non_blocking=True)
            last = b == p.in_bytes
            if last:
                s.ev_h2d1.record(cs)
                ev = s.ev_h2d1
            else:
                ev = self.torch.cuda.Event()
                ev.record(cs)
        s.copy_off = b
        return ev, b - a, last

    def _launch(self, L, group):
        """Enqueues one batched launch over the slots in `group` on the compute stream."""
        torch = self.torch
        cs = self.compute_stream
        L.slots = group
        tot = L.totals.data_ptr()
        descs = (sphint.MeshDesc * len(group))()
        for i, s in enumerate(group):
            cs.wait_event(s.ev_h2d1)  # already complete (the loop checked): orders the streams
            descs[i] = s.payload.desc(s.arena.data_ptr(), tot + 8 * (i + 1))
        ws = self.ws
        sphint.batch_run_raw(descs, len(group), self.mode, ws.data_ptr(), ws.numel(),
                             cs.cuda_stream)
        with torch.cuda.stream(cs):
            L.ev_done.record(cs)
            # the error word (header word 1) and the hit totals, for every request
            L.totals[0:1].copy_(ws[:8].view(torch.int64), non_blocking=True)
            L.host[:len(group) + 1].copy_(L.totals[:len(group) + 1], non_blocking=True)
            L.ev_read.record(cs)

    def _collect(self, s, total):
        """Outputs of a finished request as host arrays (counts, flags, hits)."""
        p = s.payload
        a = s.arena
        o = p.out_offs
        k = total
        with self.torch.cuda.stream(self.read_stream):
            res = dict(total=total,
                       count=a[o["count"]:o["count"] + p.nnz].cpu().numpy(),
                       flags=a[o["flags"]:o["flags"] + p.nnz].cpu().numpy(),
                       x=a[o["x"]:o["x"] + 8 * k].view(self.torch.float64).cpu().numpy(),
                       y=a[o["y"]:o["y"] + 8 * k].view(self.torch.float64).cpu().numpy(),
                       pair=a[o["pair"]:o["pair"] + 8 * k].view(self.torch.int64).cpu().numpy(),
                       root=a[o["root"]:o["root"] + k].cpu().numpy())
        return res

    def run(self, arrivals, payload_of, keep_outputs=False):
        """Serves requests i = 0..len(arrivals)-1 arriving at ``arrivals[i]`` seconds after
        the start; ``payload_of(i)`` gives request i's Payload.  Returns a report dict (and
        the outputs by request id when ``keep_outputs``: True keeps every request's, a
        callable keeps those of the ids it accepts; each with its launch's sequence number
        and size, and its admission and completion times).  Every request's hit total and
        the error word of its launch are checked."""
        torch = self.torch
        keep = keep_outputs if callable(keep_outputs) else (lambda rid: bool(keep_outputs))
        n = len(arrivals)
        biggest = 0
        for p in {id(payload_of(i)): payload_of(i) for i in range(n)}.values():
            biggest = max(biggest, p.nnz)
            if p.footprint > self.budget:
                raise sphint.SphintError(f"a request needs {p.footprint} bytes, over the budget")
        # pairs per launch: at most max_launch_pairs, and a workspace of at most a sixteenth
        # of the budget (about 4 bytes per pair), but always room for the largest request
        cap_pairs = max(biggest, min(self.max_launch_pairs, self.budget // 16 // 5))
        self._workspace(cap_pairs)
        if self.reserved > self.budget:
            raise sphint.SphintError("the launch workspace alone exceeds the budget")
        torch.cuda.synchronize(self.device)
        # the device clock on the host's: the midpoint of the shortest of a few record and
        # wait round trips of one event (its error is at most half that round trip)
        ev_ref, t_ref, best = None, 0.0, float("inf")
        for _ in range(16):
            ev = torch.cuda.Event(enable_timing=True)
            tb = time.perf_counter()
            ev.record()
            ev.synchronize()
            ta = time.perf_counter()
            if ta - tb < best:
                ev_ref, t_ref, best = ev, (tb + ta) / 2, ta - tb
        t0 = time.perf_counter()
        queue = collections.deque()   # arrived, not admitted
        copying = []                  # admitted, inputs not all enqueued for copying
        chunks = collections.deque()  # copies in flight: (event, bytes, slot, last chunk?)
        chunk_bytes = 0
        ready = collections.deque()   # inputs on the device, not launched
        inflight = collections.deque()
        idle_launches = list(self.launches)
        nxt = done = 0
        lat, lat_nocopy, h2d, sizes = [], [], [], []
        pairs = hits = 0
        outputs = {}
        busy = set()
        blocked = 0
        n_launch = 0
        per_launch = []
        shared = 0
        max_resident = 0
        while done < n:
            now = time.perf_counter() - t0
            progressed = False
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            # completions, in launch order
            while inflight and inflight[0].ev_read.query():
                L = inflight.popleft()
                vals = L.host[:len(L.slots) + 1].numpy()
                err = (int(vals[0]) >> 32) & 0xffffffff  # header word 1: the error bits
                if err:
                    raise sphint.SphintError(f"launch reported device error bits {err:#x}")
                t_done = t_ref + ev_ref.elapsed_time(L.ev_done) / 1e3 - t0
                for i, s in enumerate(L.slots):
                    p, rid = s.payload, s.rid
                    total = int(vals[i + 1])
                    if total > p.capacity:
                        raise sphint.SphintError(f"request {rid}: {total} hits over capacity")
                    c = s.ev_h2d0.elapsed_time(s.ev_h2d1) / 1e3
                    lat.append(t_done - arrivals[rid])
                    sizes.append(p.nnz)
                    lat_nocopy.append(t_done - arrivals[rid] - c)
                    h2d.append(c)
                    pairs += p.nnz
                    hits += total
                    if keep(rid):
                        outputs[rid] = self._collect(s, total)
                        outputs[rid].update(launch=L.seq, launch_size=len(L.slots),
                                            t_admit=s.t_admit, t_done=t_done)
                    s.rid = s.payload = None
                    busy.discard(s)
                    done += 1
                if len(L.slots) > 1:
                    shared += len(L.slots)
                L.slots = []
                idle_launches.append(L)
                progressed = True
            # admissions
            free = [s for s in self.slots if s not in busy]
            while queue and free:
                rid = queue[0]
                p = payload_of(rid)
                s = self._fit(free, p.footprint)
                if s is None:
                    blocked += 1
                    break
                queue.popleft()
                free.remove(s)
                busy.add(s)
                s.t_admit = time.perf_counter() - t0
                self._admit(s, rid, p)
                copying.append(s)
                progressed = True
            max_resident = max(max_resident, len(busy))
            # copies: finished chunks retire (a request whose last chunk finished can join a
            # launch), then the queue is topped up from the request with the fewest bytes left
            while chunks and chunks[0][0].query():
                ev, nb, s, last = chunks.popleft()
                chunk_bytes -= nb
                if last:
                    ready.append(s)
                progressed = True
            while copying and chunk_bytes < self.copy_inflight:
                s = min(copying, key=lambda q: q.payload.in_bytes - q.copy_off)
                ev, nb, last = self._copy_chunk(s)
                chunks.append((ev, nb, s, last))
                chunk_bytes += nb
                if last:
                    copying.remove(s)
                progressed = True
            # launches: every request whose inputs are on the device joins the next launch
            while ready and idle_launches:
                group = [ready.popleft()]
                npairs = group[0].payload.nnz
                while (ready and len(group) < self.max_batch
                       and npairs + ready[0].payload.nnz <= cap_pairs):
                    npairs += ready[0].payload.nnz
                    group.append(ready.popleft())
                L = idle_launches.pop()
                L.seq = n_launch
                self._launch(L, group)
                inflight.append(L)
                n_launch += 1
                per_launch.append(len(group))
                progressed = True
            if not progressed:
                time.sleep(0)
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        rep = dict(requests=n, wall_s=wall, req_per_s=n / wall, pairs=pairs,
                   pairs_per_s=pairs / wall, hits=hits,
                   latency_ms={"p50": 1e3 * _pct(lat, 50), "p99": 1e3 * _pct(lat, 99),
                               "max": 1e3 * max(lat)},
                   latency_without_h2d_ms={"p50": 1e3 * _pct(lat_nocopy, 50),
                                           "p99": 1e3 * _pct(lat_nocopy, 99)},
                   h2d_ms={"p50": 1e3 * _pct(h2d, 50), "p99": 1e3 * _pct(h2d, 99)},
                   latency_smaller_half_ms=_small_half(lat, sizes),
                   launches=n_launch, requests_per_launch_mean=n / max(n_launch, 1),
                   requests_per_launch_max=max(per_launch) if per_launch else 0,
                   shared_launch_frac=shared / n, max_resident_requests=max_resident,
                   slots=len(self.slots), depth=self.depth, max_batch=self.max_batch,
                   launch_pairs_cap=cap_pairs, budget_bytes=self.budget,
                   reserved_bytes=self.reserved, admission_waits_on_budget=blocked,
                   requests_checked=done, mode=self.mode)
        return (rep, outputs) if keep_outputs else rep

    def close(self):
        for s in self.slots:
            s.arena = None
            s.capacity = 0
        self.ws = None
        self.ws_pairs = -1
        self.reserved = 0


def request_pool(n_payloads, seed_tag=4, arcs_lo=1e3, arcs_hi=1e6, lat_lo=1, lat_hi=1000):
    """``n_payloads`` distinct requests drawn from the serving size distribution (the first
    requests of ``inputs.request_stream``), packed as Payloads."""
    _, specs = inputs.request_stream(arcs_lo=arcs_lo, arcs_hi=arcs_hi, lat_lo=lat_lo,
                                     lat_hi=lat_hi, seed_tag=seed_tag, max_requests=n_payloads)
    out = []
    for n_arcs, n_lat, seed in specs:
        m = inputs.random_mesh(inputs.rng(seed_tag, seed), n_arcs, n_lat)
        out.append(Payload(m))
    return out
