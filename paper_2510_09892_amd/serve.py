"""Serving loop for arc x constant-latitude intersection requests on one GPU.

Each request is one mesh: arcs (binary64 SoA endpoints), a latitude table and CSR
candidate lists.  Requests arrive over time.  One is admitted when a slot is free and its
device footprint (inputs + CSR + 2 nnz hit slots + counts, flags and workspace) fits the
device-memory budget; its inputs go from pinned host memory into the slot's device arena
with one copy on the slot's stream, and the library call is enqueued behind that copy.
Slots run on separate streams, so a request's copy overlaps other requests' kernels, and
requests that arrive while others are on the device are admitted as soon as a slot and
memory are free (continuous batching; the library itself orders its kernel launches on the
device, whose grids each cover the whole device).  A slot's arena is kept for later
requests and grows (within the budget) only when a request does not fit.

Latency runs from a request's arrival to the completion of its kernel on the device
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


def _align(n):
    return (n + ALIGN - 1) // ALIGN * ALIGN


class Payload:
    """One request's inputs packed into one pinned host buffer, and its device layout."""

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
        sizes = dict(count=self.nnz, flags=self.nnz, total=8, x=8 * cap, y=8 * cap,
                     pair=8 * cap, root=cap, ws=sphint.workspace_size(self.nnz))
        self.out_offs = {}
        for k, b in sizes.items():
            self.out_offs[k] = o
            o = _align(o + b)
        self.footprint = o
        self.ws_bytes = sizes["ws"]

    def launch(self, base, mode, stream):
        """Enqueues the library call on the arena at device address ``base``."""
        a = [base + off for off in self.in_offs]
        o = {k: base + v for k, v in self.out_offs.items()}
        sphint.arc_constlat_raw(
            self.n_arcs, (a[0], a[1], a[2]), (a[3], a[4], a[5]), a[6], self.n_lat, a[7], a[8],
            self.nnz, (o["x"], o["y"], o["pair"], o["root"], self.capacity), o["count"],
            o["flags"], o["total"], mode, o["ws"], self.ws_bytes, stream)


class _Slot:
    def __init__(self, torch, device):
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.arena = None
        self.capacity = 0
        self.rid = None
        self.payload = None
        self.ev_h2d0 = torch.cuda.Event(enable_timing=True)
        self.ev_h2d1 = torch.cuda.Event(enable_timing=True)
        self.ev_done = torch.cuda.Event(enable_timing=True)


def _pct(v, q):
    if not len(v):
        return None
    return float(np.percentile(np.asarray(v), q))


class Server:
    """Admission by device-memory budget, one stream per slot, latency accounting."""

    def __init__(self, mode="eft", budget_bytes=64 << 30, slots=8, device="cuda"):
        import torch
        self.torch = torch
        self.mode = mode
        self.budget = int(budget_bytes)
        self.device = torch.device(device)
        self.slots = [_Slot(torch, self.device) for _ in range(slots)]
        self.reserved = 0  # bytes held by slot arenas

    # -- arena management (only free slots are touched: nothing of theirs is in flight)
    def _fit(self, free, need):
        """A free slot whose arena holds `need` bytes, growing one within the budget if
        necessary (releasing idle arenas of other free slots first); None if none can.
        The budget bounds the bytes the slots' arenas hold; memory of a released arena
        stays in PyTorch's cache and serves the next arena."""
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
        # allocated on the device's default stream, so that a released arena's memory is
        # reusable by every slot (only idle slots' arenas are ever released or replaced)
        s.arena = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        s.capacity = need
        self.reserved += need
        return s

    def _issue(self, s, rid, p):
        s.rid, s.payload = rid, p
        base = s.arena.data_ptr()
        with self.torch.cuda.stream(s.stream):
            s.ev_h2d0.record(s.stream)
            s.arena[:p.in_bytes].copy_(p.host, non_blocking=True)
            s.ev_h2d1.record(s.stream)
            p.launch(base, self.mode, s.stream.cuda_stream)
            s.ev_done.record(s.stream)

    def _collect(self, s):
        """Outputs of a finished slot as host arrays (counts, flags, hits)."""
        p = s.payload
        a = s.arena
        with self.torch.cuda.stream(s.stream):
            o = p.out_offs
            total = int(a[o["total"]:o["total"] + 8].view(self.torch.int64).cpu()[0])
            sphint.check_raw(a.data_ptr() + o["ws"], total, p.capacity)
            k = total
            res = dict(total=total,
                       count=a[o["count"]:o["count"] + p.nnz].cpu().numpy(),
                       flags=a[o["flags"]:o["flags"] + p.nnz].cpu().numpy(),
                       x=a[o["x"]:o["x"] + 8 * k].view(self.torch.float64).cpu().numpy(),
                       y=a[o["y"]:o["y"] + 8 * k].view(self.torch.float64).cpu().numpy(),
                       pair=a[o["pair"]:o["pair"] + 8 * k].view(self.torch.int64).cpu().numpy(),
                       root=a[o["root"]:o["root"] + k].cpu().numpy())
        return res

    def run(self, arrivals, payload_of, keep_outputs=False, check_every=0):
        """Serves requests i = 0..len(arrivals)-1 arriving at ``arrivals[i]`` seconds after
        the start; ``payload_of(i)`` gives request i's Payload.  Returns a report dict (and
        the outputs by request id when ``keep_outputs``: True keeps every request's, a
        callable keeps those of the ids it accepts).  ``check_every`` = k > 0 also reads back
        the hit total and error word of every k-th request."""
        torch = self.torch
        keep = keep_outputs if callable(keep_outputs) else (lambda rid: bool(keep_outputs))
        n = len(arrivals)
        for p in {id(payload_of(i)): payload_of(i) for i in range(n)}.values():
            if p.footprint > self.budget:
                raise sphint.SphintError(f"a request needs {p.footprint} bytes, over the budget")
        torch.cuda.synchronize(self.device)
        ev_ref = torch.cuda.Event(enable_timing=True)
        tb = time.perf_counter()
        ev_ref.record()
        ev_ref.synchronize()
        t_ref = (tb + time.perf_counter()) / 2
        t0 = time.perf_counter()
        queue = collections.deque()
        nxt = 0
        done = 0
        lat, lat_nocopy, h2d = [], [], []
        pairs = hits = 0
        outputs = {}
        busy = []
        blocked = 0
        max_inflight = 0
        while done < n:
            now = time.perf_counter() - t0
            progressed = False
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            for s in list(busy):
                if s.ev_done.query():
                    busy.remove(s)
                    p, rid = s.payload, s.rid
                    t_done = t_ref + ev_ref.elapsed_time(s.ev_done) / 1e3 - t0
                    c = s.ev_h2d0.elapsed_time(s.ev_h2d1) / 1e3
                    lat.append(t_done - arrivals[rid])
                    lat_nocopy.append(t_done - arrivals[rid] - c)
                    h2d.append(c)
                    pairs += p.nnz
                    kept = keep(rid)
                    if kept or (check_every and rid % check_every == 0):
                        r = self._collect(s)
                        hits += r["total"]
                        if kept:
                            outputs[rid] = r
                    s.rid = s.payload = None
                    done += 1
                    progressed = True
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
                self._issue(s, rid, p)
                busy.append(s)
                progressed = True
            max_inflight = max(max_inflight, len(busy))
            if not progressed:
                time.sleep(0)
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        rep = dict(requests=n, wall_s=wall, req_per_s=n / wall, pairs=pairs,
                   pairs_per_s=pairs / wall,
                   latency_ms={"p50": 1e3 * _pct(lat, 50), "p99": 1e3 * _pct(lat, 99),
                               "max": 1e3 * max(lat)},
                   latency_without_h2d_ms={"p50": 1e3 * _pct(lat_nocopy, 50),
                                           "p99": 1e3 * _pct(lat_nocopy, 99)},
                   h2d_ms={"p50": 1e3 * _pct(h2d, 50), "p99": 1e3 * _pct(h2d, 99)},
                   slots=len(self.slots), max_inflight=max_inflight,
                   budget_bytes=self.budget, reserved_bytes=self.reserved,
                   admission_waits_on_budget=blocked, mode=self.mode)
        if keep_outputs or check_every:
            rep["hits_checked"] = hits
        return (rep, outputs) if keep_outputs else rep

    def close(self):
        for s in self.slots:
            s.arena = None
            s.capacity = 0
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
