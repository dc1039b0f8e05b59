"""GPU: the serving loop (continuous batching) and launches from several streams.

* Every request's outputs in a served mix (several requests merged into each persistent
  launch, admission held back by a small device-memory budget) are bit-identical to the
  same request run alone.
* Small requests arriving while a large one is resident are admitted at once, merged into
  shared persistent launches and finish before it; their outputs equal their single calls.
* Launches on different streams at once give the results of the same launches run one
  after the other (the library orders its launches on the device).
* A few served requests are checked against the oracle.
* At the serving configuration's own rate (Poisson, 2000 requests/s, requests of
  log-uniform 1e3..1e6 arcs x 1..1000 latitudes, 64 GiB budget, 32 slots), a sample of the
  served requests equals the same requests run alone.
"""

import sys

import numpy as np
import pytest

from oracle import batch as OB
from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

FLAG_MASK = 31
KEYS = ("count", "flags", "x", "y", "pair", "root")


def note(msg):
    print(f"[gpu-serve] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def alone(torch, mesh, mode):
    from paper_2510_09892_amd import sphint
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in mesh.soa()]
    lz, off, idx = (torch.from_numpy(a).cuda() for a in (mesh.lat_z, mesh.lat_offsets, mesh.lat_idx))
    out = sphint.Output(mesh.nnz)
    sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:]), lz, off, idx, mode=mode, out=out)
    torch.cuda.synchronize()
    t = out.check()
    return dict(total=t, count=out.count.cpu().numpy(), flags=out.flags.cpu().numpy(),
                x=out.x[:t].cpu().numpy(), y=out.y[:t].cpu().numpy(),
                pair=out.pair[:t].cpu().numpy(), root=out.root[:t].cpu().numpy())


def same_bytes(a, b):
    return all(np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8))
               for k in KEYS) and a["total"] == b["total"]


@pytest.mark.parametrize("mode", ["eft", "naive"])
def test_served_mix_equals_alone(torch_cuda, mode):
    from paper_2510_09892_amd import serve
    torch = torch_cuda
    note(f"building request pool ({mode})")
    meshes = []
    g = inputs.rng(31)
    pool = []
    for k in range(10):
        m = inputs.random_mesh(inputs.rng(31, k + 1), int(g.integers(500, 30_000)),
                               int(g.integers(1, 400)))
        meshes.append(m)
        pool.append(serve.Payload(m))
    n_req = 60
    arrivals = np.sort(inputs.rng(32).uniform(0.0, 0.004, n_req))  # a burst: requests pile up
    which = [int(v) for v in inputs.rng(33).integers(0, len(pool), n_req)]
    budget = 3 * max(p.footprint for p in pool)
    srv = serve.Server(mode=mode, budget_bytes=budget, slots=4)
    note(f"serving {n_req} requests, budget {budget} bytes, 4 slots")
    rep, outs = srv.run(arrivals, lambda i: pool[which[i]], keep_outputs=True)
    srv.close()
    note(f"served: {rep['req_per_s']:.0f} req/s, {rep['launches']} launches, up to "
         f"{rep['requests_per_launch_max']} requests each, budget waits "
         f"{rep['admission_waits_on_budget']}")
    assert rep["requests"] == n_req and len(outs) == n_req
    assert rep["max_resident_requests"] > 1
    assert rep["requests_per_launch_max"] > 1 and rep["launches"] < n_req
    assert rep["admission_waits_on_budget"] > 0
    ref = {}
    for rid in range(n_req):
        k = which[rid]
        if k not in ref:
            ref[k] = alone(torch, meshes[k], mode)
        assert same_bytes(outs[rid], ref[k]), (rid, k)
    # two served requests against the oracle
    for k in sorted(ref, key=lambda k: meshes[k].nnz)[:2]:
        soa = meshes[k].expand().soa()
        r = ref[k]
        if mode == "eft":
            ex = OB.exact(*soa, workers=1)
            np.testing.assert_array_equal(r["count"], ex.count)
            np.testing.assert_array_equal(r["flags"] & FLAG_MASK, ex.flags)
        else:
            nv = OB.naive_fp64(*soa, workers=1)
            np.testing.assert_array_equal(r["count"], nv.count)
            np.testing.assert_array_equal(r["x"], np.array(nv.hit_x))


def test_concurrent_streams_equal_serial(torch_cuda):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    P = [inputs.ill_conditioned(600_000, seed_tag=34 + k) for k in range(3)]
    dev = [[torch.from_numpy(a).cuda() for a in p.soa()] for p in P]
    note("serial launches")
    serial = []
    for d in dev:
        out = sphint.Output(len(d[6]))
        sphint.arc_constlat(tuple(d[:3]), tuple(d[3:6]), d[6], mode="eft", out=out)
        torch.cuda.synchronize()
        t = out.check()
        serial.append((t, out.count.cpu().numpy(), out.x[:t].cpu().numpy()))
    note("concurrent launches on three streams, four rounds")
    streams = [torch.cuda.Stream() for _ in dev]
    outs = [sphint.Output(len(d[6])) for d in dev]
    for _ in range(4):
        for d, s, o in zip(dev, streams, outs):
            sphint.arc_constlat(tuple(d[:3]), tuple(d[3:6]), d[6], mode="eft", out=o, stream=s)
    torch.cuda.synchronize()
    for (t, c, x), o in zip(serial, outs):
        assert o.check() == t
        assert np.array_equal(o.count.cpu().numpy(), c)
        assert np.array_equal(o.x[:t].cpu().numpy().view(np.uint8), x.view(np.uint8))


@pytest.mark.parametrize("mode", ["eft", "naive"])
def test_full_rate_stream_sampled_equals_alone(torch_cuda, mode):
    from paper_2510_09892_amd import serve
    torch = torch_cuda
    _, specs = inputs.request_stream(seed_tag=4, max_requests=16)
    note(f"building 16 request meshes ({mode})")
    meshes = [inputs.random_mesh(inputs.rng(4, seed), n_arcs, n_lat) for n_arcs, n_lat, seed in specs]
    pool = [serve.Payload(m) for m in meshes]
    arrivals, _ = inputs.request_stream(rate_hz=2000.0, duration_s=2.0, seed_tag=4)
    srv = serve.Server(mode=mode, budget_bytes=64 << 30, slots=32)
    note(f"serving {len(arrivals)} requests at 2000/s")
    rep, outs = srv.run(arrivals, lambda i: pool[i % len(pool)],
                        keep_outputs=lambda rid: rid % 53 == 0)
    srv.close()
    note(f"served: {rep['req_per_s']:.0f} req/s, p99 {rep['latency_ms']['p99']:.3f} ms, "
         f"{len(outs)} outputs kept")
    assert rep["requests"] == len(arrivals) and len(outs) == (len(arrivals) + 52) // 53
    ref = {}
    for rid, r in outs.items():
        k = rid % len(pool)
        if k not in ref:
            ref[k] = alone(torch, meshes[k], mode)
        assert same_bytes(r, ref[k]), (rid, k)


def test_small_requests_behind_a_large_one(torch_cuda):
    """A large request arrives first; small requests arriving while it is resident (its
    inputs still being copied) are admitted at once, copied on other copy streams, merged
    into shared persistent launches and finished before it (no head-of-line blocking);
    every output equals its request's single call."""
    from paper_2510_09892_amd import serve
    torch = torch_cuda
    large = inputs.random_mesh(inputs.rng(35, 1), 2_000_000, 1800)
    smalls = [inputs.random_mesh(inputs.rng(35, 2 + k), 2000 + 700 * k, 20 + 5 * k)
              for k in range(6)]
    meshes = [large] + smalls
    pool = [serve.Payload(m) for m in meshes]
    note(f"large request: {large.nnz} pairs; small: {[m.nnz for m in smalls]}")
    arrivals = np.array([0.0] + [2e-4 + 1e-5 * k for k in range(len(smalls))])
    srv = serve.Server(mode="eft", budget_bytes=16 << 30, slots=16)
    srv.run(arrivals * 0.0, lambda i: pool[i])  # warm-up: arenas, code
    rep, outs = srv.run(arrivals, lambda i: pool[i], keep_outputs=True)
    srv.close()
    big = outs[0]
    note(f"large: launch {big['launch']}, done at {1e3 * big['t_done']:.3f} ms; small: "
         + ", ".join(f"launch {outs[i]['launch']} (size {outs[i]['launch_size']}, admitted "
                     f"{1e3 * outs[i]['t_admit']:.3f}, done {1e3 * outs[i]['t_done']:.3f} ms)"
                     for i in range(1, len(pool))))
    for i in range(1, len(pool)):
        assert outs[i]["t_admit"] < big["t_done"], i   # admitted while the large one ran
        assert outs[i]["t_done"] < big["t_done"], i    # and not queued behind it
    assert max(outs[i]["launch_size"] for i in range(1, len(pool))) > 1  # merged launches
    for i, m in enumerate(meshes):
        assert same_bytes(outs[i], alone(torch, m, "eft")), i
