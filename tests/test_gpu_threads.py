"""GPU: the library driven from several host threads at once.

Four Python threads (ctypes releases the interpreter lock during library calls, so the
library's host code runs concurrently) each enqueue a sequence of calls on their own
stream: dense EFT, CSR EFT with arc records shared (dense candidate lists), CSR naive, and a
batched plan.  The cross-stream launch order, the occupancy caches and plan launches must
stay consistent: after all threads finish, every output equals the same call run alone
before.
"""

import sys
import threading

import numpy as np
import pytest

from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("count", "flags", "x", "y", "pair", "root")


def note(msg):
    print(f"[gpu-threads] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def read(out):
    t = int(out.total.item())
    return dict(total=t, count=out.count.cpu().numpy(), flags=out.flags.cpu().numpy(),
                x=out.x[:t].cpu().numpy(), y=out.y[:t].cpu().numpy(),
                pair=out.pair[:t].cpu().numpy(), root=out.root[:t].cpu().numpy())


def same(a, b):
    return a["total"] == b["total"] and all(
        np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8))
        for k in KEYS)


def test_threads_equal_serial(torch_cuda):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    dense = inputs.ill_conditioned(300_000, seed_tag=60)
    ddev = [torch.from_numpy(a).cuda() for a in dense.soa()]
    mesh = inputs.random_mesh(inputs.rng(61), 20_000, 2000)
    assert 2 * mesh.nnz >= 5 * mesh.n_arcs  # shared arc records in single calls
    md = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in mesh.soa()]
    lz, off, idx = (torch.from_numpy(a).cuda() for a in (mesh.lat_z, mesh.lat_offsets, mesh.lat_idx))
    pm = [inputs.random_mesh(inputs.rng(62, k), 3000 + 1000 * k, 300) for k in range(3)]

    def plan_devs():
        out = []
        for m in pm:
            d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()]
            out.append(dict(p1=tuple(d[:3]), p2=tuple(d[3:]), lat_z=torch.from_numpy(m.lat_z).cuda(),
                            lat_offsets=torch.from_numpy(m.lat_offsets).cuda(),
                            lat_idx=torch.from_numpy(m.lat_idx).cuda(), out=sphint.Output(m.nnz)))
        return out

    jobs = {
        "dense-eft": lambda o, s: sphint.arc_constlat(tuple(ddev[:3]), tuple(ddev[3:6]), ddev[6],
                                                      mode="eft", out=o, stream=s),
        "csr-eft": lambda o, s: sphint.arc_constlat(tuple(md[:3]), tuple(md[3:]), lz, off, idx,
                                                    mode="eft", out=o, stream=s),
        "csr-naive": lambda o, s: sphint.arc_constlat(tuple(md[:3]), tuple(md[3:]), lz, off, idx,
                                                      mode="naive", out=o, stream=s),
    }
    sizes = {"dense-eft": len(dense), "csr-eft": mesh.nnz, "csr-naive": mesh.nnz}
    ref = {}
    for name, fn in jobs.items():
        o = sphint.Output(sizes[name])
        fn(o, None)
        torch.cuda.synchronize()
        o.check()
        ref[name] = read(o)
    pdevs = plan_devs()
    plan = sphint.BatchPlan(pdevs, mode="eft")
    plan.launch()
    torch.cuda.synchronize()
    plan.check()
    ref_plan = [read(d["out"]) for d in pdevs]

    outs = {name: sphint.Output(sizes[name]) for name in jobs}
    streams = {name: torch.cuda.Stream() for name in list(jobs) + ["plan"]}
    errors = []
    start = threading.Barrier(len(streams))

    def run(name):
        try:
            start.wait()
            for _ in range(12):
                if name == "plan":
                    plan.launch(stream=streams[name])
                else:
                    jobs[name](outs[name], streams[name])
        except Exception as e:  # reported after join
            errors.append((name, repr(e)))

    note("four threads, twelve launches each, own streams")
    ts = [threading.Thread(target=run, args=(n,)) for n in streams]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for name in jobs:
        outs[name].check()
        assert same(read(outs[name]), ref[name]), name
    plan.check()
    for k, d in enumerate(pdevs):
        assert same(read(d["out"]), ref_plan[k]), k
    plan.close()
