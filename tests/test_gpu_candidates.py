"""GPU: candidate lists (sphint_candidates_count / _fill) through the C ABI.

* Against the exact oracle: on arcs of every workload shape with latitudes placed at their
  exact endpoint heights and great-circle tops (and one ulp on either side), every latitude
  an arc meets is among its GPU-built candidates, and no candidate lies beyond the slack
  outside the arc's exact height range.
* Offsets and indices equal the host build of the same rule bit for bit (the rule itself
  is pinned against the exact oracle in tests/test_candidates.py).
* Built on the GPU and fed to the intersection call, they give the same hits as the
  host-built candidate lists of the workload generators (both contain every intersection;
  extra candidates give no hits).
* Empty inputs, and a capacity below the candidate count.
"""

import os
import sys

import numpy as np
import pytest

from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_candidates import SLACK, exact_range, host_candidates, workload  # noqa: E402


def note(msg):
    print(f"[gpu-cand] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


@pytest.fixture(scope="module")
def hc():
    import ctypes
    from test_candidates import LIBPATH
    lib = ctypes.CDLL(LIBPATH)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_candidates.argtypes = ([ctypes.c_int64] + [dp] * 6 + [dp, ctypes.c_int32,
                                                ctypes.c_double, ip, ip])
    return lib


def gpu_candidates(torch, p1, p2, lat, pad=0.0):
    from paper_2510_09892_amd import sphint
    d1 = [torch.from_numpy(np.ascontiguousarray(p1[:, k])).cuda() for k in range(3)]
    d2 = [torch.from_numpy(np.ascontiguousarray(p2[:, k])).cuda() for k in range(3)]
    off, idx = sphint.candidates(tuple(d1), tuple(d2), torch.from_numpy(lat).cuda(), pad)
    torch.cuda.synchronize()
    return off.cpu().numpy(), idx.cpu().numpy()


def expected(first, count):
    off = np.zeros(len(first) + 1, np.int64)
    np.cumsum(count, out=off[1:])
    idx = np.concatenate([np.arange(f, f + c, dtype=np.int32) for f, c in zip(first, count)]
                         + [np.zeros(0, np.int32)])
    return off, idx


def oracle_workload():
    """The CPU test's arcs (uniform and ill-conditioned, latitudes at their exact endpoint
    heights and tops and one ulp around them), plus short mesh-like arcs and cubed-sphere
    edges with the same latitude placement."""
    p1, p2, lat = workload()
    m = inputs.random_mesh(inputs.rng(75), 40, 50)
    c = inputs.cubed_sphere(ne=4, n_lat=180)
    sel = np.arange(0, len(c.p1), 7)
    q1 = np.concatenate([p1, m.p1, c.p1[sel]])
    q2 = np.concatenate([p2, m.p2, c.p2[sel]])
    extra = []
    for i in range(len(p1), len(q1)):
        lo, hi = exact_range(q1[i], q2[i])
        for v in (float(lo), float(hi)):
            extra += [v, np.nextafter(v, 2.0), np.nextafter(v, -2.0)]
    lat = np.unique(np.concatenate([lat, m.lat_z, c.lat_z, np.array(extra)]))
    return q1, q2, lat[(lat >= -1.0) & (lat <= 1.0)]


def test_gpu_candidates_against_the_exact_oracle(torch_cuda):
    from decimal import Decimal
    from oracle import batch as OB
    p1, p2, lat = oracle_workload()
    n, L = len(p1), len(lat)
    note(f"oracle: {n} arcs x {L} latitudes")
    off, idx = gpu_candidates(torch_cuda, p1, p2, lat)
    cand = np.zeros((n, L), bool)
    for i in range(n):
        cand[i, idx[off[i]:off[i + 1]]] = True
    a = np.repeat(np.arange(n), L)
    k = np.tile(np.arange(L), n)
    ex = OB.exact(p1[a, 0], p1[a, 1], p1[a, 2], p2[a, 0], p2[a, 1], p2[a, 2], lat[k],
                  workers=min(16, os.cpu_count() or 1))
    hit = ex.count.reshape(n, L) > 0
    missed = hit & ~cand
    assert not missed.any(), np.argwhere(missed)[:5]
    assert hit.sum() > 300
    tol = Decimal(SLACK) + Decimal(1e-15)
    for i in range(n):
        lo, hi = exact_range(p1[i], p2[i])
        for kk in idx[off[i]:off[i + 1]]:
            z = Decimal(float(lat[kk]))
            assert lo - tol <= z <= hi + tol, (i, kk)


@pytest.mark.parametrize("case", ["random", "cubed", "dense-lats", "ill"])
def test_gpu_candidates_equal_host_build(torch_cuda, hc, case):
    if case == "random":
        m = inputs.random_mesh(inputs.rng(70), 50_000, 700)
        p1, p2, lat = m.p1, m.p2, m.lat_z
    elif case == "cubed":
        m = inputs.cubed_sphere(ne=48, n_lat=1800)
        p1, p2, lat = m.p1, m.p2, m.lat_z
    elif case == "dense-lats":  # a table larger than the LDS stage (global binary search)
        m = inputs.random_mesh(inputs.rng(71), 20_000, 10)
        p1, p2 = m.p1, m.p2
        lat = np.sin(np.deg2rad(np.linspace(-89.99, 89.99, 9000)))
    else:
        P = inputs.ill_conditioned(30_000, seed_tag=72)
        p1, p2 = P.p1, P.p2
        lat = np.unique(np.concatenate([np.sin(np.deg2rad(np.linspace(-90, 90, 3000))), P.z0[::10]]))
    note(f"{case}: {len(p1)} arcs x {len(lat)} latitudes")
    first, count = host_candidates(hc, p1, p2, lat, 1e-12)
    off, idx = gpu_candidates(torch_cuda, p1, p2, lat, 1e-12)
    e_off, e_idx = expected(first, count)
    np.testing.assert_array_equal(off, e_off)
    np.testing.assert_array_equal(idx, e_idx)


def test_gpu_candidates_feed_the_intersection(torch_cuda):
    """Same hits (arc, latitude, root, point) from GPU-built lists as from host-built ones."""
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    m = inputs.random_mesh(inputs.rng(73), 40_000, 900)
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()]
    lz = torch.from_numpy(m.lat_z).cuda()
    off_g, idx_g = sphint.candidates(tuple(d[:3]), tuple(d[3:]), lz)
    res = {}
    for name, off, idx in (("gpu", off_g, idx_g),
                           ("host", torch.from_numpy(m.lat_offsets).cuda(),
                            torch.from_numpy(m.lat_idx).cuda())):
        out = sphint.Output(len(idx))
        sphint.arc_constlat(tuple(d[:3]), tuple(d[3:]), lz, off, idx, mode="eft", out=out)
        torch.cuda.synchronize()
        t = out.check()
        pair = out.pair[:t].cpu().numpy()
        offn = off.cpu().numpy()
        arc = np.searchsorted(offn, pair, side="right") - 1
        lat = idx.cpu().numpy()[pair]
        res[name] = sorted(zip(arc.tolist(), lat.tolist(), out.root[:t].cpu().numpy().tolist(),
                               out.x[:t].cpu().numpy().tolist(), out.y[:t].cpu().numpy().tolist()))
    note(f"hits: gpu lists {len(res['gpu'])}, host lists {len(res['host'])}")
    assert res["gpu"] == res["host"] and len(res["gpu"]) > 1000


def test_gpu_candidates_empty_and_capacity(torch_cuda):
    from paper_2510_09892_amd import sphint
    import ctypes
    torch = torch_cuda
    lib = sphint.load()
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    off, idx = sphint.candidates((e, e, e), (e, e, e), torch.zeros(3, dtype=torch.float64, device="cuda"))
    assert off.cpu().tolist() == [0] and len(idx) == 0
    m = inputs.random_mesh(inputs.rng(74), 3000, 200)
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()]
    lz = torch.from_numpy(m.lat_z).cuda()
    off, idx = sphint.candidates(tuple(d[:3]), tuple(d[3:]), lz)
    n = len(idx)
    assert n > 100
    wsb = int(lib.sphint_candidates_workspace_size(len(m.p1)))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    off2 = torch.empty(len(m.p1) + 1, dtype=torch.int64, device="cuda")
    nnz = torch.zeros(1, dtype=torch.int64, device="cuda")
    small = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    P = sphint.PtsSoA
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.sphint_candidates_count(len(m.p1), P(*[t.data_ptr() for t in d[:3]]),
                                       P(*[t.data_ptr() for t in d[3:]]), lz.data_ptr(), len(lz),
                                       0.0, off2.data_ptr(), nnz.data_ptr(), ws.data_ptr(), wsb,
                                       st) == 0
    cap = n // 2
    assert lib.sphint_candidates_fill(len(m.p1), off2.data_ptr(), small.data_ptr(), cap,
                                      ws.data_ptr(), wsb, st) == 0
    torch.cuda.synchronize()
    assert int(nnz.item()) == n
    got = small.cpu().numpy()
    np.testing.assert_array_equal(got[:cap], idx.cpu().numpy()[:cap])
    assert np.all(got[cap:] == -7)
