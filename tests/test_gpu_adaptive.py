"""GPU: the adaptive evaluation (sphint_arc_constlat_adaptive) through the C ABI.

* Every output (counts, roots, flags with the RECOMPUTED bit, both point slots) equals the
  CPU build of the same per-pair code bit for bit, at several tolerances; small batches are
  also checked against the oracle (tests/test_hostcheck_adaptive.py's comparison: exact
  decisions, accepted points within tol and equal to the binary64 replica, recomputed points
  equal to the AccuX replica).
* Ragged sizes, an empty call, a repeated call (the queue is reset), the recomputed count.
* Full 1e7-pair workloads (uniform and ill-conditioned) against the CPU build, and a
  stratified sample against the oracle.
"""

import os
import sys

import numpy as np
import pytest

from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import test_hostcheck as TH  # noqa: E402
from test_hostcheck_adaptive import check_adaptive, run_adaptive  # noqa: E402

RECOMPUTED = 128


def note(msg):
    print(f"[gpu-adaptive] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


@pytest.fixture(scope="module")
def hc():
    import ctypes
    lib = ctypes.CDLL(TH.LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_adaptive.argtypes = ([ctypes.c_int64] + [dp] * 7 + [ctypes.c_double] +
                                              [ip] * 4 + [dp] * 4 + [ip])
    return lib


def gpu(torch, soa, tol, out=None):
    """Returns host arrays in the host build's format plus the recomputed count."""
    from paper_2510_09892_amd import sphint
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in soa]
    out = sphint.arc_constlat_adaptive(tuple(d[:3]), tuple(d[3:6]), d[6], tol, out=out)
    torch.cuda.synchronize()
    x = out.x.cpu().numpy().reshape(-1, 2)
    y = out.y.cpu().numpy().reshape(-1, 2)
    root = out.root.cpu().numpy().reshape(-1, 2).astype(np.int32)
    count = out.count.cpu().numpy().astype(np.int32)
    flags = out.flags.cpu().numpy().astype(np.int32)
    cert = ((flags & RECOMPUTED) == 0).astype(np.int32)
    res = (count, flags & 127, root[:, 0].copy(), root[:, 1].copy(), x[:, 0].copy(),
           y[:, 0].copy(), x[:, 1].copy(), y[:, 1].copy(), cert)
    return res, int(out.recomputed.item()), out


def same(a, b):
    for u, v in zip(a, b):
        assert np.array_equal(u, v, equal_nan=True)


def small_sets():
    sets = [("uniform", inputs.uniform_arcs(3000, seed_tag=51).soa()),
            ("ill", inputs.ill_conditioned(3000, seed_tag=52).soa()),
            ("integer", TH._integer_cases())]
    return sets


@pytest.mark.parametrize("tol", [0.0, 4.0, 64.0, 1024.0])
def test_small_batches_equal_host_build_and_oracle(torch_cuda, hc, tol):
    for name, soa in small_sets():
        note(f"{name} tol={tol}: {len(soa[0])} pairs")
        res, rec, _ = gpu(torch_cuda, soa, tol)
        ref = run_adaptive(hc, soa, tol)
        same(res, ref)
        assert rec == int(np.sum(res[-1] == 0))
        if tol in (4.0, 64.0):
            check_adaptive(soa, res, tol)


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_ragged_sizes(torch_cuda, hc, n):
    soa = inputs.uniform_arcs(n, seed_tag=53 + n).soa()
    note(f"ragged n={n}")
    res, _, _ = gpu(torch_cuda, soa, 64.0)
    same(res, run_adaptive(hc, soa, 64.0))
    check_adaptive(soa, res, 64.0)


def test_empty_and_repeated_calls(torch_cuda, hc):
    from paper_2510_09892_amd import sphint
    z = torch_cuda.zeros(0, dtype=torch_cuda.float64, device="cuda")
    out = sphint.arc_constlat_adaptive((z, z, z), (z, z, z), z, 16.0)
    torch_cuda.cuda.synchronize()
    assert int(out.recomputed.item()) == 0
    soa = inputs.ill_conditioned(5000, seed_tag=54).soa()
    note("repeated calls on one output")
    res1, rec1, o = gpu(torch_cuda, soa, 16.0)
    res2, rec2, _ = gpu(torch_cuda, soa, 16.0, out=o)
    same(res1, res2)
    assert rec1 == rec2 > 0


@pytest.fixture(scope="module", params=["uniform", "ill"])
def full(request, torch_cuda):
    note(f"full size: generating 1e7 {request.param} pairs")
    P = (inputs.uniform_arcs(10_000_000, seed_tag=0) if request.param == "uniform"
         else inputs.ill_conditioned(10_000_000, seed_tag=1))
    soa = P.soa()
    res, rec, _ = gpu(torch_cuda, soa, 64.0)
    return request.param, P, soa, res, rec


def test_full_size_equals_host_build_and_sampled_oracle(full, hc):
    name, P, soa, res, rec = full
    note(f"full size {name}: every pair against the CPU build ({rec} recomputed)")
    same(res, run_adaptive(hc, soa, 64.0))
    sel = inputs.stratified_sample(P, 400, seed=13) if name == "ill" else np.arange(0, len(P), 7919)
    note(f"full size {name}: {len(sel)} sampled pairs against the oracle")
    sub = [a[sel].copy() for a in soa]
    check_adaptive(sub, [a[sel] for a in res], 64.0)
