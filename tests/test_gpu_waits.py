"""GPU: the bounded waits' error path, forced from the host.

A launch must end even when a wait inside it cannot be satisfied (its grid not all
resident, say).  With the wait limit set to zero every wait gives up at its first check:
the kernels still finish normally (outputs undefined, never written out of bounds), the
error is reported by sphint_check / sphint_batch_check, and calls made after the limit is
restored give the normal results.  Covers the single call (scanner) and a batch plan with
the scanner and with decoupled look-back.
"""

import sys

import numpy as np
import pytest

from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-waits] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def test_zero_wait_limit_reports_error_and_recovers(torch_cuda):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    P = inputs.ill_conditioned(600_000, seed_tag=80)
    dev = [torch.from_numpy(a).cuda() for a in P.soa()]
    ref = sphint.Output(len(P))
    sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode="eft", out=ref)
    torch.cuda.synchronize()
    t_ref = ref.check()
    meshes = [inputs.random_mesh(inputs.rng(81, k), 30_000 + 5_000 * k, 400) for k in range(4)]
    devs = []
    for m in meshes:
        d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in m.soa()]
        devs.append(dict(p1=tuple(d[:3]), p2=tuple(d[3:]), lat_z=torch.from_numpy(m.lat_z).cuda(),
                         lat_offsets=torch.from_numpy(m.lat_offsets).cuda(),
                         lat_idx=torch.from_numpy(m.lat_idx).cuda(), out=sphint.Output(m.nnz)))
    try:
        sphint.set_wait_limit(0.0)
        note("single call, wait limit 0")
        out = sphint.Output(len(P))
        sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode="eft", out=out)
        torch.cuda.synchronize()
        with pytest.raises(sphint.SphintError, match="internal limit"):
            out.check()
        plan = sphint.BatchPlan(devs, mode="naive")
        try:
            for lb in (False, True):
                note(f"batch plan, wait limit 0, look-back {lb}")
                plan.set_params(1, 0)    # one-row tiles: many waits
                plan.set_lookback(lb)    # (re)lays out the plan with the limit in force
                plan.launch()
                torch.cuda.synchronize()
                with pytest.raises(sphint.SphintError, match="internal limit"):
                    plan.check()
        finally:
            plan.close()
    finally:
        sphint.set_wait_limit(2.0)
    note("limit restored")
    out = sphint.Output(len(P))
    sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode="eft", out=out)
    torch.cuda.synchronize()
    assert out.check() == t_ref
    assert torch.equal(out.count, ref.count) and torch.equal(out.x[:t_ref], ref.x[:t_ref])
    plan = sphint.BatchPlan(devs, mode="naive")
    try:
        plan.set_params(1, 0)
        plan.set_lookback(True)
        plan.launch()
        torch.cuda.synchronize()
        plan.check()
    finally:
        plan.close()
