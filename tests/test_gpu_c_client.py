"""GPU: the C ABI from a plain C program.

tests/c_client/sphint_client.c uses only include/sphint.h and the HIP runtime API (built
with gcc by __graft_entry__.build(), or tests/c_client/build_client.py).  On dense pairs of
the ill-conditioned workload (a ragged size) it makes a naive and an EFT call with a
workspace sized by sphint_workspace_size; its counts, flags and hits must equal the Python
binding's bit for bit.  It also repeats each call with a hit capacity one short of the
total, which sphint_check must report as SPHINT_E_CAPACITY with the same total, and makes a
call without a count array, which must be refused with SPHINT_E_INVAL.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2510_09892_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "c_client", "sphint_client")
OK, E_INVAL, E_CAPACITY = 0, 1, 2


def note(msg):
    print(f"[c-client] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    return torch


def _read_client(path, n):
    raw = open(path, "rb").read()
    pos = 0

    def take(dtype, count):
        nonlocal pos
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a

    res = {}
    for mode in ("naive", "eft"):
        st = take(np.int32, 4)
        t, t2 = (int(v) for v in take(np.int64, 2))
        r = dict(call=int(st[0]), check=int(st[1]), short=int(st[2]), inval=int(st[3]),
                 total=t, total_short=t2, count=take(np.uint8, n), flags=take(np.uint8, n))
        r.update(x=take(np.float64, t), y=take(np.float64, t), pair=take(np.int64, t),
                 root=take(np.uint8, t))
        res[mode] = r
    assert pos == len(raw)
    return res


def test_c_client_equals_binding(torch_cuda, tmp_path):
    from paper_2510_09892_amd import sphint
    torch = torch_cuda
    if not os.path.exists(CLIENT):
        pytest.fail(f"{CLIENT} is not built (python __graft_entry__.py)")
    P = inputs.ill_conditioned(20_011, seed_tag=115)
    soa = [np.ascontiguousarray(a, dtype=np.float64) for a in P.soa()]
    n = len(soa[0])
    inp, outp = tmp_path / "pairs.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.int64(n).tobytes())
        for a in soa:
            f.write(a.tobytes())
    note(f"running the C client on {n} pairs")
    r = subprocess.run([CLIENT, str(inp), str(outp)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    got = _read_client(outp, n)
    dev = [torch.from_numpy(a).cuda() for a in soa]
    for mode in ("naive", "eft"):
        note(f"{mode}: against the binding")
        c = got[mode]
        assert c["call"] == OK and c["check"] == OK
        assert c["inval"] == E_INVAL
        assert c["total"] > 0 and c["short"] == E_CAPACITY and c["total_short"] == c["total"]
        out = sphint.Output(n)
        sphint.arc_constlat(tuple(dev[:3]), tuple(dev[3:6]), dev[6], mode=mode, out=out)
        torch.cuda.synchronize()
        t = out.check()
        assert t == c["total"]
        ref = dict(count=out.count, flags=out.flags, x=out.x[:t], y=out.y[:t],
                   pair=out.pair[:t], root=out.root[:t])
        for key, v in ref.items():
            assert np.array_equal(v.cpu().numpy().view(np.uint8), c[key].view(np.uint8)), key
