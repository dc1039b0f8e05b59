"""The C-ABI library without a GPU: exports, pure calls and argument validation.

Every function include/sphint.h declares must be exported by libsphint.so; calls that
fail validation return SPHINT_E_INVAL before any HIP call, so they run on a CPU host.
"""

import ctypes
import os
import re

import pytest

from paper_2510_09892_amd import sphint

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sphint.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sphint_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sphint_arc_constlat", "sphint_workspace_size", "sphint_batch_plan_create",
              "sphint_batch_autotune", "sphint_batch_launch", "sphint_plan_destroy",
              "sphint_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = sphint.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(sphint.EXPORTS)


def test_pure_calls():
    lib = sphint.load()
    assert lib.sphint_version().decode().startswith("sphint")
    assert lib.sphint_status_string(0).decode() == "ok"
    # header + one status word per 64 pairs + a 4-byte pair-to-arc entry per pair
    assert lib.sphint_workspace_size(0) == 256 + 8
    assert lib.sphint_workspace_size(64) == 256 + 8 + 4 * 64
    assert lib.sphint_workspace_size(65) == 256 + 16 + 4 * 65
    assert lib.sphint_workspace_size(10_000_000) == 256 + 8 * 156250 + 4 * 10_000_000


def _call(**kw):
    lib = sphint.load()
    d = dict(n=4, p1=sphint.PtsSoA(1, 2, 3), p2=sphint.PtsSoA(4, 5, 6), lat_z=7, n_lat=4,
             off=None, idx=None, nnz=4, out=sphint.Hits(8, 9, 10, 11, 8), count=12, flags=None,
             total=13, mode=1, ws=256, ws_bytes=1 << 20, stream=None)
    d.update(kw)
    return lib.sphint_arc_constlat(d["n"], d["p1"], d["p2"], d["lat_z"], d["n_lat"], d["off"],
                                   d["idx"], d["nnz"], d["out"], d["count"], d["flags"],
                                   d["total"], d["mode"], d["ws"], d["ws_bytes"], d["stream"])


@pytest.mark.parametrize("bad", [
    dict(n=-1), dict(nnz=5), dict(n_lat=3), dict(mode=7), dict(total=None),
    dict(ws=None), dict(ws=260), dict(ws_bytes=8), dict(count=None),
    dict(p1=sphint.PtsSoA(1, None, 3)), dict(out=sphint.Hits(None, 9, 10, 11, 8)),
    dict(off=100, idx=None, nnz=3), dict(off=100, idx=200, nnz=3, n_lat=0),
    dict(out=sphint.Hits(8, 9, 10, 11, -1)),
    # size limits: more than 2^40 pairs; more than 2^31 tiles of 192 pairs (EFT); 2^32 arcs
    # in CSR form (arc ids are 32-bit) -- all rejected on the host, with no memory touched
    dict(n=2**40 + 1, nnz=2**40 + 1, n_lat=2**40 + 1, ws_bytes=1 << 62),
    dict(n=5 * 10**11, nnz=5 * 10**11, n_lat=5 * 10**11, ws_bytes=1 << 62),
    dict(off=100, idx=200, n=2**32, nnz=4, ws_bytes=1 << 62),
])
def test_invalid_arguments_rejected_before_launch(bad):
    assert _call(**bad) == sphint.E_INVAL


def _noalloc(**kw):
    lib = sphint.load()
    d = dict(n=4, p1=sphint.PtsSoA(1, 2, 3), p2=sphint.PtsSoA(4, 5, 6), lat_z=7, n_lat=4,
             off=None, idx=None, nnz=4, out=sphint.Hits(8, 9, 10, 11, 8), count=12, flags=None,
             total=13, err=None, mode=1, stream=None)
    d.update(kw)
    return lib.sphint_arc_constlat_noalloc(d["n"], d["p1"], d["p2"], d["lat_z"], d["n_lat"],
                                           d["off"], d["idx"], d["nnz"], d["out"], d["count"],
                                           d["flags"], d["total"], d["err"], d["mode"],
                                           d["stream"])


def _noalloc_limits():
    """Largest dense and CSR pair counts whose scratch fits SPHINT_NOALLOC_SCRATCH_BYTES."""
    m = re.search(r"#define\s+SPHINT_NOALLOC_SCRATCH_BYTES\s+\(\(size_t\)(\d+)\s*<<\s*(\d+)\)",
                  open(HEADER).read())
    cap = int(m.group(1)) << int(m.group(2))
    assert cap == sphint.NOALLOC_SCRATCH_BYTES
    tiles = lambda n: max(1, -(-n // 64))  # noqa: E731
    dense = (cap - 256) // 8 * 64
    assert 256 + 8 * tiles(dense) <= cap < 256 + 8 * tiles(dense + 1)
    csr = (cap - 256 - 8) // 4
    while 256 + 8 * tiles(csr) + 4 * csr > cap:
        csr -= 1
    return dense, csr


@pytest.mark.parametrize("bad", [
    dict(n=-1), dict(nnz=5), dict(mode=7), dict(total=None), dict(count=None),
    dict(p1=sphint.PtsSoA(1, None, 3)), dict(off=100, idx=None, nnz=3),
    dict(out=sphint.Hits(8, 9, 10, 11, -1)),
    "dense+1", "csr+1",
])
def test_noalloc_rejects_before_launch(bad):
    """Invalid arguments, and any call whose scratch would exceed the static array, are
    rejected on the host before the array or the device is touched."""
    dense, csr = _noalloc_limits()
    if bad == "dense+1":
        bad = dict(n=dense + 1, nnz=dense + 1, n_lat=dense + 1)
    elif bad == "csr+1":
        bad = dict(off=100, idx=200, n=1000, nnz=csr + 1)
    assert _noalloc(**bad) == sphint.E_INVAL


def test_batch_run_workspace_and_rejections():
    """sphint_batch_run: workspace size, and rejections before any launch (no GPU)."""
    lib = sphint.load()
    # header, argument table, tile bases, one tile state per 64 pairs (+1 per mesh + 1), and
    # the CSR pair-to-arc tables: grows by 4 bytes per pair plus 8 per 64 pairs
    base = lib.sphint_batch_run_workspace_size(1, 0)
    assert base > 256 and base % 8 == 0
    assert lib.sphint_batch_run_workspace_size(1, 64) == base + 8 + 4 * 64
    assert lib.sphint_batch_run_workspace_size(2, 64) == base + 16 + 4 * 64
    assert lib.sphint_batch_run_workspace_size(-1, 0) == 0

    def desc(csr=True, nnz=4, n_arcs=4):
        d = sphint.MeshDesc()
        d.n_arcs, d.n_lat, d.nnz = n_arcs, 4 if csr else n_arcs, nnz
        d.p1, d.p2 = sphint.PtsSoA(1, 2, 3), sphint.PtsSoA(4, 5, 6)
        d.lat_z = 7
        d.lat_offsets, d.lat_idx = (8, 9) if csr else (None, None)
        d.out = sphint.Hits(10, 11, 12, 13, 2 * nnz)
        d.out_count, d.out_flags, d.out_total = 14, None, 15
        return d

    def call(descs, ws=256, wsb=1 << 30, mode=1):
        arr = (sphint.MeshDesc * max(1, len(descs)))(*descs)
        return lib.sphint_batch_run(arr, len(descs), mode, ws, wsb, None)

    assert call([]) == sphint.E_INVAL                                   # no mesh
    assert call([desc()] * 17) == sphint.E_INVAL                        # above the maximum
    assert call([desc(True), desc(False)]) == sphint.E_INVAL            # mixed forms
    assert call([desc(nnz=-1)]) == sphint.E_INVAL                       # a bad mesh
    assert call([desc()], mode=5) == sphint.E_INVAL
    assert call([desc()], ws=None) == sphint.E_INVAL
    assert call([desc()], ws=260) == sphint.E_INVAL                     # misaligned
    assert call([desc()], wsb=lib.sphint_batch_run_workspace_size(1, 4) - 1) == sphint.E_INVAL


def test_wait_limit_validation():
    lib = sphint.load()
    for bad in (-1.0, float("nan"), float("inf"), 3601.0):
        assert lib.sphint_set_wait_limit(bad) == sphint.E_INVAL
    assert lib.sphint_set_wait_limit(2.0) == sphint.OK  # the default


def test_batch_rejects_bad_arguments():
    lib = sphint.load()
    h = ctypes.c_void_p()
    assert lib.sphint_batch_plan_create(None, 0, 1, ctypes.byref(h)) == sphint.E_INVAL
    arr = (sphint.MeshDesc * 1)()
    arr[0].n_arcs = -1
    assert lib.sphint_batch_plan_create(arr, 1, 1, ctypes.byref(h)) == sphint.E_INVAL
    assert lib.sphint_batch_launch(None, None) == sphint.E_INVAL
    assert lib.sphint_set_profile_events(ctypes.c_void_p(1), None) == sphint.E_INVAL
    v = ctypes.c_int()
    assert lib.sphint_batch_scan(None, ctypes.byref(v)) == sphint.E_INVAL
    assert lib.sphint_batch_set_scan(None, 0) == sphint.E_INVAL
    assert lib.sphint_batch_share(None, ctypes.byref(v)) == sphint.E_INVAL
    assert lib.sphint_batch_set_share(None, 1) == sphint.E_INVAL
    assert lib.sphint_batch_set_params(None, 3, 0) == sphint.E_INVAL


def _aa(**kw):
    lib = sphint.load()
    P = sphint.PtsSoA
    d = dict(n=4, a1=P(1, 2, 3), a2=P(4, 5, 6), n_a=4, b1=P(7, 8, 9), b2=P(10, 11, 12), n_b=4,
             ia=None, ib=None, out=P(13, 14, 15), count=16, flags=None, mode=1, stream=None)
    d.update(kw)
    return lib.sphint_arc_arc(d["n"], d["a1"], d["a2"], d["n_a"], d["b1"], d["b2"], d["n_b"],
                              d["ia"], d["ib"], d["out"], d["count"], d["flags"], d["mode"],
                              d["stream"])


@pytest.mark.parametrize("bad", [
    dict(n=-1), dict(n_a=-1, ia=100), dict(n_a=3), dict(n_b=5), dict(mode=2), dict(count=None),
    dict(out=sphint.PtsSoA(13, None, 15)), dict(a2=sphint.PtsSoA(4, 5, None)),
    dict(b1=sphint.PtsSoA(None, 8, 9), ib=100, n_b=1),
])
def test_arc_arc_invalid_arguments_rejected_before_launch(bad):
    assert _aa(**bad) == sphint.E_INVAL


def test_arc_arc_empty_call_is_a_no_op():
    assert _aa(n=0, n_a=0, n_b=0, count=None, out=sphint.PtsSoA(None, None, None)) == sphint.OK


def test_adaptive_workspace_and_invalid_arguments():
    lib = sphint.load()
    # 64 queue counters 128 bytes apart, then 64 queue regions of ceil(chunks / 64) * 256
    # entries (4 bytes), chunks = ceil(n / 256)
    assert lib.sphint_adaptive_workspace_size(0) == 8192
    assert lib.sphint_adaptive_workspace_size(64) == 8192 + 4 * 64 * 256
    assert lib.sphint_adaptive_workspace_size(256 * 65) == 8192 + 4 * 64 * 512
    assert lib.sphint_adaptive_workspace_size(10_000_000) == 8192 + 4 * 64 * 611 * 256
    P = sphint.PtsSoA
    out = sphint.DenseOut(1, 2, None, 3, None)

    def call(**kw):
        d = dict(n=4, p1=P(1, 2, 3), p2=P(4, 5, 6), z0=7, tol=16.0, out=out, rec=None, ws=256,
                 wsb=1 << 20)
        d.update(kw)
        return lib.sphint_arc_constlat_adaptive(d["n"], d["p1"], d["p2"], d["z0"], d["tol"],
                                                d["out"], d["rec"], d["ws"], d["wsb"], None)
    for bad in (dict(n=-1), dict(n=1 << 32), dict(tol=-1.0), dict(tol=float("nan")),
                dict(ws=None), dict(ws=260), dict(wsb=8192), dict(z0=None),
                dict(p2=P(4, None, 6)), dict(out=sphint.DenseOut(1, None, None, 3, None)),
                dict(out=sphint.DenseOut(1, 2, None, None, None))):
        assert call(**bad) == sphint.E_INVAL, bad


def test_circle_points_invalid_arguments():
    lib = sphint.load()
    P = sphint.PtsSoA
    ok = dict(n=4, p1=P(1, 2, 3), p2=P(4, 5, 6), z0=7, f=0, x=8, y=9, o=10)

    def call(**kw):
        d = dict(ok)
        d.update(kw)
        return lib.sphint_circle_points(d["n"], d["p1"], d["p2"], d["z0"], d["f"], d["x"], d["y"],
                                        d["o"], None)
    for bad in (dict(n=-1), dict(f=-1), dict(f=5), dict(z0=None), dict(x=None), dict(o=None),
                dict(p1=P(1, None, 3))):
        assert call(**bad) == sphint.E_INVAL, bad
    assert call(n=0, z0=None, x=None, y=None, o=None) == sphint.OK


def _defines(text, prefix):
    return {m.group(1): int(m.group(2)) for m in
            re.finditer(r"#define\s+(" + prefix + r"[A-Z0-9_]+)\s+(\d+)u?", text)}


def _enum_values(path, names):
    text = open(path).read()
    return {n: int(re.search(r"\b" + n + r"\s*=\s*(\d+)u?", text).group(1)) for n in names}


def test_flag_bits_agree_across_header_kernels_and_binding():
    """The bits the kernels write are the ones the header and the binding name."""
    hdr = open(HEADER).read()
    csrc = os.path.join(ROOT, "paper_2510_09892_amd", "csrc")
    f = _defines(hdr, "SPHINT_F_")
    k = _enum_values(os.path.join(csrc, "sphint_pair.hpp"),
                     ["F_EXISTS", "F_TANGENT", "F_DEGEN_N", "F_HORIZ", "F_NONFINITE",
                      "F_FALLBACK", "F_INTERNAL"])
    for name, v in k.items():
        assert f["SPHINT_" + name] == v, name
        assert getattr(sphint, name) == v, name
    assert f["SPHINT_F_RECOMPUTED"] == sphint.F_RECOMPUTED  # the adaptive kernel uses the macro
    # the kernels' internal re-evaluation marker never reaches out_flags as a public bit
    internal = _enum_values(os.path.join(csrc, "sphint_pair.hpp"), ["F_NEEDEXACT"])
    assert internal["F_NEEDEXACT"] not in {v for n, v in f.items() if n != "SPHINT_F_RECOMPUTED"}
    aa = _defines(hdr, "SPHINT_AA_")
    ka = _enum_values(os.path.join(csrc, "sphint_arcarc.hpp"),
                      ["AA_HIT", "AA_DEGEN", "AA_COPLANAR", "AA_NONFINITE", "AA_EXACT",
                       "AA_INTERNAL"])
    for name, v in ka.items():
        assert aa["SPHINT_" + name] == v, name
        assert getattr(sphint, name) == v, name


def test_binding_rejects_host_tensors_before_any_call():
    """Host tensors never reach the library as device pointers (no GPU needed)."""
    import torch
    z = torch.zeros(4, dtype=torch.float64)
    p = (z, z, z)
    with pytest.raises(sphint.SphintError):
        sphint.arc_constlat(p, p, z)
    with pytest.raises(sphint.SphintError):
        sphint._req(z, torch.float64, "lat_z")
    with pytest.raises(sphint.SphintError):
        sphint._soa((z, z))
