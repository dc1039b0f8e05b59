"""Python binding of libsphint (include/sphint.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels on the GPU.  PyTorch
provides device memory and the current HIP stream; no torch arithmetic touches the data.
Importing works without a GPU (for symbol checks); calls need a ROCm device and raise if
the library was not built.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "libsphint.so")

NAIVE = 0
EFT = 1
MODES = {"naive": NAIVE, "naive_fp64": NAIVE, "eft": EFT, "eft_fp64": EFT, NAIVE: NAIVE, EFT: EFT}

OK, E_INVAL, E_CAPACITY, E_HIP, E_NOMEM, E_DEVICE = range(6)
F_EXISTS, F_TANGENT, F_DEGEN_N, F_HORIZ, F_NONFINITE = 1, 2, 4, 8, 16
F_FALLBACK, F_INTERNAL = 32, 64  # diagnostic bits of the EFT mode
ROOT_PLUS, ROOT_MINUS = 0, 1
F_RECOMPUTED = 128
NOALLOC_SCRATCH_BYTES = 64 << 20  # SPHINT_NOALLOC_SCRATCH_BYTES
BATCH_RUN_MAX = 16  # SPHINT_BATCH_RUN_MAX
AA_HIT, AA_DEGEN, AA_COPLANAR, AA_NONFINITE, AA_EXACT, AA_INTERNAL = 1, 4, 8, 16, 32, 64

EXPORTS = ("sphint_arc_constlat", "sphint_workspace_size", "sphint_check",
           "sphint_arc_constlat_noalloc", "sphint_set_wait_limit",
           "sphint_set_profile_events",
           "sphint_batch_plan_create", "sphint_batch_autotune", "sphint_batch_launch",
           "sphint_batch_params", "sphint_batch_set_params", "sphint_batch_check",
           "sphint_plan_destroy", "sphint_batch_run_workspace_size", "sphint_batch_run",
           "sphint_batch_scan", "sphint_batch_set_scan", "sphint_batch_share",
           "sphint_batch_set_share",
           "sphint_candidates_workspace_size", "sphint_candidates_count",
           "sphint_candidates_fill",
           "sphint_arc_arc",
           "sphint_adaptive_workspace_size", "sphint_arc_constlat_adaptive",
           "sphint_circle_points",
           "sphint_status_string",
           "sphint_version")


class PtsSoA(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class Hits(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("pair", ctypes.c_void_p),
                ("root", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class DenseOut(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("root", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_arcs", ctypes.c_int64), ("n_lat", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("p1", PtsSoA), ("p2", PtsSoA), ("lat_z", ctypes.c_void_p),
                ("lat_offsets", ctypes.c_void_p), ("lat_idx", ctypes.c_void_p),
                ("out", Hits), ("out_count", ctypes.c_void_p), ("out_flags", ctypes.c_void_p),
                ("out_total", ctypes.c_void_p)]


class SphintError(RuntimeError):
    pass


_lib = None


def load():
    """The loaded library (ctypes), with argument types set.  Raises if not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise SphintError(f"{LIBPATH} is missing: build it with python -m paper_2510_09892_amd.build")
    lib = ctypes.CDLL(LIBPATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    lib.sphint_arc_constlat.argtypes = [i64, PtsSoA, PtsSoA, vp, i64, vp, vp, i64, Hits, vp, vp,
                                        vp, ctypes.c_int, vp, sz, vp]
    lib.sphint_arc_constlat.restype = ctypes.c_int
    lib.sphint_arc_constlat_noalloc.argtypes = [i64, PtsSoA, PtsSoA, vp, i64, vp, vp, i64, Hits,
                                                vp, vp, vp, vp, ctypes.c_int, vp]
    lib.sphint_arc_constlat_noalloc.restype = ctypes.c_int
    lib.sphint_workspace_size.argtypes = [i64]
    lib.sphint_workspace_size.restype = sz
    lib.sphint_set_wait_limit.argtypes = [ctypes.c_double]
    lib.sphint_set_wait_limit.restype = ctypes.c_int
    lib.sphint_set_profile_events.argtypes = [vp, vp]
    lib.sphint_set_profile_events.restype = ctypes.c_int
    lib.sphint_check.argtypes = [vp, i64, i64]
    lib.sphint_check.restype = ctypes.c_int
    lib.sphint_batch_plan_create.argtypes = [ctypes.POINTER(MeshDesc), ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(vp)]
    lib.sphint_batch_plan_create.restype = ctypes.c_int
    lib.sphint_batch_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    lib.sphint_batch_autotune.restype = ctypes.c_int
    lib.sphint_batch_launch.argtypes = [vp, vp]
    lib.sphint_batch_launch.restype = ctypes.c_int
    lib.sphint_batch_params.argtypes = [vp, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int)]
    lib.sphint_batch_params.restype = ctypes.c_int
    lib.sphint_batch_set_params.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.sphint_batch_set_params.restype = ctypes.c_int
    lib.sphint_batch_scan.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.sphint_batch_scan.restype = ctypes.c_int
    lib.sphint_batch_set_scan.argtypes = [vp, ctypes.c_int]
    lib.sphint_batch_set_scan.restype = ctypes.c_int
    lib.sphint_batch_share.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.sphint_batch_share.restype = ctypes.c_int
    lib.sphint_batch_set_share.argtypes = [vp, ctypes.c_int]
    lib.sphint_batch_set_share.restype = ctypes.c_int
    lib.sphint_batch_check.argtypes = [vp]
    lib.sphint_batch_check.restype = ctypes.c_int
    lib.sphint_candidates_workspace_size.argtypes = [i64]
    lib.sphint_candidates_workspace_size.restype = sz
    lib.sphint_candidates_count.argtypes = [i64, PtsSoA, PtsSoA, vp, i64, ctypes.c_double, vp, vp,
                                            vp, sz, vp]
    lib.sphint_candidates_count.restype = ctypes.c_int
    lib.sphint_candidates_fill.argtypes = [i64, vp, vp, i64, vp, sz, vp]
    lib.sphint_candidates_fill.restype = ctypes.c_int
    lib.sphint_arc_arc.argtypes = [i64, PtsSoA, PtsSoA, i64, PtsSoA, PtsSoA, i64, vp, vp,
                                   PtsSoA, vp, vp, ctypes.c_int, vp]
    lib.sphint_arc_arc.restype = ctypes.c_int
    lib.sphint_adaptive_workspace_size.argtypes = [i64]
    lib.sphint_adaptive_workspace_size.restype = sz
    lib.sphint_arc_constlat_adaptive.argtypes = [i64, PtsSoA, PtsSoA, vp, ctypes.c_double,
                                                 DenseOut, vp, vp, sz, vp]
    lib.sphint_arc_constlat_adaptive.restype = ctypes.c_int
    lib.sphint_circle_points.argtypes = [i64, PtsSoA, PtsSoA, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.sphint_circle_points.restype = ctypes.c_int
    lib.sphint_batch_run_workspace_size.argtypes = [ctypes.c_int, i64]
    lib.sphint_batch_run_workspace_size.restype = sz
    lib.sphint_batch_run.argtypes = [ctypes.POINTER(MeshDesc), ctypes.c_int, ctypes.c_int, vp,
                                     sz, vp]
    lib.sphint_batch_run.restype = ctypes.c_int
    lib.sphint_plan_destroy.argtypes = [vp]
    lib.sphint_plan_destroy.restype = None
    lib.sphint_status_string.argtypes = [ctypes.c_int]
    lib.sphint_status_string.restype = ctypes.c_char_p
    lib.sphint_version.argtypes = []
    lib.sphint_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, what):
    if status != OK:
        msg = load().sphint_status_string(status).decode()
        raise SphintError(f"{what}: {msg} (status {status})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _req(t, dtype, name, device=None, length=None):
    """Raises SphintError unless t is a contiguous CUDA tensor of `dtype` (on `device`, with
    `length` elements when given): a host tensor, a strided view or a short array must not
    reach a kernel as a raw pointer."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
        raise SphintError(f"{name} must be a {dtype} CUDA tensor")
    if not t.is_contiguous():
        raise SphintError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise SphintError(f"{name} is on {t.device}, expected {device}")
    if length is not None and t.numel() != length:
        raise SphintError(f"{name} has {t.numel()} entries, expected {length}")
    return t


def _check_pairs(p1, p2, lat_z, lat_offsets, lat_idx):
    """Validates one mesh's tensors; returns (PtsSoA p1, PtsSoA p2, n_arcs, nnz)."""
    import torch
    s1, n_arcs = _soa(p1)
    s2, n2 = _soa(p2)
    if n2 != n_arcs:
        raise SphintError("p1 and p2 differ in length")
    _req(lat_z, torch.float64, "lat_z")
    dev = lat_z.device
    for comp in (*(p1 if not isinstance(p1, torch.Tensor) else (p1,)),
                 *(p2 if not isinstance(p2, torch.Tensor) else (p2,))):
        if comp.device != dev:
            raise SphintError("endpoints and lat_z must be on one device")
    if lat_offsets is None:
        if lat_idx is not None:
            raise SphintError("lat_idx given without lat_offsets")
        if lat_z.numel() != n_arcs:
            raise SphintError("dense form: lat_z needs one latitude per arc")
        nnz = n_arcs
    else:
        if lat_idx is None:
            raise SphintError("CSR form needs lat_idx")
        _req(lat_offsets, torch.int64, "lat_offsets", dev, n_arcs + 1)
        _req(lat_idx, torch.int32, "lat_idx", dev)
        nnz = lat_idx.numel()
    return s1, s2, n_arcs, nnz


def _check_output(out, nnz, dev):
    """The Output must be sized for nnz pairs and live on the inputs' device."""
    import torch
    if out.nnz != nnz:
        raise SphintError("output buffers sized for a different number of pairs")
    cap = out.capacity
    for t, dt, name, n in ((out.x, torch.float64, "out.x", cap), (out.y, torch.float64, "out.y", cap),
                           (out.pair, torch.int64, "out.pair", cap),
                           (out.root, torch.uint8, "out.root", cap),
                           (out.count, torch.uint8, "out.count", nnz),
                           (out.total, torch.int64, "out.total", 1)):
        _req(t, dt, name, dev, n)
    if out.workspace is not None:
        _req(out.workspace, torch.uint8, "out.workspace", dev, out.ws_bytes)
    if out.flags is not None:
        _req(out.flags, torch.uint8, "out.flags", dev, nnz)


def _soa(p):
    """(x, y, z) device float64 tensors -> PtsSoA; accepts a (3, n) tensor too."""
    import torch
    if isinstance(p, torch.Tensor):
        if p.dim() != 2 or p.shape[0] != 3:
            raise SphintError("endpoints must be (x, y, z) tensors or a (3, n) tensor")
        p = (p[0], p[1], p[2])
    for t in p:
        if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda
                or not t.is_contiguous()):
            raise SphintError("endpoint components must be contiguous float64 CUDA tensors")
    if not (p[0].numel() == p[1].numel() == p[2].numel()) or p[0].dim() != 1:
        raise SphintError("endpoint components must be 1-D and of equal length")
    if not (p[0].device == p[1].device == p[2].device):
        raise SphintError("endpoint components must be on one device")
    return PtsSoA(p[0].data_ptr(), p[1].data_ptr(), p[2].data_ptr()), len(p[0])


class Output:
    """Caller-owned device buffers for one call (reusable across calls of the same size)."""

    def __init__(self, nnz, capacity=None, flags=True, device="cuda", workspace=True):
        """workspace=False: no workspace (for arc_constlat_noalloc, whose workspace is the
        library's own static device array)."""
        import torch
        cap = 2 * nnz if capacity is None else int(capacity)
        self.nnz = nnz
        self.capacity = cap
        self.x = torch.empty(cap, dtype=torch.float64, device=device)
        self.y = torch.empty(cap, dtype=torch.float64, device=device)
        self.pair = torch.empty(cap, dtype=torch.int64, device=device)
        self.root = torch.empty(cap, dtype=torch.uint8, device=device)
        self.count = torch.empty(nnz, dtype=torch.uint8, device=device)
        self.flags = torch.empty(nnz, dtype=torch.uint8, device=device) if flags else None
        self.total = torch.zeros(1, dtype=torch.int64, device=device)
        self.error = torch.zeros(1, dtype=torch.int32, device=device)
        if workspace:
            ws = int(load().sphint_workspace_size(nnz))
            # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
            self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
            self.ws_bytes = ws
        else:
            self.workspace, self.ws_bytes = None, 0

    def hits(self):
        """Synchronises; returns (x, y, pair, root) trimmed to the total."""
        t = int(self.total.item())
        if t > self.capacity:
            raise SphintError(f"capacity {self.capacity} < {t} hits")
        return self.x[:t], self.y[:t], self.pair[:t], self.root[:t]

    def check(self):
        """Synchronises; raises if the kernel reported an internal limit or overflowed."""
        t = int(self.total.item())
        if self.workspace is None:  # filled by arc_constlat_noalloc: its error word
            if int(self.error.item()) != 0:
                _check(E_DEVICE, "sphint_arc_constlat_noalloc")
            if t > self.capacity:
                _check(E_CAPACITY, "sphint_arc_constlat_noalloc")
            return t
        _check(load().sphint_check(ctypes.c_void_p(self.workspace.data_ptr()), t, self.capacity),
               "sphint_check")
        return t

    def hits_struct(self):
        return Hits(self.x.data_ptr(), self.y.data_ptr(), self.pair.data_ptr(),
                    self.root.data_ptr(), self.capacity)


def arc_constlat(p1, p2, lat_z, lat_offsets=None, lat_idx=None, mode="eft", out=None,
                 stream=None):
    """Enqueue sphint_arc_constlat on the current (or given) stream; returns the Output.

    Dense form: lat_z has one latitude per arc.  CSR form: lat_offsets (int64, n_arcs + 1)
    and lat_idx (int32, nnz) index into lat_z.  Nothing is synchronised.
    """
    lib = load()
    s1, s2, n_arcs, nnz = _check_pairs(p1, p2, lat_z, lat_offsets, lat_idx)
    if out is None:
        out = Output(nnz, device=lat_z.device)
    _check_output(out, nnz, lat_z.device)
    if out.workspace is None:
        raise SphintError("arc_constlat needs an Output with a workspace")
    st = lib.sphint_arc_constlat(n_arcs, s1, s2, _ptr(lat_z), len(lat_z), _ptr(lat_offsets),
                                 _ptr(lat_idx), nnz, out.hits_struct(), _ptr(out.count),
                                 _ptr(out.flags), _ptr(out.total), MODES[mode],
                                 _ptr(out.workspace), out.ws_bytes, _stream(stream))
    _check(st, "sphint_arc_constlat")
    return out


def arc_constlat_noalloc(p1, p2, lat_z, lat_offsets=None, lat_idx=None, mode="eft", out=None,
                         stream=None):
    """Enqueue sphint_arc_constlat_noalloc (no workspace: the library's static device array
    serves as one); arguments and results as arc_constlat.  The Output's `error` word
    receives the kernels' error bits."""
    import torch
    lib = load()
    s1, s2, n_arcs, nnz = _check_pairs(p1, p2, lat_z, lat_offsets, lat_idx)
    if out is None:
        out = Output(nnz, device=lat_z.device, workspace=False)
    _check_output(out, nnz, lat_z.device)
    _req(out.error, torch.int32, "out.error", lat_z.device, 1)
    st = lib.sphint_arc_constlat_noalloc(n_arcs, s1, s2, _ptr(lat_z), len(lat_z),
                                         _ptr(lat_offsets), _ptr(lat_idx), nnz,
                                         out.hits_struct(), _ptr(out.count), _ptr(out.flags),
                                         _ptr(out.total), _ptr(out.error), MODES[mode],
                                         _stream(stream))
    _check(st, "sphint_arc_constlat_noalloc")
    return out


def set_wait_limit(seconds):
    """sphint_set_wait_limit: the limit of every bounded wait inside later launches."""
    _check(load().sphint_set_wait_limit(float(seconds)), "sphint_set_wait_limit")


def candidates(p1, p2, lat_z, pad=0.0, stream=None):
    """CSR candidate lists on the GPU (sphint_candidates_count, then _fill): returns
    (lat_offsets int64 [n_arcs + 1], lat_idx int32 [nnz]) device tensors.  lat_z must be
    ascending.  Synchronises once, to read nnz."""
    import torch
    lib = load()
    s1, n_arcs = _soa(p1)
    s2, n2 = _soa(p2)
    if n2 != n_arcs:
        raise SphintError("p1 and p2 differ in length")
    if lat_z.dtype != torch.float64 or not lat_z.is_cuda:
        raise SphintError("lat_z must be a float64 CUDA tensor")
    dev = lat_z.device
    wsb = int(lib.sphint_candidates_workspace_size(n_arcs))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    off = torch.empty(n_arcs + 1, dtype=torch.int64, device=dev)
    nnz = torch.zeros(1, dtype=torch.int64, device=dev)
    st = _stream(stream)
    _check(lib.sphint_candidates_count(n_arcs, s1, s2, _ptr(lat_z), len(lat_z), float(pad),
                                       _ptr(off), _ptr(nnz), _ptr(ws), wsb, st),
           "sphint_candidates_count")
    (torch.cuda.current_stream(dev) if stream is None else stream).synchronize()
    n = int(nnz.item())
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    _check(lib.sphint_candidates_fill(n_arcs, _ptr(off), _ptr(idx), n, _ptr(ws), wsb, st),
           "sphint_candidates_fill")
    return off, idx[:n]


class ArcArcOutput:
    """Dense per-pair results of sphint_arc_arc: point (x, y, z), count (0/1), flags."""

    def __init__(self, n_pairs, flags=True, device="cuda"):
        import torch
        self.n = n_pairs
        self.x, self.y, self.z = (torch.empty(n_pairs, dtype=torch.float64, device=device)
                                  for _ in range(3))
        self.count = torch.empty(n_pairs, dtype=torch.uint8, device=device)
        self.flags = torch.empty(n_pairs, dtype=torch.uint8, device=device) if flags else None


def arc_arc(a1, a2, b1, b2, ia=None, ib=None, mode="eft", out=None, stream=None):
    """Enqueue sphint_arc_arc: pair k is arc ia[k] of A = a1 -> a2 with arc ib[k] of
    B = b1 -> b2 (arc k when an index tensor is None; int32 index tensors).  Returns the
    ArcArcOutput; nothing is synchronised."""
    import torch
    lib = load()
    sa1, n_a = _soa(a1)
    sa2, n2 = _soa(a2)
    sb1, n_b = _soa(b1)
    sb2, n3 = _soa(b2)
    if n2 != n_a or n3 != n_b:
        raise SphintError("arc endpoint arrays differ in length")
    for t in (ia, ib):
        if t is not None and (t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous()):
            raise SphintError("pair indices must be contiguous int32 CUDA tensors")
    if ia is not None and ib is not None and len(ia) != len(ib):
        raise SphintError("ia and ib differ in length")
    n = len(ia) if ia is not None else (len(ib) if ib is not None else n_a)
    if out is None:
        out = ArcArcOutput(n, device=a1[0].device)
    if out.n != n:
        raise SphintError("output buffers sized for a different number of pairs")
    st = lib.sphint_arc_arc(n, sa1, sa2, n_a, sb1, sb2, n_b, _ptr(ia), _ptr(ib),
                            PtsSoA(out.x.data_ptr(), out.y.data_ptr(), out.z.data_ptr()),
                            _ptr(out.count), _ptr(out.flags), MODES[mode], _stream(stream))
    _check(st, "sphint_arc_arc")
    return out


class AdaptiveOutput:
    """Dense per-pair results of sphint_arc_constlat_adaptive (two slots per pair)."""

    def __init__(self, n, device="cuda"):
        import torch
        self.n = n
        self.x = torch.empty(2 * n, dtype=torch.float64, device=device)
        self.y = torch.empty(2 * n, dtype=torch.float64, device=device)
        self.root = torch.empty(2 * n, dtype=torch.uint8, device=device)
        self.count = torch.empty(n, dtype=torch.uint8, device=device)
        self.flags = torch.empty(n, dtype=torch.uint8, device=device)
        self.recomputed = torch.zeros(1, dtype=torch.int64, device=device)
        ws = int(load().sphint_adaptive_workspace_size(n))
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        self.ws_bytes = ws

    def struct(self):
        return DenseOut(self.x.data_ptr(), self.y.data_ptr(), self.root.data_ptr(),
                        self.count.data_ptr(), self.flags.data_ptr())


def arc_constlat_adaptive(p1, p2, z0, tol, out=None, stream=None):
    """Enqueue sphint_arc_constlat_adaptive (dense pairs: arc i with latitude z0[i]); points
    within max(tol, 4) * 2^-53 of the exact ones.  Returns the AdaptiveOutput; nothing is
    synchronised."""
    import torch
    lib = load()
    s1, n = _soa(p1)
    s2, n2 = _soa(p2)
    if n2 != n or len(z0) != n:
        raise SphintError("p1, p2 and z0 differ in length")
    if z0.dtype != torch.float64 or not z0.is_cuda:
        raise SphintError("z0 must be a float64 CUDA tensor")
    if out is None:
        out = AdaptiveOutput(n, device=z0.device)
    if out.n != n:
        raise SphintError("output buffers sized for a different number of pairs")
    st = lib.sphint_arc_constlat_adaptive(n, s1, s2, _ptr(z0), float(tol), out.struct(),
                                          _ptr(out.recomputed), _ptr(out.workspace), out.ws_bytes,
                                          _stream(stream))
    _check(st, "sphint_arc_constlat_adaptive")
    return out


FORMULAS = {"eq22": 0, "eq21": 1, "eq71": 2, "kahan": 3, "accux": 4}


def circle_points(p1, p2, z0, formula, stream=None):
    """Enqueue sphint_circle_points: both great-circle x latitude-circle points of every
    dense pair by one formula (name or SPHINT_FORMULA_* value).  Returns (x [2n], y [2n],
    ok [n]) device tensors; nothing is synchronised."""
    import torch
    lib = load()
    s1, n = _soa(p1)
    s2, n2 = _soa(p2)
    if n2 != n or len(z0) != n:
        raise SphintError("p1, p2 and z0 differ in length")
    if z0.dtype != torch.float64 or not z0.is_cuda:
        raise SphintError("z0 must be a float64 CUDA tensor")
    f = FORMULAS.get(formula, formula)
    x = torch.empty(2 * n, dtype=torch.float64, device=z0.device)
    y = torch.empty(2 * n, dtype=torch.float64, device=z0.device)
    ok = torch.empty(n, dtype=torch.uint8, device=z0.device)
    _check(lib.sphint_circle_points(n, s1, s2, _ptr(z0), int(f), _ptr(x), _ptr(y), _ptr(ok),
                                    _stream(stream)), "sphint_circle_points")
    return x, y, ok


def arc_constlat_raw(n_arcs, p1, p2, lat_z, n_lat, lat_offsets, lat_idx, nnz, hits, count,
                     flags, total, mode, workspace, workspace_bytes, stream):
    """sphint_arc_constlat on raw device addresses (ints; 0 for NULL), for callers that manage
    their own device memory.  ``p1``/``p2`` are (x, y, z) address triples, ``hits`` is
    (x, y, pair, root, capacity), ``stream`` a hipStream_t value.  Nothing is synchronised."""
    st = load().sphint_arc_constlat(
        n_arcs, PtsSoA(*p1), PtsSoA(*p2), lat_z or None, n_lat, lat_offsets or None,
        lat_idx or None, nnz, Hits(*hits), count or None, flags or None, total, MODES[mode],
        workspace, workspace_bytes, ctypes.c_void_p(stream))
    _check(st, "sphint_arc_constlat")


def workspace_size(nnz):
    """sphint_workspace_size: workspace bytes for a call over nnz pairs."""
    return int(load().sphint_workspace_size(nnz))


def check_raw(workspace, host_total, capacity):
    """sphint_check on a raw workspace address (synchronous)."""
    _check(load().sphint_check(ctypes.c_void_p(workspace), host_total, capacity), "sphint_check")


class KernelTimer:
    """HIP events the library records around its main kernel (sphint_set_profile_events).

    ``arm(k)`` selects event pair k for the next call; ``durations_ms()`` synchronises and
    returns the kernel time of every armed pair.
    """

    def __init__(self, n):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(n):
            a, b = ctypes.c_void_p(), ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(a)) or self.hip.hipEventCreate(ctypes.byref(b)):
                raise SphintError("hipEventCreate failed")
            self.ev.append((a, b))
        self.armed = []

    def arm(self, k):
        a, b = self.ev[k]
        _check(load().sphint_set_profile_events(a, b), "sphint_set_profile_events")
        self.armed.append(k)

    def disarm(self):
        _check(load().sphint_set_profile_events(None, None), "sphint_set_profile_events")

    def durations_ms(self):
        out = []
        for k in self.armed:
            a, b = self.ev[k]
            self.hip.hipEventSynchronize(b)
            ms = ctypes.c_float()
            if self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b):
                raise SphintError("hipEventElapsedTime failed")
            out.append(ms.value)
        return out

    def close(self):
        self.disarm()
        for a, b in self.ev:
            self.hip.hipEventDestroy(a)
            self.hip.hipEventDestroy(b)
        self.ev = []


def mesh_descs(meshes):
    """Validated sphint_mesh_desc array for meshes given as dicts of device tensors (p1, p2,
    lat_z, optional lat_offsets/lat_idx) with an Output under "out"."""
    arr = (MeshDesc * len(meshes))()
    for k, m in enumerate(meshes):
        off = m.get("lat_offsets")
        s1, s2, n_arcs, nnz = _check_pairs(m["p1"], m["p2"], m["lat_z"], off, m.get("lat_idx"))
        out = m["out"]
        _check_output(out, nnz, m["lat_z"].device)
        arr[k] = MeshDesc(n_arcs, len(m["lat_z"]), out.nnz, s1, s2, m["lat_z"].data_ptr(),
                          off.data_ptr() if off is not None else None,
                          m["lat_idx"].data_ptr() if off is not None else None,
                          out.hits_struct(), out.count.data_ptr(),
                          out.flags.data_ptr() if out.flags is not None else None,
                          out.total.data_ptr())
    return arr


def batch_run_workspace_size(n_meshes, total_nnz):
    """sphint_batch_run_workspace_size."""
    return int(load().sphint_batch_run_workspace_size(int(n_meshes), int(total_nnz)))


def batch_run(meshes, mode="eft", workspace=None, stream=None):
    """Enqueue sphint_batch_run: up to BATCH_RUN_MAX meshes (dicts as for BatchPlan) in one
    persistent launch without a plan.  Returns the workspace tensor (its header holds the
    launch's error word for sphint_check); nothing is synchronised."""
    import torch
    if not 1 <= len(meshes) <= BATCH_RUN_MAX:
        raise SphintError(f"batch_run takes 1..{BATCH_RUN_MAX} meshes")
    arr = mesh_descs(meshes)
    need = batch_run_workspace_size(len(meshes), sum(m["out"].nnz for m in meshes))
    dev = meshes[0]["lat_z"].device
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _req(workspace, torch.uint8, "workspace", dev)
    if workspace.numel() < need:
        raise SphintError(f"workspace of {workspace.numel()} bytes, {need} needed")
    batch_run_raw(arr, len(meshes), mode, workspace.data_ptr(), workspace.numel(),
                  _stream(stream).value)
    return workspace


def batch_run_raw(descs, n_meshes, mode, workspace, workspace_bytes, stream):
    """sphint_batch_run on a MeshDesc array of raw device addresses (``stream`` a hipStream_t
    value)."""
    _check(load().sphint_batch_run(descs, n_meshes, MODES[mode], ctypes.c_void_p(workspace),
                                   workspace_bytes, ctypes.c_void_p(stream)), "sphint_batch_run")


class BatchPlan:
    """sphint_batch_* over a list of meshes (each a dict of device tensors + Output)."""

    def __init__(self, meshes, mode="eft"):
        lib = load()
        self._keep = meshes
        arr = mesh_descs(meshes)
        h = ctypes.c_void_p()
        _check(lib.sphint_batch_plan_create(arr, len(meshes), MODES[mode], ctypes.byref(h)),
               "sphint_batch_plan_create")
        self.handle = h

    def autotune(self, cache_path=None, stream=None):
        c = cache_path.encode() if cache_path else None
        _check(load().sphint_batch_autotune(self.handle, c, _stream(stream)), "sphint_batch_autotune")

    def launch(self, stream=None):
        _check(load().sphint_batch_launch(self.handle, _stream(stream)), "sphint_batch_launch")

    def params(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(load().sphint_batch_params(self.handle, ctypes.byref(a), ctypes.byref(b)),
               "sphint_batch_params")
        return a.value, b.value

    def set_params(self, pairs_per_thread, wg_per_cu):
        _check(load().sphint_batch_set_params(self.handle, pairs_per_thread, wg_per_cu),
               "sphint_batch_set_params")

    def lookback(self):
        """True when tile offsets come from decoupled look-back, False for the scanner."""
        v = ctypes.c_int()
        _check(load().sphint_batch_scan(self.handle, ctypes.byref(v)), "sphint_batch_scan")
        return bool(v.value)

    def set_lookback(self, on):
        _check(load().sphint_batch_set_scan(self.handle, 1 if on else 0), "sphint_batch_set_scan")

    def share(self):
        """True when an EFT plan over CSR lists shares arc records among a tile's rows."""
        v = ctypes.c_int()
        _check(load().sphint_batch_share(self.handle, ctypes.byref(v)), "sphint_batch_share")
        return bool(v.value)

    def set_share(self, on):
        _check(load().sphint_batch_set_share(self.handle, 1 if on else 0),
               "sphint_batch_set_share")

    def check(self):
        """Synchronises; raises if a kernel of the last launch reported an internal limit or
        a mesh's hits overflowed its capacity."""
        _check(load().sphint_batch_check(self.handle), "sphint_batch_check")

    def close(self):
        if self.handle:
            load().sphint_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
