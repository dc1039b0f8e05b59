"""Seeded synthetic inputs for arc x constant-latitude workloads.

This module draws arcs and latitudes; it computes no intersection (no normal, no s^2, no
hit test).  It is the only code shared by the tests, the benchmark and the oracle side.
Arrays are binary64, structure-of-arrays.

Workloads (sizes are defaults; tests pass smaller ones):

* ``uniform_arcs``   p1 uniform on the sphere, p2 at angular distance d ~ U[1e-3, 0.2] rad
  along a uniform bearing, one latitude z0 ~ U(arc z-range) per arc (dense 1:1).
* ``ill_conditioned``  three equal parts, after the paper's secondary data set (Sec. 7):
  (a) arc length log-uniform in [1e-10, 1e-6] rad, z0 in the z-range;
  (b) arcs containing their apex (or nadir), latitude sliced within r ~ U(0, 1e-12] of
      the extremum, 1% placed just beyond it (no intersection);
  (c) both endpoints within 1e-6 rad of a pole, z0 in the z-range.
* ``cubed_sphere``   all unique edges of an equiangular gnomonic cubed sphere with ne x ne
  cells per face, plus latitude lines, and CSR candidate lists from z-range overlap.
* ``mesh_batch`` / ``request_stream``: many uneven meshes for batched and served runs;
  ``device_arcs`` / ``device_mesh_batch`` draw the same shapes on the GPU with torch's
  seeded generator (the 64-mesh batch holds 7e7 arcs, too many to draw on the host in a
  benchmark run).
* ``arc_pairs``      arc x arc pairs in four equal parts: crossing-shaped arcs (B through a
  point near A's midpoint, about half of them cross), short arcs (1e-9 to 1e-6 rad), nearly
  parallel arcs (endpoints tilted by 1e-9 to 1e-3) and mesh-like shared vertices (b1 = a2
  exactly).

Endpoints are computed in binary64 and left as rounded (not re-normalised), so they are not
exactly unit vectors, as the paper allows (Sec. 1.2 footnote).  The arc z-range used to
place z0 is approximate (binary64 trigonometry); exact decisions belong to the code under
test and to the oracle.
"""

from __future__ import annotations

import numpy as np

SEED_BASE = 20251009


def rng(tag: int, stream: int = 0) -> np.random.Generator:
    """PCG64 stream for workload ``tag`` (seed SEED_BASE + tag)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE + tag, stream]))


class Pairs:
    """Dense 1:1 arc-latitude pairs as SoA arrays; ``part`` labels sub-populations."""

    def __init__(self, p1, p2, z0, part=None):
        self.p1 = np.ascontiguousarray(p1, dtype=np.float64)   # (n, 3)
        self.p2 = np.ascontiguousarray(p2, dtype=np.float64)
        self.z0 = np.ascontiguousarray(z0, dtype=np.float64)
        self.part = np.zeros(len(z0), np.int8) if part is None else np.asarray(part, np.int8)

    def __len__(self):
        return len(self.z0)

    def soa(self):
        """(x1, y1, z1, x2, y2, z2, z0) contiguous 1-D arrays."""
        return tuple(np.ascontiguousarray(a) for a in
                     (self.p1[:, 0], self.p1[:, 1], self.p1[:, 2],
                      self.p2[:, 0], self.p2[:, 1], self.p2[:, 2], self.z0))

    def take(self, idx):
        return Pairs(self.p1[idx], self.p2[idx], self.z0[idx], self.part[idx])


# ----------------------------------------------------------------- arc construction

def random_unit(g: np.random.Generator, n: int) -> np.ndarray:
    v = g.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _local_frame(p):
    """Unit north and east vectors at points p (n, 3); undefined exactly at the poles."""
    r = np.hypot(p[:, 0], p[:, 1])
    east = np.stack([-p[:, 1] / r, p[:, 0] / r, np.zeros_like(r)], axis=1)
    north = np.stack([-p[:, 2] * p[:, 0] / r, -p[:, 2] * p[:, 1] / r, r], axis=1)
    return north, east


def arc_from(p1, d, bearing):
    """p2 = cos(d) p1 + sin(d) (cos(b) north + sin(b) east): the point at distance d."""
    north, east = _local_frame(p1)
    t = np.cos(bearing)[:, None] * north + np.sin(bearing)[:, None] * east
    return np.cos(d)[:, None] * p1 + np.sin(d)[:, None] * t


def z_range(p1, p2):
    """Approximate [zlo, zhi] of the minor arc p1 -> p2 (binary64 trigonometry)."""
    u = p1 / np.linalg.norm(p1, axis=1, keepdims=True)
    w = p2 / np.linalg.norm(p2, axis=1, keepdims=True)
    c = np.sum(u * w, axis=1)
    v = w - c[:, None] * u
    nv = np.linalg.norm(v, axis=1)
    v = v / np.where(nv > 0, nv, 1.0)[:, None]
    theta12 = np.arctan2(np.linalg.norm(np.cross(u, w), axis=1), c)
    R = np.hypot(u[:, 2], v[:, 2])
    phi = np.mod(np.arctan2(v[:, 2], u[:, 2]), 2 * np.pi)    # where z(theta) = +R
    phim = np.mod(phi + np.pi, 2 * np.pi)                     # where z(theta) = -R
    lo = np.minimum(u[:, 2], w[:, 2])
    hi = np.maximum(u[:, 2], w[:, 2])
    hi = np.where(phi <= theta12, np.maximum(hi, R), hi)
    lo = np.where(phim <= theta12, np.minimum(lo, -R), lo)
    return lo, hi


def _z_in_range(g, p1, p2):
    lo, hi = z_range(p1, p2)
    return lo + (hi - lo) * g.random(len(lo))


# ----------------------------------------------------------------- dense workloads

def uniform_arcs(n: int = 100_000, seed_tag: int = 0, d_lo=1e-3, d_hi=0.2) -> Pairs:
    g = rng(seed_tag)
    p1 = random_unit(g, n)
    d = g.uniform(d_lo, d_hi, n)
    p2 = arc_from(p1, d, g.uniform(0.0, 2 * np.pi, n))
    return Pairs(p1, p2, _z_in_range(g, p1, p2))


def _short_arcs(g, n):
    p1 = random_unit(g, n)
    d = np.exp(g.uniform(np.log(1e-10), np.log(1e-6), n))
    p2 = arc_from(p1, d, g.uniform(0.0, 2 * np.pi, n))
    return p1, p2, _z_in_range(g, p1, p2)


def _near_tangent(g, n, beyond_frac=0.01):
    """Arcs through their apex (north) or nadir (south), z0 within r of the extremum."""
    lat = np.deg2rad(g.uniform(0.0, 89.9, n))
    lon = g.uniform(0.0, 2 * np.pi, n)
    A = np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], axis=1)
    east = np.stack([-np.sin(lon), np.cos(lon), np.zeros(n)], axis=1)  # horizontal at A
    a = g.uniform(1e-3, 0.1, n)
    b = g.uniform(1e-3, 0.1, n)
    p1 = np.cos(a)[:, None] * A - np.sin(a)[:, None] * east
    p2 = np.cos(b)[:, None] * A + np.sin(b)[:, None] * east
    south = g.random(n) < 0.5
    p1[south, 2] *= -1.0
    p2[south, 2] *= -1.0
    # height of the extremum of the great circle through the rounded endpoints, in
    # extended precision: |z|max = |n_xy| / |n|
    q1 = p1.astype(np.longdouble)
    q2 = p2.astype(np.longdouble)
    nn = np.cross(q1, q2)
    zext = np.sqrt(nn[:, 0] ** 2 + nn[:, 1] ** 2) / np.sqrt(np.sum(nn * nn, axis=1))
    r = (1.0 - g.random(n)) * 1e-12                      # U(0, 1e-12]
    beyond = g.random(n) < beyond_frac
    mag = np.where(beyond, zext + r.astype(np.longdouble), zext - r.astype(np.longdouble))
    z0 = np.where(south, -mag, mag).astype(np.float64)
    return p1, p2, z0


def _near_pole(g, n):
    c1 = g.uniform(0.0, 1e-6, n)
    c2 = g.uniform(0.0, 1e-6, n)
    l1 = g.uniform(0.0, 2 * np.pi, n)
    l2 = g.uniform(0.0, 2 * np.pi, n)
    sgn = np.where(g.random(n) < 0.5, 1.0, -1.0)
    p1 = np.stack([np.sin(c1) * np.cos(l1), np.sin(c1) * np.sin(l1), sgn * np.cos(c1)], axis=1)
    p2 = np.stack([np.sin(c2) * np.cos(l2), np.sin(c2) * np.sin(l2), sgn * np.cos(c2)], axis=1)
    return p1, p2, _z_in_range(g, p1, p2)


def ill_conditioned(n: int = 10_000_000, seed_tag: int = 1) -> Pairs:
    """Three equal parts (a) short, (b) near-tangent, (c) near-pole; ``part`` = 0, 1, 2."""
    sizes = [n // 3, n // 3, n - 2 * (n // 3)]
    parts = [_short_arcs(rng(seed_tag, 1), sizes[0]),
             _near_tangent(rng(seed_tag, 2), sizes[1]),
             _near_pole(rng(seed_tag, 3), sizes[2])]
    p1 = np.concatenate([p[0] for p in parts])
    p2 = np.concatenate([p[1] for p in parts])
    z0 = np.concatenate([p[2] for p in parts])
    part = np.concatenate([np.full(s, k, np.int8) for k, s in enumerate(sizes)])
    return Pairs(p1, p2, z0, part)


def stratified_sample(pairs: Pairs, per_part: int, seed: int = 7) -> np.ndarray:
    """Sorted indices: ``per_part`` uniform draws (without replacement) from each part."""
    g = np.random.Generator(np.random.PCG64(seed))
    idx = []
    for k in np.unique(pairs.part):
        members = np.flatnonzero(pairs.part == k)
        take = min(per_part, len(members))
        idx.append(g.choice(members, size=take, replace=False))
    return np.sort(np.concatenate(idx))


# ----------------------------------------------------------------- CSR workloads

class CsrMesh:
    """Arcs (SoA endpoints), sorted latitude table ``lat_z`` and CSR candidate lists.

    Pair k of arc i is (i, lat_idx[k]) for k in [lat_offsets[i], lat_offsets[i+1]).
    """

    def __init__(self, p1, p2, lat_z, lat_offsets, lat_idx):
        self.p1 = np.ascontiguousarray(p1, dtype=np.float64)
        self.p2 = np.ascontiguousarray(p2, dtype=np.float64)
        self.lat_z = np.ascontiguousarray(lat_z, dtype=np.float64)
        self.lat_offsets = np.ascontiguousarray(lat_offsets, dtype=np.int64)
        self.lat_idx = np.ascontiguousarray(lat_idx, dtype=np.int32)

    @property
    def n_arcs(self):
        return len(self.p1)

    @property
    def nnz(self):
        return int(self.lat_offsets[-1])

    def soa(self):
        return tuple(np.ascontiguousarray(a) for a in
                     (self.p1[:, 0], self.p1[:, 1], self.p1[:, 2],
                      self.p2[:, 0], self.p2[:, 1], self.p2[:, 2]))

    def expand(self) -> Pairs:
        """The candidate pairs as dense 1:1 pairs (for reference checks)."""
        arc = np.repeat(np.arange(self.n_arcs), np.diff(self.lat_offsets))
        return Pairs(self.p1[arc], self.p2[arc], self.lat_z[self.lat_idx])


def candidates(p1, p2, lat_z, pad=1e-12):
    """CSR lists of the latitudes of sorted ``lat_z`` inside each arc's (padded) z-range."""
    lo, hi = z_range(p1, p2)
    first = np.searchsorted(lat_z, lo - pad, side="left")
    last = np.searchsorted(lat_z, hi + pad, side="right")
    cnt = (last - first).astype(np.int64)
    offsets = np.zeros(len(p1) + 1, np.int64)
    np.cumsum(cnt, out=offsets[1:])
    nnz = int(offsets[-1])
    arc = np.repeat(np.arange(len(p1), dtype=np.int64), cnt)
    idx = (np.arange(nnz, dtype=np.int64) - offsets[arc] + first[arc]).astype(np.int32)
    return offsets, idx


def latitude_lines(count: int, first_deg: float, step_deg: float) -> np.ndarray:
    return np.sin(np.deg2rad(first_deg + step_deg * np.arange(count)))


def cubed_sphere_edges(ne: int):
    """Unique edges of the equiangular gnomonic cubed sphere, ne x ne cells per face.

    Nodes are identified by integer lattice coordinates on the cube surface, so edges
    shared by two faces appear once: 12 ne^2 edges for 6 ne^2 cells.
    """
    k = np.arange(ne + 1)
    t = np.tan(-np.pi / 4 + (np.pi / 2) * k / ne)            # gnomonic coordinate per index
    I, J = np.meshgrid(k, k, indexing="ij")
    keys, coords = [], []
    faces = [(0, ne), (0, 0), (1, ne), (1, 0), (2, ne), (2, 0)]  # (fixed axis, index)
    for axis, val in faces:
        lat = np.empty(I.shape + (3,), np.int64)
        free = [a for a in range(3) if a != axis]
        lat[..., axis] = val
        lat[..., free[0]] = I
        lat[..., free[1]] = J
        keys.append(lat.reshape(-1, 3))
    # unique lattice points in lexicographic order (a scalar key sorts the same way, since
    # every coordinate lies in [0, ne])
    allkeys = np.concatenate(keys)
    code_sorted = np.unique(allkeys[:, 0] * (ne + 1) ** 2 + allkeys[:, 1] * (ne + 1) + allkeys[:, 2])
    lattice = np.stack([code_sorted // (ne + 1) ** 2, (code_sorted // (ne + 1)) % (ne + 1),
                        code_sorted % (ne + 1)], axis=1)
    order = np.arange(len(code_sorted))
    xyz = t[lattice]
    pts = xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
    edges = []
    for axis, val in faces:
        free = [a for a in range(3) if a != axis]
        for da, db in ((1, 0), (0, 1)):
            ii, jj = np.meshgrid(np.arange(ne + 1 - da), np.arange(ne + 1 - db), indexing="ij")
            a = np.empty(ii.shape + (3,), np.int64)
            a[..., axis] = val
            a[..., free[0]] = ii
            a[..., free[1]] = jj
            b = a.copy()
            b[..., free[0]] += da
            b[..., free[1]] += db
            ca = (a[..., 0] * (ne + 1) ** 2 + a[..., 1] * (ne + 1) + a[..., 2]).ravel()
            cb = (b[..., 0] * (ne + 1) ** 2 + b[..., 1] * (ne + 1) + b[..., 2]).ravel()
            ia = order[np.searchsorted(code_sorted, ca)]
            ib = order[np.searchsorted(code_sorted, cb)]
            edges.append(np.stack([np.minimum(ia, ib), np.maximum(ia, ib)], axis=1))
    e = np.concatenate(edges)
    npts = np.int64(len(pts))
    ekey = np.unique(e[:, 0] * npts + e[:, 1])  # lexicographic (low node, high node) order
    return pts[ekey // npts], pts[ekey % npts]


def cubed_sphere(ne: int = 1024, n_lat: int = 1800, first_deg: float = -89.95,
                 step_deg: float = 0.1) -> CsrMesh:
    """Regridding-shaped CSR workload: cubed-sphere edges x a lat-lon grid's latitudes."""
    p1, p2 = cubed_sphere_edges(ne)
    lat_z = latitude_lines(n_lat, first_deg, step_deg)
    off, idx = candidates(p1, p2, lat_z)
    return CsrMesh(p1, p2, lat_z, off, idx)


def random_mesh(g: np.random.Generator, n_arcs: int, n_lat: int, d_hi: float = 0.05) -> CsrMesh:
    """Uneven synthetic mesh: arcs as ``uniform_arcs`` with d <= d_hi, n_lat uniform lines."""
    p1 = random_unit(g, n_arcs)
    d = g.uniform(1e-3, d_hi, n_arcs)
    p2 = arc_from(p1, d, g.uniform(0.0, 2 * np.pi, n_arcs))
    step = 180.0 / n_lat
    lat_z = latitude_lines(n_lat, -90.0 + step / 2, step)
    off, idx = candidates(p1, p2, lat_z)
    return CsrMesh(p1, p2, lat_z, off, idx)


def mesh_batch(n_meshes: int = 64, arcs_lo: float = 1e3, arcs_hi: float = 1e7,
               lat_lo: int = 10, lat_hi: int = 3600, seed_tag: int = 3):
    """Many independent meshes of log-uniform size and uniform latitude count."""
    g = rng(seed_tag)
    sizes = np.floor(np.exp(g.uniform(np.log(arcs_lo), np.log(arcs_hi), n_meshes))).astype(int)
    lats = g.integers(lat_lo, lat_hi + 1, n_meshes)
    return [random_mesh(rng(seed_tag, 1 + m), int(s), int(L)) for m, (s, L) in enumerate(zip(sizes, lats))]


def request_stream(rate_hz: float = 2000.0, duration_s: float = 10.0, arcs_lo=1e3, arcs_hi=1e6,
                   lat_lo=1, lat_hi=1000, seed_tag: int = 4, max_requests=None):
    """Poisson arrivals: (arrival_times, [(n_arcs, n_lat, seed), ...]); meshes built lazily."""
    g = rng(seed_tag)
    gaps = g.exponential(1.0 / rate_hz, int(rate_hz * duration_s * 1.5) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    if max_requests is not None:
        t = t[:max_requests]
    n = len(t)
    arcs = np.floor(np.exp(g.uniform(np.log(arcs_lo), np.log(arcs_hi), n))).astype(int)
    lats = np.floor(np.exp(g.uniform(np.log(lat_lo), np.log(lat_hi + 1), n))).astype(int)
    lats = np.clip(lats, lat_lo, lat_hi)
    return t, [(int(a), int(L), 1000 + i) for i, (a, L) in enumerate(zip(arcs, lats))]


# ----------------------------------------------------------------- arc x arc workloads

class ArcPairs:
    """Dense arc x arc pairs: A = a1 -> a2 and B = b1 -> b2, (n, 3) each; ``part`` labels."""

    def __init__(self, a1, a2, b1, b2, part=None):
        self.a1, self.a2, self.b1, self.b2 = (np.ascontiguousarray(v, dtype=np.float64)
                                              for v in (a1, a2, b1, b2))
        self.part = np.zeros(len(self.a1), np.int8) if part is None else np.asarray(part, np.int8)

    def __len__(self):
        return len(self.a1)

    def soa_a(self):
        return tuple(np.ascontiguousarray(v[:, c]) for v in (self.a1, self.a2) for c in range(3))

    def soa_b(self):
        return tuple(np.ascontiguousarray(v[:, c]) for v in (self.b1, self.b2) for c in range(3))

    def take(self, idx):
        return ArcPairs(self.a1[idx], self.a2[idx], self.b1[idx], self.b2[idx], self.part[idx])


def _unit(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _through(g, c, half_lo, half_hi):
    """An arc through c (unit, (n, 3)) along a uniform bearing, each half U[half_lo, half_hi]."""
    n = len(c)
    br = g.uniform(0.0, 2 * np.pi, n)
    b1 = arc_from(c, g.uniform(half_lo, half_hi, n), br)
    b2 = arc_from(c, g.uniform(half_lo, half_hi, n), br + np.pi)
    return b1, b2


def arc_pairs(n: int = 10_000_000, seed_tag: int = 5) -> ArcPairs:
    g = rng(seed_tag)
    sizes = [n // 4 + (1 if k < n % 4 else 0) for k in range(4)]
    out = []
    # (0) crossing-shaped: A of length U[0.05, 1], B through a point near A's midpoint
    m = sizes[0]
    a1 = random_unit(g, m)
    a2 = arc_from(a1, g.uniform(0.05, 1.0, m), g.uniform(0.0, 2 * np.pi, m))
    c = arc_from(_unit(a1 + a2), g.uniform(0.0, 0.5, m), g.uniform(0.0, 2 * np.pi, m))
    out.append((a1, a2, *_through(g, _unit(c), 0.05, 0.5)))
    # (1) short: A log-uniform in [1e-9, 1e-6] rad, B of half-length 1e-7 near its midpoint
    m = sizes[1]
    a1 = random_unit(g, m)
    a2 = arc_from(a1, np.exp(g.uniform(np.log(1e-9), np.log(1e-6), m)),
                  g.uniform(0.0, 2 * np.pi, m))
    c = arc_from(_unit(a1 + a2), g.uniform(0.0, 1e-7, m), g.uniform(0.0, 2 * np.pi, m))
    out.append((a1, a2, *_through(g, _unit(c), 1e-8, 1e-7)))
    # (2) nearly parallel: B's endpoints are A's tilted by 1e-9 .. 1e-3
    m = sizes[2]
    a1 = random_unit(g, m)
    a2 = arc_from(a1, np.full(m, 0.05), g.uniform(0.0, 2 * np.pi, m))
    tilt = np.exp(g.uniform(np.log(1e-9), np.log(1e-3), (m, 1)))
    out.append((a1, a2, a1 + tilt * random_unit(g, m), a2 + tilt * random_unit(g, m)))
    # (3) mesh-like: B starts exactly at A's end (a shared vertex)
    m = sizes[3]
    a1 = random_unit(g, m)
    a2 = arc_from(a1, g.uniform(1e-3, 0.05, m), g.uniform(0.0, 2 * np.pi, m))
    b2 = arc_from(a2, g.uniform(1e-3, 0.05, m), g.uniform(0.0, 2 * np.pi, m))
    out.append((a1, a2, a2.copy(), b2))
    part = np.concatenate([np.full(sz, k, np.int8) for k, sz in enumerate(sizes)])
    return ArcPairs(*(np.concatenate([o[i] for o in out]) for i in range(4)), part=part)


# ----------------------------------------------------------- drawn on the device

def device_arcs(torch, gen, n: int, d_lo: float = 1e-3, d_hi: float = 0.05):
    """As ``arc_from`` on uniform points, drawn on the current CUDA device: p1 uniform on the
    sphere, p2 at distance d ~ U[d_lo, d_hi] along a uniform bearing.  Returns the (x, y, z)
    components of p1 and p2 as contiguous float64 device tensors."""
    import math
    f64 = dict(dtype=torch.float64, device="cuda")
    p = torch.randn(n, 3, generator=gen, **f64)
    p = p / p.norm(dim=1, keepdim=True)
    d = d_lo + (d_hi - d_lo) * torch.rand(n, generator=gen, **f64)
    b = 2 * math.pi * torch.rand(n, generator=gen, **f64)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    r = torch.hypot(x, y)
    east = torch.stack([-y / r, x / r, torch.zeros_like(r)], dim=1)
    north = torch.stack([-z * x / r, -z * y / r, r], dim=1)
    t = torch.cos(b)[:, None] * north + torch.sin(b)[:, None] * east
    q = torch.cos(d)[:, None] * p + torch.sin(d)[:, None] * t
    return [p[:, k].contiguous() for k in range(3)], [q[:, k].contiguous() for k in range(3)]


def device_mesh_sizes(n_meshes: int = 64, arcs_lo: float = 1e3, arcs_hi: float = 1e7,
                      lat_lo: int = 10, lat_hi: int = 3600, seed_tag: int = 3):
    """Arcs (log-uniform) and latitude counts (uniform) of the uneven mesh batch."""
    g = rng(seed_tag)
    sizes = np.floor(np.exp(g.uniform(np.log(arcs_lo), np.log(arcs_hi), n_meshes))).astype(int)
    lats = g.integers(lat_lo, lat_hi + 1, n_meshes)
    return sizes, lats


def device_mesh_arcs(torch, n_meshes: int = 64, seed_tag: int = 3):
    """The uneven batch's arcs and latitude tables drawn on the device, one dict per mesh
    with p1, p2 (component tensors) and lat_z (L uniformly spaced latitude lines at
    -90 + (k + 1/2) 180 / L degrees).  Candidate lists are left to the caller."""
    sizes, lats = device_mesh_sizes(n_meshes, seed_tag=seed_tag)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(SEED_BASE + seed_tag)
    out = []
    for n, L in zip(sizes, lats):
        p1, p2 = device_arcs(torch, gen, int(n))
        step = 180.0 / int(L)
        lat_z = torch.from_numpy(latitude_lines(int(L), -90.0 + step / 2, step)).cuda()
        out.append(dict(p1=tuple(p1), p2=tuple(p2), lat_z=lat_z))
    return out
