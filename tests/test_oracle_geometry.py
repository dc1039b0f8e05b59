"""Pins for the exact oracle (oracle.geometry) from outside itself.

Each check below is fixed by the geometry, not by re-typing Eq. (2.2):
closed forms (equator, meridians, poles), invariants of the true intersection, an
independent angle-parametrised derivation (oracle.angle, mpmath), a brute-force
containment test by orientation, and metamorphic symmetries.
"""

import itertools
import math
from decimal import Decimal

import mpmath as mp
import numpy as np
import pytest

from oracle import geometry as G
from oracle import angle
from paper_2510_09892_amd import inputs

U = 2.0 ** -53
TINY = Decimal(10) ** -80


def dec(v):
    return Decimal(v)


def _hits(x1, x2, z0):
    c, pts = G.intersect(x1, x2, z0)
    return c, pts


# ----------------------------------------------------------------- closed forms

def test_equator_crossing_closed_form():
    """z0 = 0: the crossing lies on the line n x e_z, i.e. +-(n_y, -n_x)/|n_xy|."""
    g = np.random.Generator(np.random.PCG64(1))
    for _ in range(200):
        a = g.standard_normal(3)
        b = g.standard_normal(3)
        a[2] = -abs(a[2])
        b[2] = abs(b[2])          # the arc goes from the south to the north: one crossing
        x1, x2 = tuple(map(float, a)), tuple(map(float, b))
        c, pts = _hits(x1, x2, 0.0)
        assert c.count == 1 and c.roots == (G.PLUS,) and c.flags == G.EXISTS
        with mp.workprec(400):
            n = [mp.mpf(x1[1]) * x2[2] - mp.mpf(x1[2]) * x2[1],
                 mp.mpf(x1[2]) * x2[0] - mp.mpf(x1[0]) * x2[2],
                 mp.mpf(x1[0]) * x2[1] - mp.mpf(x1[1]) * x2[0]]
            r = mp.sqrt(n[0] ** 2 + n[1] ** 2)
            cand = [(-n[1] / r, n[0] / r), (n[1] / r, -n[0] / r)]
            # the ascending crossing: z increases along n x P; pick the candidate with
            # (n x P)_z > 0
            asc = [p for p in cand if n[0] * p[1] - n[1] * p[0] > 0][0]
            assert abs(dec(str(asc[0])) - pts[0][0]) < Decimal("1e-90")
            assert abs(dec(str(asc[1])) - pts[0][1]) < Decimal("1e-90")


@pytest.mark.parametrize("direction", [(1.0, 0.0), (3.0, 4.0), (1.0, 1.0), (-5.0, 12.0)])
def test_meridian_arcs(direction):
    """Arcs along a meridian of direction (a, b): P = sqrt(1 - z0^2) (a, b)/|(a, b)|."""
    a, b = direction
    g = np.random.Generator(np.random.PCG64(2))
    for _ in range(50):
        h1, h2 = sorted(g.uniform(-3, 3, 2))
        k1, k2 = np.round(g.uniform(0.25, 2.0, 2) * 1024) / 1024   # k*a, k*b exact
        x1 = (k1 * a, k1 * b, float(h1))
        x2 = (k2 * a, k2 * b, float(h2))
        z1 = h1 / math.sqrt((k1 * a) ** 2 + (k1 * b) ** 2 + h1 ** 2)
        z2 = h2 / math.sqrt((k2 * a) ** 2 + (k2 * b) ** 2 + h2 ** 2)
        z0 = float(g.uniform(min(z1, z2), max(z1, z2)))
        c, pts = _hits(x1, x2, z0)
        assert c.count == 1 and c.flags == G.EXISTS
        with mp.workprec(400):
            r = mp.sqrt(1 - mp.mpf(z0) ** 2) / mp.sqrt(mp.mpf(a) ** 2 + mp.mpf(b) ** 2)
            assert abs(dec(str(r * a)) - pts[0][0]) < Decimal("1e-90")
            assert abs(dec(str(r * b)) - pts[0][1]) < Decimal("1e-90")


def test_pole_tangency():
    """A meridian arc over the pole touches z0 = 1 once, at (0, 0): s^2 = 0 exactly."""
    x1 = (1.0, 0.0, 3.0)
    x2 = (-1.0, 0.0, 2.0)
    c, pts = _hits(x1, x2, 1.0)
    assert c.count == 1 and c.flags == G.EXISTS | G.TANGENT
    assert pts[0] == (0, 0) or (abs(pts[0][0]) < TINY and abs(pts[0][1]) < TINY)
    c, _ = _hits(x1, x2, -1.0)      # south pole is not on this arc
    assert c.count == 0 and c.flags == G.EXISTS | G.TANGENT
    c, _ = _hits(x1, x2, 1.0 + 2 ** -52)
    assert c.count == 0 and c.flags == 0


def test_endpoint_ties_inclusive():
    """Closed arc: a latitude through an endpoint (exactly representable height) counts."""
    # endpoint on the equator, z0 = 0
    c, pts = _hits((1.0, 0.0, 0.0), (0.0, 1.0, 1.0), 0.0)
    assert c.count == 1
    assert abs(pts[0][0] - 1) < TINY and abs(pts[0][1]) < TINY
    # endpoint at the pole, z0 = 1: the other side of the arc goes down
    c, pts = _hits((0.0, 0.0, 2.0), (1.0, 0.0, 0.0), 1.0)
    assert c.count == 1 and c.flags & G.TANGENT
    # latitude just beyond the endpoint height: no hit
    c, _ = _hits((1.0, 0.0, 0.0), (0.0, 1.0, 1.0), -2.0 ** -60)
    assert c.count == 0


def test_degenerate_flags():
    assert G.classify((1.0, 2.0, 3.0), (2.0, 4.0, 6.0), 0.1) == (0, (), G.DEGEN_N)
    assert G.classify((1.0, 2.0, 3.0), (-1.0, -2.0, -3.0), 0.1) == (0, (), G.DEGEN_N)
    assert G.classify((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), 0.0) == (0, (), G.DEGEN_N)
    assert G.classify((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.0) == (0, (), G.HORIZ)
    assert G.classify((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.5) == (0, (), G.HORIZ)
    assert G.classify((math.nan, 0.0, 0.0), (0.0, 1.0, 0.0), 0.5) == (0, (), G.NONFINITE)
    assert G.classify((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), math.inf) == (0, (), G.NONFINITE)
    # |z0| > 1 never meets the sphere
    assert G.classify((1.0, 0.0, -1.0), (0.0, 1.0, 1.0), 1.5).count == 0


# ----------------------------------------------------------------- invariants

def _samples():
    a = inputs.uniform_arcs(300, seed_tag=11)
    b = inputs.ill_conditioned(300, seed_tag=12)
    for P in (a, b):
        for i in range(len(P)):
            yield tuple(map(float, P.p1[i])), tuple(map(float, P.p2[i])), float(P.z0[i])


def test_invariants_on_workloads():
    """|P|^2 + z0^2 = 1, n . P = 0, (n x P)_z = +-s matching the root label."""
    checked = 0
    for x1, x2, z0 in _samples():
        c, pts = _hits(x1, x2, z0)
        t = G.exact_terms(x1, x2, z0)
        K = t["K"]
        with mp.workprec(500):
            n = [mp.mpf(t["Nx"]), mp.mpf(t["Ny"]), mp.mpf(t["Nz"])]
            s = mp.sqrt(mp.mpf(t["s2"])) if t["s2"] >= 0 else None
            for r, (px, py) in zip(c.roots, pts):
                X, Y, Z = mp.mpf(str(px)), mp.mpf(str(py)), mp.mpf(z0)
                assert abs(X * X + Y * Y + Z * Z - 1) < mp.mpf(10) ** -90
                nn = mp.sqrt(sum(v * v for v in n))
                assert abs((n[0] * X + n[1] * Y + n[2] * Z) / nn) < mp.mpf(10) ** -90
                cz = (n[0] * Y - n[1] * X) / mp.mpf(2) ** (2 * K)    # (n x P)_z, true scale
                sig = 1 if r == G.PLUS else -1
                strue = s / mp.mpf(2) ** (3 * K)
                assert abs(cz - sig * strue) < mp.mpf(10) ** -90 * (1 + nn / mp.mpf(2) ** (2 * K))
                checked += 1
    assert checked > 400


# ----------------------------------------------------------------- independent derivation

def _cross_check(x1, x2, z0):
    c, pts = _hits(x1, x2, z0)
    alt, margin = angle.intersect(x1, x2, z0)
    if margin < mp.mpf(10) ** -60:
        return False
    assert c.count == len(alt), (x1, x2, z0, c, alt)
    assert tuple(r for r, *_ in alt) == c.roots
    for (r, th, ax, ay), (px, py) in zip(alt, pts):
        assert abs(dec(mp.nstr(ax, 90)) - px) < Decimal("1e-80")
        assert abs(dec(mp.nstr(ay, 90)) - py) < Decimal("1e-80")
    return True


def test_angle_derivation_agrees_on_workloads():
    n = sum(_cross_check(*s) for s in _samples())
    assert n > 500


def test_angle_derivation_agrees_random_latitudes():
    """Random arcs of every length up to pi and latitudes across [-1, 1]: 0, 1, 2 hits."""
    g = np.random.Generator(np.random.PCG64(3))
    seen = set()
    for _ in range(600):
        x1 = tuple(map(float, g.standard_normal(3)))
        x2 = tuple(map(float, g.standard_normal(3)))
        z0 = float(g.uniform(-1, 1))
        if _cross_check(x1, x2, z0):
            seen.add(G.classify(x1, x2, z0).count)
    assert seen == {0, 1, 2}


# ----------------------------------------------------------------- brute force

def _orientation_hits(x1, x2, z0):
    """Brute force: all circle points at height z0 (angle form), kept if on the closed
    minor arc by orientation: (x1 x P) . n >= 0 and (P x x2) . n >= 0 (with tolerance)."""
    with mp.workprec(300):
        a = [mp.mpf(v) for v in x1]
        b = [mp.mpf(v) for v in x2]
        n = [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]
        nn = mp.sqrt(sum(v * v for v in n))
        if nn == 0:
            return []
        nh = [v / nn for v in n]
        # orthonormal basis of the plane: e1 = n x e_z direction (horizontal), e2 = nh x e1
        h = mp.sqrt(nh[0] ** 2 + nh[1] ** 2)
        if h == 0:
            return []
        e1 = [nh[1] / h, -nh[0] / h, mp.mpf(0)]
        e2 = [nh[1] * e1[2] - nh[2] * e1[1], nh[2] * e1[0] - nh[0] * e1[2],
              nh[0] * e1[1] - nh[1] * e1[0]]
        # z(t) = cos t e1_z + sin t e2_z = sin t e2_z
        if abs(mp.mpf(z0)) > abs(e2[2]):
            return []
        t0 = mp.asin(mp.mpf(z0) / e2[2])
        out = []
        for t in (t0, mp.pi - t0):
            P = [mp.cos(t) * e1[k] + mp.sin(t) * e2[k] for k in range(3)]
            o1 = sum((a[(k + 1) % 3] * P[(k + 2) % 3] - a[(k + 2) % 3] * P[(k + 1) % 3]) * n[k]
                     for k in range(3))
            o2 = sum((P[(k + 1) % 3] * b[(k + 2) % 3] - P[(k + 2) % 3] * b[(k + 1) % 3]) * n[k]
                     for k in range(3))
            eps = mp.mpf(10) ** -70
            if o1 >= -eps and o2 >= -eps:
                if not any(abs(P[0] - q[0]) + abs(P[1] - q[1]) < mp.mpf(10) ** -60 for q in out):
                    out.append(P)
        return out


def test_exhaustive_small_integer_arcs():
    """Every arc between nonzero vectors of {-1,0,1}^3 and z0 in a grid including the
    tie heights 0 and +-1: hit sets agree with the orientation brute force exactly."""
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0), repeat=3) if any(v)]
    for x1 in verts:
        for x2 in verts:
            for z0 in (-1.0, -0.5, 0.0, 0.375, 1.0):
                c, pts = _hits(x1, x2, z0)
                ref = _orientation_hits(x1, x2, z0)
                if c.flags & (G.DEGEN_N | G.HORIZ):
                    continue
                assert c.count == len(ref), (x1, x2, z0, c, len(ref))
                for px, py in pts:
                    assert any(abs(dec(mp.nstr(q[0], 80)) - px) < Decimal("1e-60") and
                               abs(dec(mp.nstr(q[1], 80)) - py) < Decimal("1e-60") for q in ref)


def test_dense_sampling_hit_counts():
    """Sign changes of z(theta) - z0 over a dense sampling of the arc, for arcs and
    latitudes where no sample is within the grid's resolution of a tie."""
    g = np.random.Generator(np.random.PCG64(5))
    agree = 0
    for _ in range(300):
        x1 = tuple(map(float, g.standard_normal(3)))
        x2 = tuple(map(float, g.standard_normal(3)))
        z0 = float(g.uniform(-1, 1))
        u = np.array(x1) / np.linalg.norm(x1)
        w = np.array(x2) / np.linalg.norm(x2)
        th12 = math.atan2(np.linalg.norm(np.cross(u, w)), float(u @ w))
        v = w - (u @ w) * u
        v /= np.linalg.norm(v)
        ts = np.linspace(0.0, th12, 20001)
        z = np.cos(ts) * u[2] + np.sin(ts) * v[2] - z0
        if np.min(np.abs(z)) < 1e-6:
            continue
        changes = int(np.sum(np.signbit(z[1:]) != np.signbit(z[:-1])))
        assert G.classify(x1, x2, z0).count == changes
        agree += 1
    assert agree > 250


# ----------------------------------------------------------------- symmetries

def _metamorphic(x1, x2, z0):
    c, pts = _hits(x1, x2, z0)
    # swapping the endpoints reverses the travel: same points, reversed order, labels swap
    c2, pts2 = _hits(x2, x1, z0)
    assert c2.count == c.count and c2.flags == c.flags
    assert c2.roots == tuple(1 - r for r in reversed(c.roots))
    assert pts2 == list(reversed(pts))
    # mirror z -> -z with z0 -> -z0: same (x, y) points, same order, labels swap
    m1, m2 = (x1[0], x1[1], -x1[2]), (x2[0], x2[1], -x2[2])
    c3, pts3 = _hits(m1, m2, -z0)
    assert c3.count == c.count and c3.roots == tuple(1 - r for r in c.roots)
    assert all(abs(a[0] - b[0]) < TINY and abs(a[1] - b[1]) < TINY for a, b in zip(pts, pts3))
    # rotate by 90 degrees about z: (x, y) -> (-y, x)
    r1, r2 = (-x1[1], x1[0], x1[2]), (-x2[1], x2[0], x2[2])
    c4, pts4 = _hits(r1, r2, z0)
    assert c4 == c
    assert all(abs(-a[1] - b[0]) < TINY and abs(a[0] - b[1]) < TINY for a, b in zip(pts, pts4))
    # scale an endpoint by a power of two: identical result
    c5, pts5 = _hits(tuple(8.0 * v for v in x1), x2, z0)
    assert c5 == c
    assert all(abs(a[0] - b[0]) < TINY and abs(a[1] - b[1]) < TINY for a, b in zip(pts, pts5))


def test_metamorphic_on_workloads():
    for s in _samples():
        _metamorphic(*s)
