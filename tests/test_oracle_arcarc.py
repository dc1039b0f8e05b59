"""Pins of the arc x arc oracle (oracle/arcarc.py).

* closed forms: an equator arc against meridian arcs, shared endpoints, a T-junction, arcs on
  one great circle, degenerate arcs;
* an independent derivation: a point q of both great circles lies on a minor arc iff the
  angles a1->q and q->a2 add up to a1->a2 (mpmath at 300 bits), checked for +-p on random,
  short and nearly parallel arcs and exhaustively on small integer arcs;
* invariants of the exact point (unit length, on both planes);
* the binary64 EFT replica within 4 * 2^-53 of the exact point.
"""

import itertools
import math

import mpmath
import numpy as np
import pytest

from oracle import arcarc as AA
from paper_2510_09892_amd import inputs

U = 2.0 ** -53


def test_equator_against_meridian():
    a1, a2 = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    b1, b2 = (1.0, 1.0, -1.0), (1.0, 1.0, 1.0)
    count, flags, p = AA.intersect(a1, a2, b1, b2)
    assert count == 1 and flags == AA.HIT
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 100
        h = Decimal(2).sqrt() / 2
        assert abs(p[0] - h) < Decimal(10) ** -90 and abs(p[1] - h) < Decimal(10) ** -90
    assert p[2] == 0
    # the same meridian on the far side of the globe misses
    assert AA.classify(a1, a2, (-1.0, -1.0, -1.0), (-1.0, -1.0, 1.0))[0] == 0
    # north of the equator only: no crossing
    assert AA.classify(a1, a2, (1.0, 1.0, 0.5), (1.0, 1.0, 1.0))[0] == 0


def test_touching_and_shared_endpoints_count():
    a1, a2 = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    c, f, p = AA.intersect(a1, a2, (1.0, 1.0, 0.0), (1.0, 1.0, 1.0))  # T-junction
    assert c == 1 and abs(float(p[2])) < 1e-40
    c, f, p = AA.intersect(a1, a2, (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))  # shared vertex
    assert c == 1 and [float(v) for v in p] == [0.0, 1.0, 0.0]
    c, f, p = AA.intersect(a1, a2, (0.0, 2.0, 0.0), (0.0, 0.0, 5.0))  # scaled endpoints
    assert c == 1 and [float(v) for v in p] == [0.0, 1.0, 0.0]


def test_degenerate_and_coplanar():
    a1, a2 = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    assert AA.classify(a1, a1, a1, a2) == (0, 0, AA.DEGEN)
    assert AA.classify(a1, (-2.0, 0.0, 0.0), a1, a2) == (0, 0, AA.DEGEN)
    assert AA.classify(a1, a2, (1.0, 1.0, 0.0), (-1.0, 1.0, 0.0)) == (0, 0, AA.COPLANAR)
    assert AA.classify(a1, a2, (0.0, 0.0, 1.0), (math.nan, 0.0, 1.0)) == (0, 0, AA.NONFINITE)


def _angle(u, v):
    cu = mpmath.matrix(u)
    cv = mpmath.matrix(v)
    cr = mpmath.matrix([cu[1] * cv[2] - cu[2] * cv[1], cu[2] * cv[0] - cu[0] * cv[2],
                        cu[0] * cv[1] - cu[1] * cv[0]])
    return mpmath.atan2(mpmath.norm(cr), cu[0] * cv[0] + cu[1] * cv[1] + cu[2] * cv[2])


def _on_arc(q, a1, a2, tol):
    return abs(_angle(a1, q) + _angle(q, a2) - _angle(a1, a2)) < tol


def _angle_count(a1, a2, b1, b2):
    """Independent count: which of +-p lies on both arcs, by angle sums (mpmath)."""
    mpmath.mp.prec = 300
    A1, A2, B1, B2 = ([mpmath.mpf(v) for v in w] for w in (a1, a2, b1, b2))
    cr = lambda u, v: [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]
    X = cr(cr(A1, A2), cr(B1, B2))
    nrm = mpmath.sqrt(sum(c * c for c in X))
    if nrm == 0:
        return None
    tol = mpmath.mpf(2) ** -200
    hits = []
    for sg in (1, -1):
        q = [sg * c / nrm for c in X]
        if _on_arc(q, A1, A2, tol) and _on_arc(q, B1, B2, tol):
            hits.append(sg)
    return hits


def _random_pairs(g, n, kind):
    out = []
    for _ in range(n):
        if kind == "short":
            P = inputs.uniform_arcs(1, seed_tag=int(g.integers(1 << 30)), d_lo=1e-9, d_hi=1e-6)
            mid = (P.p1[0] + P.p2[0]) / 2
            q1 = inputs.arc_from(mid[None, :], np.array([1e-7]), np.array([g.uniform(0, 6.3)]))[0]
            out.append((tuple(P.p1[0]), tuple(P.p2[0]), tuple(q1), tuple(2 * mid - q1)))
        elif kind == "parallel":
            a1 = inputs.random_unit(g, 1)[0]
            a2 = inputs.arc_from(a1[None, :], np.array([0.05]), np.array([g.uniform(0, 6.3)]))[0]
            tilt = 10.0 ** g.uniform(-9, -3)
            b1 = a1 + tilt * inputs.random_unit(g, 1)[0]
            b2 = a2 + tilt * inputs.random_unit(g, 1)[0]
            out.append((tuple(a1), tuple(a2), tuple(b1), tuple(b2)))
        else:  # B through a point near A's midpoint: about half of the pairs cross
            P = inputs.uniform_arcs(1, seed_tag=int(g.integers(1 << 30)), d_lo=0.05, d_hi=1.0)
            mid = (P.p1[0] + P.p2[0]) / 2
            c = inputs.arc_from(mid[None, :], np.array([g.uniform(0, 0.5)]),
                                np.array([g.uniform(0, 6.3)]))[0]
            br = g.uniform(0, 6.3)
            b1 = inputs.arc_from(c[None, :], np.array([g.uniform(0.05, 0.5)]), np.array([br]))[0]
            b2 = inputs.arc_from(c[None, :], np.array([g.uniform(0.05, 0.5)]), np.array([br + math.pi]))[0]
            out.append((tuple(P.p1[0]), tuple(P.p2[0]), tuple(b1), tuple(b2)))
    return out


@pytest.mark.parametrize("kind", ["uniform", "short", "parallel"])
def test_angle_derivation_agrees(kind):
    g = np.random.Generator(np.random.PCG64(80 + len(kind)))
    pairs = _random_pairs(g, 60 if kind != "uniform" else 120, kind)
    hits = 0
    for a1, a2, b1, b2 in pairs:
        c, sg, fl = AA.classify(a1, a2, b1, b2)
        ref = _angle_count(a1, a2, b1, b2)
        assert ref is not None
        assert c == len(ref) and (c == 0 or ref == [sg]), (a1, a2, b1, b2)
        hits += c
    assert hits > 5


def test_exhaustive_small_integer_arcs():
    verts = [v for v in itertools.product((-1.0, 0.0, 1.0, 2.0), repeat=3) if any(v)]
    g = np.random.Generator(np.random.PCG64(90))
    checked = 0
    for _ in range(1500):
        a1, a2, b1, b2 = (verts[int(i)] for i in g.integers(0, len(verts), 4))
        c, sg, fl = AA.classify(a1, a2, b1, b2)
        if fl & (AA.DEGEN | AA.COPLANAR):
            continue
        na = np.cross(a1, a2)
        if np.dot(a1, a2) < 0 and not np.any(na):  # antipodal pairs are degenerate too
            continue
        ref = _angle_count(a1, a2, b1, b2)
        if ref is None:
            continue
        assert c == len(ref) and (c == 0 or ref == [sg]), (a1, a2, b1, b2)
        checked += 1
    assert checked > 800


def test_point_invariants_and_eft_replica_within_4u():
    g = np.random.Generator(np.random.PCG64(91))
    worst_eft = worst_naive = 0.0
    n_hits = 0
    for kind in ("uniform", "short", "parallel"):
        for a1, a2, b1, b2 in _random_pairs(g, 80, kind):
            for sg in (1, -1):
                p = AA.point(a1, a2, b1, b2, sg)
                from decimal import Decimal
                assert abs(sum(c * c for c in p) - 1) < Decimal(10) ** -90
                na = np.cross(a1, a2)
                nb = np.cross(b1, b2)
                # on both planes (exact normals in rationals are not needed at this tolerance)
                assert abs(sum(Decimal(float(x)) * c for x, c in zip(na, p))) < Decimal(10) ** -14
                q = AA.eft_point(a1, a2, b1, b2, sg)
                e = max(abs(Decimal(v) - c) for v, c in zip(q, p)) / Decimal(U)
                worst_eft = max(worst_eft, float(e))
                qn = AA.naive_point(a1, a2, b1, b2, sg)
                en = max(abs(Decimal(v) - c) for v, c in zip(qn, p)) / Decimal(U)
                worst_naive = max(worst_naive, float(en))
                n_hits += 1
    assert worst_eft <= 4.0, worst_eft
    assert worst_naive > 1e3  # the naive cross products lose digits on short/parallel arcs
