"""Intersection of two great-circle arcs (oracle; test infrastructure only).

Next application the paper names for its accurate cross product (Sec. 1, and Sec. 9): two
minor arcs A = a1 -> a2 and B = b1 -> b2 meet where their great circles do, at the two
antipodal points +-p with p = (a1 x a2) x (b1 x b2) / |...| ("three cross products and a
normalisation"), provided the point lies on both closed arcs.

Containment reduces to orientations.  With n_A = a1 x a2 and n_B = b1 x b2, a point q = +-p
on both great circles lies on the minor arc A iff (a1 x q).n_A >= 0 and (q x a2).n_A >= 0;
by the Binet-Cauchy identity and n_A.a_i = 0 these are
    (a1 x p).n_A = |n_A|^2 (n_B . a1),     (p x a2).n_A = -|n_A|^2 (n_B . a2),
and likewise on B with the roles swapped:
    (b1 x p).n_B = -|n_B|^2 (n_A . b1),    (p x b2).n_B = |n_B|^2 (n_A . b2).
So with the four orientation signs
    sa1 = sign(n_B . a1), sa2 = sign(n_B . a2), sb1 = sign(n_A . b1), sb2 = sign(n_A . b2)
the point +p is on both arcs iff sa1 >= 0 >= sa2 and sb2 >= 0 >= sb1, and -p iff all four
inequalities are reversed.  Both can hold only when sa1 = sa2 = 0, i.e. a1 and a2 lie in
B's plane: the arcs share their great circle (COPLANAR: no isolated point is reported).
Each sign is a 3x3 determinant of input vectors, decided exactly here in integers.

Points: p in 100-digit decimal from the exact integer vector (n_A x n_B).  Alongside, the
binary64 replicas of the library's two evaluations, step by step:
* naive: every cross product, the norm and the division in plain binary64;
* EFT: n_A and n_B by AccuDOP (Alg. 4, read as in the latitude path) with the TwoSum
  renormalisation; each component X_c = nA_i nB_j - nA_j nB_i of n_A x n_B by AccuDOP on
  the leading parts, with the four first-order products of the trailing parts (one
  multiplication and three FMAs) added to its error term before the final sum (the
  second-order products are below u^2 of the result and are dropped); |X|^2 by
  SumOfSquares (Alg. 5), one binary64 square root and three divisions.
"""

from __future__ import annotations

import math
from decimal import Decimal, localcontext

from . import eft as E
from .geometry import scaled_ints

HIT = 1        # the arcs meet in one point
DEGEN = 4      # an arc with coincident or antipodal endpoints (zero normal)
COPLANAR = 8   # the arcs lie on one great circle
NONFINITE = 16

DIGITS = 100


def _sign(v):
    return (v > 0) - (v < 0)


def _cross(u, v):
    return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])


def _dot(u, v):
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]


def classify(a1, a2, b1, b2):
    """(count, sign, flags): count 0/1; sign +1 or -1 says which of +-p is the point."""
    vals = (*a1, *a2, *b1, *b2)
    if not all(math.isfinite(v) for v in vals):
        return 0, 0, NONFINITE
    ints, _ = scaled_ints(vals)
    A1, A2, B1, B2 = ints[0:3], ints[3:6], ints[6:9], ints[9:12]
    NA, NB = _cross(A1, A2), _cross(B1, B2)
    if NA == (0, 0, 0) or NB == (0, 0, 0):
        return 0, 0, DEGEN
    sa1, sa2 = _sign(_dot(NB, A1)), _sign(_dot(NB, A2))
    sb1, sb2 = _sign(_dot(NA, B1)), _sign(_dot(NA, B2))
    if sa1 == 0 and sa2 == 0:
        return 0, 0, COPLANAR
    if sa1 >= 0 >= sa2 and sb2 >= 0 >= sb1:
        return 1, 1, HIT
    if sa1 <= 0 <= sa2 and sb2 <= 0 <= sb1:
        return 1, -1, HIT
    return 0, 0, 0


def point(a1, a2, b1, b2, sign):
    """sign * (n_A x n_B) / |n_A x n_B| in DIGITS-digit decimal (exact up to that rounding)."""
    ints, _ = scaled_ints((*a1, *a2, *b1, *b2))
    A1, A2, B1, B2 = ints[0:3], ints[3:6], ints[6:9], ints[9:12]
    X = _cross(_cross(A1, A2), _cross(B1, B2))
    with localcontext() as ctx:
        ctx.prec = DIGITS
        r = Decimal(_dot(X, X)).sqrt()
        return tuple(Decimal(sign * c) / r for c in X)


def intersect(a1, a2, b1, b2):
    count, sign, flags = classify(a1, a2, b1, b2)
    return count, flags, (point(a1, a2, b1, b2, sign) if count else None)


# ------------------------------------------------------------------ binary64 replicas

def naive_point(a1, a2, b1, b2, sign):
    nA = _cross(a1, a2)
    nB = _cross(b1, b2)
    X = _cross(nA, nB)
    r = math.sqrt(_dot(X, X))
    return tuple((sign * c) / r for c in X)


def naive_classify(a1, a2, b1, b2):
    """The binary64 decisions of the naive evaluation (same rule, rounded signs)."""
    vals = (*a1, *a2, *b1, *b2)
    if not all(math.isfinite(v) for v in vals):
        return 0, 0, NONFINITE
    nA, nB = _cross(a1, a2), _cross(b1, b2)
    if nA == (0.0, 0.0, 0.0) or nB == (0.0, 0.0, 0.0):
        return 0, 0, DEGEN
    sa1, sa2 = _sign(_dot(nB, a1)), _sign(_dot(nB, a2))
    sb1, sb2 = _sign(_dot(nA, b1)), _sign(_dot(nA, b2))
    if sa1 == 0 and sa2 == 0:
        return 0, 0, COPLANAR
    if sa1 >= 0 >= sa2 and sb2 >= 0 >= sb1:
        return 1, 1, HIT
    if sa1 <= 0 <= sa2 and sb2 <= 0 <= sb1:
        return 1, -1, HIT
    return 0, 0, 0


def _normal_pairs(u, v):
    """AccuDOP (Alg. 4) for each component of u x v, renormalised by TwoSum."""
    out = []
    for (a, b, c, d) in ((u[1], v[2], u[2], v[1]), (u[2], v[0], u[0], v[2]),
                         (u[0], v[1], u[1], v[0])):
        h, l = E.accu_dop(a, b, c, d)
        out.append(E.two_sum(h, l))
    return out


def eft_point(a1, a2, b1, b2, sign):
    nA = _normal_pairs(a1, a2)
    nB = _normal_pairs(b1, b2)

    def comp(i, j):  # nA_i nB_j - nA_j nB_i over the (leading, trailing) pairs
        (ai, ei), (aj, ej) = nA[i], nA[j]
        (bi, fi), (bj, fj) = nB[i], nB[j]
        dop, err = E.accu_dop(ai, bj, aj, bi)
        t = ai * fj
        t = E.fma(ei, bj, t)
        t = E.fma(-aj, fi, t)
        t = E.fma(-ej, bi, t)
        return dop + (err + t)

    X = (comp(1, 2), comp(2, 0), comp(0, 1))
    S, s = E.sum_of_squares(X)
    r = math.sqrt(S)
    return tuple((sign * c) / r for c in X)
