"""Alternative binary64 formulas for the arc-latitude points (oracle; test infrastructure only).

The paper compares its method with other ways of evaluating the same intersection (Sec. 7,
the accuracy comparison, and Sec. S2 on Kahan's determinant).  The binary64 ones are
replicated here, each operation as the library's ablation kernel performs it:

* ``eq22``  Eq. (2.2) on the raw normal n = x1 x x2 (the direct evaluation, ``naive.point``);
* ``eq21``  Eq. (2.1) on the unit normal n^ = n / |n|:
            P = -(z0 n^x n^z +- s n^y, z0 n^y n^z -+ s n^x) / (n^x^2 + n^y^2),
            s = sqrt(n^x^2 + n^y^2 - z0^2);
* ``eq71``  Eq. (7.1): Eq. (2.1) with the denominator 1 - n^z^2 and s = sqrt(1 - n^z^2 - z0^2),
            which cancels catastrophically when n^z^2 is close to 1;
* ``kahan`` Eq. (2.2) with each normal component by Kahan's DiffOfProd (Alg. 3).

Every formula is written once over an arithmetic object, so the same code runs in binary64
(the replica) and in 100-digit decimal: the decimal run must reproduce the exact points of
``geometry.points`` (the pin that each formula, its signs and its root labels are right).
Upper signs are PLUS, as in Eq. (2.2).  Operation order (left to right unless bracketed):

    |n|^2 = (nx nx + ny ny) + nz nz,  r = sqrt(|n|^2),  n^ = (nx / r, ny / r, nz / r)
    eq21: T = n^x n^x + n^y n^y,  s2 = T - z0 z0
    eq71: T = 1 - n^z n^z,        s2 = T - z0 z0
    ax = (n^x n^z) z0, bx = s n^y, ay = (n^y n^z) z0, by = s n^x
    P+ = (-((ax + bx) / T), -((ay - by) / T)),  P- = (-((ax - bx) / T), -((ay + by) / T))

A formula whose existence quantity (s2, or its denominator) is negative or zero for a pair
returns None: that variant reports no points there.
"""

from __future__ import annotations

import math
from decimal import Decimal, localcontext

from . import eft as E
from .geometry import PLUS

DIGITS = 100


class Binary64:
    @staticmethod
    def num(v):
        return float(v)

    sqrt = staticmethod(math.sqrt)
    fma = staticmethod(E.fma)


class Dec:
    @staticmethod
    def num(v):
        return Decimal(v)

    @staticmethod
    def sqrt(v):
        return v.sqrt()

    @staticmethod
    def fma(a, b, c):
        return a * b + c


def _normal(x1, x2, A, kahan=False):
    x1 = [A.num(v) for v in x1]
    x2 = [A.num(v) for v in x2]
    if kahan:
        def dop(a, d, b, c):  # a*d - b*c by Alg. 3 as printed
            bc = b * c
            err = A.fma(-b, c, bc)
            return A.fma(a, d, -bc) + err
        return (dop(x1[1], x2[2], x1[2], x2[1]), dop(x1[2], x2[0], x1[0], x2[2]),
                dop(x1[0], x2[1], x1[1], x2[0]))
    return (x1[1] * x2[2] - x1[2] * x2[1], x1[2] * x2[0] - x1[0] * x2[2],
            x1[0] * x2[1] - x1[1] * x2[0])


def _eq22(n, z0, root, A):
    nx, ny, nz = n
    S2 = nx * nx + ny * ny
    S3 = S2 + nz * nz
    s2 = S2 - S3 * (z0 * z0)
    if not S2 > 0 or s2 < 0:
        return None
    s = A.sqrt(s2)
    ax, bx, ay, by = (nx * nz) * z0, s * ny, (ny * nz) * z0, s * nx
    if root == PLUS:
        return (-((ax + bx) / S2), -((ay - by) / S2))
    return (-((ax - bx) / S2), -((ay + by) / S2))


def _unit(n, A):
    nx, ny, nz = n
    r = A.sqrt((nx * nx + ny * ny) + nz * nz)
    if not r > 0:
        return None
    return nx / r, ny / r, nz / r


def _eq21_71(h, z0, root, A, eq71):
    hx, hy, hz = h
    T = (A.num(1) - hz * hz) if eq71 else hx * hx + hy * hy
    s2 = T - z0 * z0
    if not T > 0 or s2 < 0:
        return None
    s = A.sqrt(s2)
    ax, bx, ay, by = (hx * hz) * z0, s * hy, (hy * hz) * z0, s * hx
    if root == PLUS:
        return (-((ax + bx) / T), -((ay - by) / T))
    return (-((ax - bx) / T), -((ay + by) / T))


def point(variant, x1, x2, z0, root, A=Binary64):
    """The variant's point for one root label, or None where it reports none."""
    z0 = A.num(z0)
    if variant in ("eq22", "kahan"):
        return _eq22(_normal(x1, x2, A, kahan=variant == "kahan"), z0, root, A)
    h = _unit(_normal(x1, x2, A), A)
    if h is None:
        return None
    return _eq21_71(h, z0, root, A, eq71=variant == "eq71")


def point_decimal(variant, x1, x2, z0, root):
    with localcontext() as ctx:
        ctx.prec = DIGITS
        return point(variant, x1, x2, z0, root, A=Dec)


VARIANTS = ("eq22", "eq21", "eq71", "kahan")
