"""The plain definition of the result, evaluated exactly (oracle; test infrastructure only).

Problem (Sec. 1.2, "Problem Definition"): binary64 inputs x1, x2 in F^3 and z0 in F.  The
great-circle arc is the shortest path between the sphere points x1/|x1| and x2/|x2| (the
footnote of Sec. 1.2 makes the formula invariant to |x1| and |x2|); it lies in the plane
through the origin with normal n = x1 x x2.  The constant-latitude circle is the sphere cut
by z = z0.  They meet in 0, 1 or 2 points.

Sec. 2: the two planes and the sphere meet iff |n_xy|^2 >= |n|^2 z0^2, in two points when
the inequality is strict, and the points are Eq. (2.2):

    P = -( z0 n_x n_z +- s n_y ,  z0 n_y n_z -+ s n_x ) / |n_xy|^2 ,   P_z = z0,
    s = sqrt(|n_xy|^2 - |n|^2 z0^2).

"Upper signs" (+ in x, - in y) is root PLUS, "lower signs" is root MINUS.  For s > 0, PLUS
is the crossing where z increases when travelling x1 -> x2, since (n x P_plus)_z = +s.

Sec. 2 also says any point found must still be checked to lie between x1 and x2, without
giving a method.  The reading taken here: along the minor arc, z(t) is a sinusoid sampled
over less than half a period, so it is monotone or has exactly one interior extremum.  The
sign of dz/dt at each endpoint, d_i = (n x x_i)_z = n_x y_i - n_y x_i, tells which:

    d1 >= 0, d2 >= 0   monotone up      PLUS  hits iff  zh1 <= z0 <= zh2
    d1 <= 0, d2 <= 0   monotone down    MINUS hits iff  zh2 <= z0 <= zh1
    d1 >  0 >  d2      apex inside      PLUS iff zh1 <= z0,  MINUS iff zh2 <= z0
    d1 <  0 <  d2      nadir inside     MINUS iff z0 <= zh1, PLUS iff z0 <= zh2

where zh_i = z_i / |x_i| is the height of the normalised endpoint (closed arc: endpoints
count), and all of it only when s^2 >= 0.  With s^2 = 0 the two roots coincide and one hit
is reported (the first in along-arc order).  Hits are listed in along-arc order: apex case
PLUS then MINUS, nadir case MINUS then PLUS.

Every sign above is decided exactly: the binary64 inputs are turned into integers with a
common power-of-two scale, and each predicate is a polynomial in those integers.
Point coordinates are Eq. (2.2) on the exact normal, with only the square root and the
final division rounded, in 100-digit decimal arithmetic.
"""

from __future__ import annotations

import math
from decimal import Decimal, localcontext
from typing import NamedTuple

# Per-pair flag bits (shared meaning with the library's public header, defined here
# independently).
EXISTS = 1      # great circle meets the latitude circle: s^2 >= 0 with n != 0, n_xy != 0
TANGENT = 2     # s^2 == 0 exactly: a double root, reported once
DEGEN_N = 4     # n == 0: coincident, antipodal or zero endpoints
HORIZ = 8       # n_xy == 0, n != 0: the great circle is the equator
NONFINITE = 16  # some input is inf or nan

PLUS = 0   # upper signs of Eq. (2.2); the ascending crossing
MINUS = 1  # lower signs of Eq. (2.2); the descending crossing

DIGITS = 100  # decimal digits for the point phase


class Classification(NamedTuple):
    count: int
    roots: tuple   # root labels in along-arc order
    flags: int


def _sign(v: int) -> int:
    return (v > 0) - (v < 0)


def scaled_ints(values):
    """Exact integers I_k and a shift K with values[k] == I_k / 2**K (finite binary64 only)."""
    ratios = [float(v).as_integer_ratio() for v in values]
    shifts = [den.bit_length() - 1 for _, den in ratios]  # den is a power of two
    K = max(shifts)
    return [num << (K - k) for (num, _), k in zip(ratios, shifts)], K


def _height_cmp(Z0: int, X: int, Y: int, Z: int, K: int) -> int:
    """sign(z0 - z/|x|) for scaled integers (z0 = Z0/2^K, x = (X,Y,Z)/2^K), exactly."""
    if Z0 == 0:
        return -_sign(Z)
    if Z == 0 or _sign(Z0) != _sign(Z):
        return _sign(Z0)
    # same nonzero sign: compare |z0| * |x| with |z|, squared, in common units:
    # z0^2 |x|^2 = Z0^2 (X^2+Y^2+Z^2) / 2^(4K),   z^2 = Z^2 / 2^(2K)
    return _sign(Z0) * _sign(Z0 * Z0 * (X * X + Y * Y + Z * Z) - (Z * Z << (2 * K)))


def exact_terms(x1, x2, z0):
    """Scaled exact normal and s^2:  n = N / 2^(2K),  s^2 = s2 / 2^(6K),  |n_xy|^2 = S2 / 2^(4K)."""
    (X1, Y1, Z1, X2, Y2, Z2, Z0), K = scaled_ints((*x1, *x2, z0))
    Nx = Y1 * Z2 - Z1 * Y2
    Ny = Z1 * X2 - X1 * Z2
    Nz = X1 * Y2 - Y1 * X2
    S2 = Nx * Nx + Ny * Ny
    S3 = S2 + Nz * Nz
    s2 = (S2 << (2 * K)) - S3 * Z0 * Z0
    return dict(K=K, X1=X1, Y1=Y1, Z1=Z1, X2=X2, Y2=Y2, Z2=Z2, Z0=Z0,
                Nx=Nx, Ny=Ny, Nz=Nz, S2=S2, S3=S3, s2=s2)


def classify(x1, x2, z0) -> Classification:
    """Exact hit count, root labels (along-arc order) and flags for one arc-latitude pair."""
    if not all(math.isfinite(v) for v in (*x1, *x2, z0)):
        return Classification(0, (), NONFINITE)
    t = exact_terms(x1, x2, z0)
    if t["Nx"] == 0 and t["Ny"] == 0 and t["Nz"] == 0:
        return Classification(0, (), DEGEN_N)
    if t["S2"] == 0:
        return Classification(0, (), HORIZ)
    sg = _sign(t["s2"])
    if sg < 0:
        return Classification(0, (), 0)
    flags = EXISTS | (TANGENT if sg == 0 else 0)
    Nx, Ny, K = t["Nx"], t["Ny"], t["K"]
    d1 = _sign(Nx * t["Y1"] - Ny * t["X1"])
    d2 = _sign(Nx * t["Y2"] - Ny * t["X2"])
    c1 = _height_cmp(t["Z0"], t["X1"], t["Y1"], t["Z1"], K)  # sign(z0 - zh1)
    c2 = _height_cmp(t["Z0"], t["X2"], t["Y2"], t["Z2"], K)  # sign(z0 - zh2)
    if d1 >= 0 and d2 >= 0:
        roots = [PLUS] if (c1 >= 0 and c2 <= 0) else []
    elif d1 <= 0 and d2 <= 0:
        roots = [MINUS] if (c2 >= 0 and c1 <= 0) else []
    elif d1 > 0:  # d1 > 0 > d2: the apex of the great circle is inside the arc
        roots = ([PLUS] if c1 >= 0 else []) + ([MINUS] if c2 >= 0 else [])
    else:         # d1 < 0 < d2: the nadir is inside the arc
        roots = ([MINUS] if c1 <= 0 else []) + ([PLUS] if c2 <= 0 else [])
    if sg == 0 and roots:
        roots = roots[:1]
    return Classification(len(roots), tuple(roots), flags)


def points(x1, x2, z0, roots):
    """Eq. (2.2) for the given root labels, as 100-digit Decimals (Px, Py).

    In scaled integers: P_x = -(Z0 Nx Nz + sigma sqrt(s2) Ny) / (2^K S2),
                        P_y = -(Z0 Ny Nz - sigma sqrt(s2) Nx) / (2^K S2),
    sigma = +1 for PLUS.  Z0 Nx Nz and 2^K S2 are exact integers; only sqrt, the two
    products with it, the two sums and the division round (at 100 digits).
    """
    if not roots:
        return []
    t = exact_terms(x1, x2, z0)
    out = []
    with localcontext() as ctx:
        ctx.prec = DIGITS
        sq = Decimal(t["s2"]).sqrt()
        den = Decimal(t["S2"] << t["K"])
        ax = Decimal(t["Z0"] * t["Nx"] * t["Nz"])
        ay = Decimal(t["Z0"] * t["Ny"] * t["Nz"])
        bx = sq * Decimal(t["Ny"])
        by = sq * Decimal(t["Nx"])
        for r in roots:
            if r == PLUS:
                out.append((-(ax + bx) / den, -(ay - by) / den))
            else:
                out.append((-(ax - bx) / den, -(ay + by) / den))
    return out


def intersect(x1, x2, z0):
    """(Classification, [(Px, Py), ...]) for one pair."""
    c = classify(x1, x2, z0)
    return c, points(x1, x2, z0, c.roots)
