"""Direct binary64 evaluation of Eq. (2.2) (oracle; test infrastructure only).

Sec. 4 analyses "the most straightforward approach": Eq. (2.2) translated operation by
operation into binary64, with no contraction into FMAs (the paper builds with
-ffp-contract=off, Sec. 7.2).  The operation order follows the evaluation tree of the
supplement's Sec. S1:

    n_x = fl(fl(y1 z2) - fl(z1 y2)),  n_y = fl(fl(z1 x2) - fl(x1 z2)),  n_z = fl(fl(x1 y2) - fl(y1 x2))
    S2 = fl(fl(n_x^2) + fl(n_y^2)),   S3 = fl(S2 + fl(n_z^2))
    s2 = fl(S2 - fl(S3 fl(z0^2))),    s = sqrt(s2)
    P_x = -fl( fl( fl(fl(n_x n_z) z0) +- fl(s n_y) ) / S2 )
    P_y = -fl( fl( fl(fl(n_y n_z) z0) -+ fl(s n_x) ) / S2 )

Existence and containment are decided with the same hit rule as the exact oracle (see
``geometry``), but every sign is the sign of a binary64 value and the endpoint heights are
the raw z1, z2 (unit-length inputs assumed, as a direct implementation does):

    d_i = fl(fl(n_x y_i) - fl(n_y x_i)),   compare z0 with z1 and z2 directly.

This is the reference for the library's naive mode, which must match it bit for bit; its
disagreements with the exact oracle are the robustness loss that mode is meant to show.
"""

from __future__ import annotations

import math

from .geometry import EXISTS, TANGENT, DEGEN_N, HORIZ, NONFINITE, PLUS, MINUS


def _sgn(v: float) -> int:
    return int(v > 0.0) - int(v < 0.0)


def normal(x1, x2):
    nx = x1[1] * x2[2] - x1[2] * x2[1]
    ny = x1[2] * x2[0] - x1[0] * x2[2]
    nz = x1[0] * x2[1] - x1[1] * x2[0]
    return nx, ny, nz


def classify(x1, x2, z0):
    """(count, roots, flags) with binary64 predicates."""
    if not all(math.isfinite(v) for v in (*x1, *x2, z0)):
        return 0, (), NONFINITE
    nx, ny, nz = normal(x1, x2)
    if nx == 0.0 and ny == 0.0 and nz == 0.0:
        return 0, (), DEGEN_N
    S2 = nx * nx + ny * ny
    if S2 == 0.0:
        return 0, (), HORIZ
    S3 = S2 + nz * nz
    s2 = S2 - S3 * (z0 * z0)
    if s2 < 0.0:
        return 0, (), 0
    flags = EXISTS | (TANGENT if s2 == 0.0 else 0)
    d1 = _sgn(nx * x1[1] - ny * x1[0])
    d2 = _sgn(nx * x2[1] - ny * x2[0])
    c1 = _sgn(z0 - x1[2])
    c2 = _sgn(z0 - x2[2])
    if d1 >= 0 and d2 >= 0:
        roots = [PLUS] if (c1 >= 0 and c2 <= 0) else []
    elif d1 <= 0 and d2 <= 0:
        roots = [MINUS] if (c2 >= 0 and c1 <= 0) else []
    elif d1 > 0:
        roots = ([PLUS] if c1 >= 0 else []) + ([MINUS] if c2 >= 0 else [])
    else:
        roots = ([MINUS] if c1 <= 0 else []) + ([PLUS] if c2 <= 0 else [])
    if s2 == 0.0 and roots:
        roots = roots[:1]
    return len(roots), tuple(roots), flags


def point(x1, x2, z0, root):
    """Eq. (2.2) in binary64 for one root label (PLUS: upper signs)."""
    nx, ny, nz = normal(x1, x2)
    S2 = nx * nx + ny * ny
    S3 = S2 + nz * nz
    s2 = S2 - S3 * (z0 * z0)
    s = math.sqrt(s2) if s2 > 0.0 else 0.0
    ax = (nx * nz) * z0
    bx = s * ny
    ay = (ny * nz) * z0
    by = s * nx
    if root == PLUS:
        return -((ax + bx) / S2), -((ay - by) / S2)
    return -((ax - bx) / S2), -((ay + by) / S2)


def intersect(x1, x2, z0):
    count, roots, flags = classify(x1, x2, z0)
    return count, roots, flags, [point(x1, x2, z0, r) for r in roots]
