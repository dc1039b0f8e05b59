"""A second, independent derivation of the intersection points (oracle cross-check only).

Instead of the line-circle construction behind Eq. (2.2), parametrise the great circle of
the arc by angle: with u = x1/|x1| and v the unit vector in the arc's plane orthogonal to u
and pointing towards x2,

    x(theta) = cos(theta) u + sin(theta) v,    theta in [0, theta12],
    z(theta) = u_z cos(theta) + v_z sin(theta) = R cos(theta - phi),

R = hypot(u_z, v_z), phi = atan2(v_z, u_z).  z(theta) = z0 has the solutions
theta = phi -+ acos(z0 / R); the first is ascending (dz/dtheta > 0), i.e. root PLUS, the
second descending (MINUS).  A solution is a hit if it falls in [0, theta12] mod 2 pi.
Everything runs in mpmath at ``prec`` bits; it shares nothing with ``geometry`` and is
used by the tests to pin ``geometry`` away from exact ties.
"""

from __future__ import annotations

import mpmath as mp

from .geometry import PLUS, MINUS


def intersect(x1, x2, z0, prec: int = 300):
    """([(root, theta, Px, Py), ...] sorted by theta, margin) with mpf values.

    ``margin`` is the distance of the decision from a tie: min over the hit tests of
    |theta|, |theta - theta12| and acos(z0/R) (the half-separation of the two roots);
    callers skip cases whose margin is tiny.
    """
    with mp.workprec(prec):
        a = [mp.mpf(v) for v in x1]
        b = [mp.mpf(v) for v in x2]
        na = mp.sqrt(sum(t * t for t in a))
        nb = mp.sqrt(sum(t * t for t in b))
        u = [t / na for t in a]
        w = [t / nb for t in b]
        c = sum(p * q for p, q in zip(u, w))
        v = [wq - c * uq for wq, uq in zip(w, u)]
        nv = mp.sqrt(sum(t * t for t in v))
        v = [t / nv for t in v]
        cr = [u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]]
        theta12 = mp.atan2(mp.sqrt(sum(t * t for t in cr)), c)
        R = mp.sqrt(u[2] ** 2 + v[2] ** 2)
        phi = mp.atan2(v[2], u[2])
        z = mp.mpf(z0)
        if R == 0 or abs(z) > R:
            return [], mp.mpf(1)
        half = mp.acos(z / R)
        two_pi = 2 * mp.pi
        out = []
        margin = half
        for root, th in ((PLUS, phi - half), (MINUS, phi + half)):
            th = th % two_pi
            margin = min(margin, abs(th), abs(th - theta12), abs(two_pi - th))
            if th <= theta12:
                ct, st = mp.cos(th), mp.sin(th)
                out.append((root, th, ct * u[0] + st * v[0], ct * u[1] + st * v[1]))
        out.sort(key=lambda t: t[1])
        return out, margin
