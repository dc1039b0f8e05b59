"""The paper's error-free-transformation algorithms in IEEE binary64 (oracle; test only).

Python floats are IEEE binary64 with correctly rounded +, -, *, / and sqrt (round to
nearest, ties to even), which is the arithmetic model of Sec. 3.  ``fma`` below rounds the
exact a*b + c once, computed in rationals, so fl(a*b - c) means one rounding as Sec. 3
requires.  Each function follows its algorithm's steps in the paper's order and notation.

Readings where the printed text is silent, garbled or inconsistent (each is listed with its
reason in the design notes):

* TwoSum, TwoProduct, FastTwoSum are not printed (Sec. 5.1 names them): the textbook
  Knuth TwoSum, the FMA TwoProduct, and Dekker's FastTwoSum are used.
* AccuDOP (Alg. 4) multiplies a*d and b*c, but Alg. 8 calls it with the operands of the
  cross product in the order (a, b, c, d) -> a*b - c*d; the normal must be n = x1 x x2
  (Table 1), so AccuDOP(a, b, c, d) here returns a*b - c*d.
* AccuDOP's compensation is printed as fl(s + fl(r1 + r2)); the exact identity
  a*b - c*d = (p1 - p2) + (r1 - r2) requires fl(s + fl(r1 - r2)), used here.
* AccSqrt is not printed (Sec. 6 cites Rump 2023, bound 25/8 u^2): the double-word square
  root with one first-order correction -- sh = RN(sqrt(a)), rho1 = fl(a - sh*sh) (one FMA),
  rho2 = fl(rho1 + e), sl = fl(rho2 / (2 sh)), then FastTwoSum(sh, sl) -- whose published
  relative error bound is 25/8 u^2.  A non-positive leading part gives (0, 0).
* The second root uses the lower signs of Eq. (2.2): AccuX with (s, e_s) negated.
* Normal renormalisation (a deviation, on by default): after heavy cancellation in
  a*b - c*d (short arcs), AccuDOP's err can be far larger than u |dop|, while Alg. 7
  drops the sum of e_i^2, which is only negligible when |e_i| <= u |x_i| (the property
  Alg. 7 itself restores with its final FastTwoSum).  On arcs of 1e-10 rad the printed
  algorithm is then off by thousands of u.  ``accux_parts(normalize_normal=True)`` passes
  each (dop, err) through TwoSum before Alg. 7; ``False`` runs the algorithm as printed.
"""

from __future__ import annotations

import math
from fractions import Fraction


# ---------------------------------------------------------------- primitive operations

def fma(a: float, b: float, c: float) -> float:
    """fl(a*b + c) with a single rounding (exact rational, then one correctly rounded step)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def two_sum(a: float, b: float):
    """Knuth's TwoSum: s = fl(a+b) and e with a + b = s + e exactly (no precondition)."""
    s = a + b
    bv = s - a
    av = s - bv
    return s, (a - av) + (b - bv)


def fast_two_sum(a: float, b: float):
    """Dekker's FastTwoSum: s = fl(a+b), e = fl(b - fl(s - a)); exact when exp(a) >= exp(b)."""
    s = a + b
    return s, b - (s - a)


def two_product(a: float, b: float):
    """TwoProduct with FMA: p = fl(a*b), e = fl(a*b - p) (exact)."""
    p = a * b
    return p, fma(a, b, -p)


# ---------------------------------------------------------------- Sec. 5 operators

def comp_dot_c(x, y):
    """Alg. 1 (CompDotC): dot product returned as the pair (p_n, s_n)."""
    p, s = two_product(x[0], y[0])
    for i in range(1, len(x)):
        h, r = two_product(x[i], y[i])
        p, q = two_sum(p, h)
        s = s + (q + r)
    return p, s


def comp_dot(x, y):
    """Alg. 2 (CompDot, Ogita-Rump-Oishi Dot2): fl(p_n + s_n) of CompDotC."""
    p, s = comp_dot_c(x, y)
    return p + s


def kahan_dop(a, b, c, d):
    """Alg. 3 (Kahan's DiffOfProd) as printed: a*d - b*c with two FMAs."""
    bc = b * c
    err = fma(-b, c, bc)
    dop = fma(a, d, -bc)
    return dop + err


def accu_dop(a, b, c, d):
    """Alg. 4 (AccuDOP), read as a*b - c*d returned as the pair (dop, err)."""
    p1, r1 = two_product(a, b)
    p2, r2 = two_product(c, d)
    dop, s = two_sum(p1, -p2)
    err = s + (r1 - r2)
    return dop, err


def sum_non_neg(A, a, B, b):
    """Alg. 6 (SumNonNeg): sum of two non-negative pairs [A, a] + [B, b]."""
    H, h = two_sum(A, B)
    c = a + b
    d = h + c
    return fast_two_sum(H, d)


def sum_of_squares(x):
    """Alg. 5 (SumOfSquares, Graillat et al. 2015): sum of x_j^2 as a pair."""
    S, s = 0.0, 0.0
    for xj in x:
        P, p = two_product(xj, xj)
        S, s = sum_non_neg(S, s, P, p)
    return S, s


def sum_of_squares_c(x, e):
    """Alg. 7 (SumOfSquaresC): sum of (x_j + e_j)^2 as a pair (S, s) with |s| <= u|S|."""
    S_, s_ = sum_of_squares(x)
    R_ = comp_dot(x, e)
    R = fma(2.0, R_, s_)
    return fast_two_sum(S_, R)


def acc_sqrt(a, e):
    """AccSqrt of the pair a + e (|e| <= u a), as the pair (s, e_s); see the module notes."""
    if not a > 0.0:
        return 0.0, 0.0
    sh = math.sqrt(a)
    rho1 = fma(-sh, sh, a)
    rho2 = rho1 + e
    sl = rho2 / (2.0 * sh)
    return fast_two_sum(sh, sl)


# ---------------------------------------------------------------- Alg. 8 (AccuX)

def accux_parts(x1, x2, z0, normalize_normal=True):
    """Steps of Alg. 8 up to AccSqrt, returned by name (for the intermediate-value tests)."""
    nx, enx = accu_dop(x1[1], x2[2], x1[2], x2[1])
    ny, eny = accu_dop(x1[2], x2[0], x1[0], x2[2])
    nz, enz = accu_dop(x1[0], x2[1], x1[1], x2[0])
    if normalize_normal:
        nx, enx = two_sum(nx, enx)
        ny, eny = two_sum(ny, eny)
        nz, enz = two_sum(nz, enz)
    S2, s2 = sum_of_squares_c([nx, ny], [enx, eny])
    S3, s3 = sum_of_squares_c([nx, ny, nz], [enx, eny, enz])
    C, eC = two_product(z0, z0)
    D, eD = comp_dot_c([S3, S3, s3, s3], [C, eC, C, eC])
    E, eE = two_sum(S2, -D)
    e = (s2 - eD) + eE
    ss, ess = fast_two_sum(E, e)
    sb, es = acc_sqrt(ss, ess)
    Fx, eFx1 = two_product(nx, nz)
    eFx2 = nx * enz
    eFx3 = nz * enx
    eFx = (eFx1 + eFx2) + eFx3
    Fy, eFy1 = two_product(ny, nz)
    eFy2 = ny * enz
    eFy3 = nz * eny
    eFy = (eFy1 + eFy2) + eFy3
    return dict(nx=nx, enx=enx, ny=ny, eny=eny, nz=nz, enz=enz, S2=S2, s2=s2, S3=S3,
                s3=s3, C=C, eC=eC, D=D, eD=eD, E=E, eE=eE, e=e, ss=ss, ess=ess, sb=sb,
                es=es, Fx=Fx, eFx=eFx, Fy=Fy, eFy=eFy)


def accux_numerators(q, z0, sigma=1):
    """The two CompDot numerators of Alg. 8 (sigma=-1: lower signs), before the division."""
    sb, es = sigma * q["sb"], sigma * q["es"]
    x = comp_dot([q["Fx"], q["eFx"], q["ny"], q["eny"], q["ny"], q["eny"]],
                 [z0, z0, sb, sb, es, es])
    y = comp_dot([q["Fy"], q["eFy"], -q["nx"], -q["enx"], -q["nx"], -q["enx"]],
                 [z0, z0, sb, sb, es, es])
    return x, y


def accux(x1, x2, z0, sigma=1, normalize_normal=True):
    """Alg. 8 (AccuX): the intersection point (P_x, P_y); sigma=+1 upper signs, -1 lower."""
    q = accux_parts(x1, x2, z0, normalize_normal)
    x, y = accux_numerators(q, z0, sigma)
    Rx = x / q["S2"]
    Ry = y / q["S2"]
    return -Rx, -Ry
