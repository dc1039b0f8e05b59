// Per-arc and per-pair evaluation of the arc x constant-latitude intersection.
//
// Problem and formula: Sec. 1.2 and Sec. 2 of Chen, Ullrich & Panetta.  Two modes:
//   * naive:  Eq. (2.2) translated operation by operation into binary64 (Sec. 4), with
//             binary64 existence/containment tests and raw endpoint heights;
//   * EFT:    Alg. 8 (AccuX) with the AccuDOP pairs renormalised, and exact existence and
//             containment decisions (filters, then expansion arithmetic).
//
// Containment (Sec. 2 leaves the method open): along the minor arc, z is monotone or has
// one interior extremum; with d_i = sign(dz/dt) at the endpoints (d_i = sign(n_x y_i -
// n_y x_i)) and c_i = sign(z0 - z_i/|x_i|):
//     d1 >= 0, d2 >= 0 : PLUS  iff c1 >= 0 && c2 <= 0
//     d1 <= 0, d2 <= 0 : MINUS iff c2 >= 0 && c1 <= 0
//     d1 > 0 > d2      : PLUS iff c1 >= 0, then MINUS iff c2 >= 0   (apex inside)
//     d1 < 0 < d2      : MINUS iff c1 <= 0, then PLUS iff c2 <= 0   (nadir inside)
// provided s^2 >= 0; at s^2 == 0 only the first listed hit is kept.  PLUS is Eq. (2.2) with
// the upper signs (the ascending crossing), MINUS the lower signs.
//
// Everything here is __host__ __device__ so the identical arithmetic can be compiled for
// the CPU in tests.  Decisions a filter cannot certify come back as UNDECIDED; the caller
// resolves them with exact_sign (on the GPU, one lane at a time per wavefront).
#pragma once
#pragma clang fp contract(off)

#include "sphint_eft.hpp"
#include "sphint_exact.hpp"

namespace sphint {

enum : unsigned {
  F_EXISTS = 1u,
  F_TANGENT = 2u,
  F_DEGEN_N = 4u,
  F_HORIZ = 8u,
  F_NONFINITE = 16u,
  F_FALLBACK = 32u,  // diagnostic: an exact expansion evaluation decided this pair
  F_INTERNAL = 64u,  // an exact evaluation exceeded its arena (outside the input domain)
  F_NEEDEXACT = 128u,  // internal: a filter could not decide; re-evaluate with exact signs
};
enum : int { ROOT_PLUS = 0, ROOT_MINUS = 1 };
constexpr int UNDECIDED = 2;

__host__ __device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// The containment rule above; returns the hit count, roots in along-arc order.
__host__ __device__ __forceinline__ int hit_rule(int d1, int d2, int c1, int c2, bool tangent,
                                                 int& r0, int& r1) {
  int n = 0;
  r0 = ROOT_PLUS;
  r1 = ROOT_MINUS;
  if (d1 >= 0 && d2 >= 0) {
    n = (c1 >= 0 && c2 <= 0);
    r0 = ROOT_PLUS;
  } else if (d1 <= 0 && d2 <= 0) {
    n = (c2 >= 0 && c1 <= 0);
    r0 = ROOT_MINUS;
  } else if (d1 > 0) {
    bool a = c1 >= 0, b = c2 >= 0;
    n = (int)a + (int)b;
    r0 = a ? ROOT_PLUS : ROOT_MINUS;
    r1 = ROOT_MINUS;
  } else {
    bool a = c1 <= 0, b = c2 <= 0;
    n = (int)a + (int)b;
    r0 = a ? ROOT_MINUS : ROOT_PLUS;
    r1 = ROOT_PLUS;
  }
  if (tangent && n > 1) n = 1;
  return n;
}

// Result of one pair: up to two points in along-arc order.
struct PairOut {
  double px0, py0, px1, py1;
  int count, r0, r1;
  unsigned flags;
};

// =========================================================================== naive mode

struct ArcNaive {
  double nx, ny, nz, S2, S3;
  double x1, y1, z1, x2, y2, z2;
  int d1, d2;
  unsigned flags;
};

__host__ __device__ __forceinline__ void arc_naive(double x1, double y1, double z1, double x2,
                                                   double y2, double z2, ArcNaive& a) {
  a.x1 = x1; a.y1 = y1; a.z1 = z1; a.x2 = x2; a.y2 = y2; a.z2 = z2;
  a.flags = 0;
  a.d1 = a.d2 = 0;
  a.nx = a.ny = a.nz = a.S2 = a.S3 = 0.0;
  if (!(finite(x1) && finite(y1) && finite(z1) && finite(x2) && finite(y2) && finite(z2))) {
    a.flags = F_NONFINITE;
    return;
  }
  a.nx = y1 * z2 - z1 * y2;
  a.ny = z1 * x2 - x1 * z2;
  a.nz = x1 * y2 - y1 * x2;
  if (a.nx == 0.0 && a.ny == 0.0 && a.nz == 0.0) {
    a.flags = F_DEGEN_N;
    return;
  }
  a.S2 = a.nx * a.nx + a.ny * a.ny;
  if (a.S2 == 0.0) {
    a.flags = F_HORIZ;
    return;
  }
  a.S3 = a.S2 + a.nz * a.nz;
  a.d1 = sgn(a.nx * y1 - a.ny * x1);
  a.d2 = sgn(a.nx * y2 - a.ny * x2);
}

__host__ __device__ __forceinline__ PairOut pair_naive(const ArcNaive& a, double z0) {
  PairOut o;
  o.count = 0;
  o.r0 = o.r1 = 0;
  o.px0 = o.py0 = o.px1 = o.py1 = 0.0;
  o.flags = a.flags;
  if (a.flags) return o;
  if (!finite(z0)) {
    o.flags = F_NONFINITE;
    return o;
  }
  double s2 = a.S2 - a.S3 * (z0 * z0);
  if (s2 < 0.0) return o;
  bool tangent = s2 == 0.0;
  o.flags = F_EXISTS | (tangent ? F_TANGENT : 0u);
  int c1 = sgn(z0 - a.z1);
  int c2 = sgn(z0 - a.z2);
  o.count = hit_rule(a.d1, a.d2, c1, c2, tangent, o.r0, o.r1);
  if (o.count == 0) return o;
  double s = __builtin_sqrt(s2);
  double ax = (a.nx * a.nz) * z0;
  double bx = s * a.ny;
  double ay = (a.ny * a.nz) * z0;
  double by = s * a.nx;
  double xp = -((ax + bx) / a.S2), yp = -((ay - by) / a.S2);  // upper signs
  double xm = -((ax - bx) / a.S2), ym = -((ay + by) / a.S2);  // lower signs
  o.px0 = o.r0 == ROOT_PLUS ? xp : xm;
  o.py0 = o.r0 == ROOT_PLUS ? yp : ym;
  o.px1 = o.r1 == ROOT_PLUS ? xp : xm;
  o.py1 = o.r1 == ROOT_PLUS ? yp : ym;
  return o;
}

// =========================================================================== EFT mode

// Sign of dz/dt at endpoint (x, y): n_x y - n_y x, filtered in two stages.
// Stage 1 (binary64): error <= 3.01 u (|n_x y| + |n_y x|) + 3.01 u^2 (|y| m_x + |x| m_y).
// Stage 2 (CompDotC over the renormalised pairs, Eq. 5.1 with n = 4): error
// <= 16.1 u^2 (|n_x y| + |n_y x|) + 3.01 u^2 (|y| m_x + |x| m_y).
// Thresholds carry a factor >= 5 (stage 1) and >= 60 (stage 2) of margin.
__host__ __device__ __forceinline__ int d_sign(const ArcEft& a, double x, double y) {
  double A = a.nx * y;
  double Bv = a.ny * x;
  double w0 = A - Bv;
  double mag = __builtin_fabs(A) + __builtin_fabs(Bv);
  double side = __builtin_fabs(y) * a.mx + __builtin_fabs(x) * a.my;
  if (__builtin_fabs(w0) > 0x1p-49 * mag + 0x1p-96 * side) return sgn(w0);
  dd p = two_prod(a.nx, y);
  double s = p.lo, ph = p.hi;
  dd h = two_prod(a.enx, y);
  dd q = two_sum(ph, h.hi);
  ph = q.hi;
  s = s + (q.lo + h.lo);
  h = two_prod(-a.ny, x);
  q = two_sum(ph, h.hi);
  ph = q.hi;
  s = s + (q.lo + h.lo);
  h = two_prod(-a.eny, x);
  q = two_sum(ph, h.hi);
  ph = q.hi;
  s = s + (q.lo + h.lo);
  double w = ph + s;
  if (__builtin_fabs(w) > 0x1p-96 * (mag + side)) return sgn(w);
  return UNDECIDED;
}

// Per-arc part of AccuX (the direction signs are decided by the caller).
__host__ __device__ __forceinline__ void arc_eft(double x1, double y1, double z1, double x2,
                                                 double y2, double z2, ArcEft& a) {
  a.flags = 0;
  a.d1 = a.d2 = 0;
  a.z1 = z1;
  a.z2 = z2;
  if (!(finite(x1) && finite(y1) && finite(z1) && finite(x2) && finite(y2) && finite(z2))) {
    a.flags = F_NONFINITE;
    return;
  }
  // Alg. 8 lines 2-4 (normal n = x1 x x2).  A component is exactly zero iff both
  // TwoProducts agree in both parts (fl(x) and x - fl(x) determine x).
  const dop3 nx = accu_dop(y1, z2, z1, y2);
  const dop3 ny = accu_dop(z1, x2, x1, z2);
  const dop3 nz = accu_dop(x1, y2, y1, x2);
  if (nx.zero && ny.zero && nz.zero) {
    a.flags = F_DEGEN_N;
    return;
  }
  if (nx.zero && ny.zero) {
    a.flags = F_HORIZ;
    return;
  }
  a.nx = nx.hi; a.enx = nx.lo; a.mx = nx.mag;
  a.ny = ny.hi; a.eny = ny.lo; a.my = ny.mag;
  a.nz = nz.hi; a.enz = nz.lo; a.mz = nz.mag;
  norms(a);  // Alg. 8 lines 5-6
  dd fx = f_pair(a.nx, a.enx, a.nz, a.enz);
  dd fy = f_pair(a.ny, a.eny, a.nz, a.enz);
  a.Fx = fx.hi; a.eFx = fx.lo;
  a.Fy = fy.hi; a.eFy = fy.lo;
  a.n21 = (x1 * x1 + y1 * y1) + z1 * z1;
  a.n22 = (x2 * x2 + y2 * y2) + z2 * z2;
  a.zz1 = z1 * z1;
  a.zz2 = z2 * z2;
  a.side = __builtin_fabs(a.nx) * a.mx + __builtin_fabs(a.ny) * a.my + __builtin_fabs(a.nz) * a.mz;
}

// s^2 = |n_xy|^2 - |n|^2 z0^2 (Alg. 8 lines 7-11) and its certified sign.
struct S2Eft {
  double ss, ess;
  int sign;  // -1, 0, 1 or UNDECIDED
};

// Error of (ss + ess) against the exact s^2 (first order):
//   u^2 [14 S2 + 40 S3 z0^2 + 6.02 (1 + z0^2) sum_i |n_i| m_i]
// from Alg. 7 (<= 11 u^2 S2 and 14 u^2 S3 over the renormalised normal), the normal error
// (3.01 u^2 m_i per component), CompDotC over four terms (Eq. 5.1, 16 u^2 S3 z0^2) and the
// compensation sum.  The filter uses 2^-96 = 1024 u^2 per term: a factor >= 25 of margin.
// Alg. 1's TwoSums run here as FastTwoSum: after the leading product S3 C, every term is at
// most about u times the running sum (|C_lo| <= u C, |s3| <= u S3), so FastTwoSum's
// precondition holds and, both being exact, it returns TwoSum's pair.
__host__ __device__ __forceinline__ S2Eft s2_eft(const ArcEft& a, double z0) {
  dd C = two_prod(z0, z0);
  dd p = two_prod(a.S3, C.hi);  // Alg. 1 over {S3, S3, s3, s3} . {C, eC, C, eC}
  double ph = p.hi, s = p.lo;
  dd h = two_prod(a.S3, C.lo);
  dd q = fast_two_sum(ph, h.hi);
  ph = q.hi;
  s = s + (q.lo + h.lo);
  h = two_prod(a.s3, C.hi);
  q = fast_two_sum(ph, h.hi);
  ph = q.hi;
  s = s + (q.lo + h.lo);
  h = two_prod(a.s3, C.lo);
  q = fast_two_sum(ph, h.hi);
  ph = q.hi;
  s = s + (q.lo + h.lo);
  dd E = two_sum(a.S2, -ph);
  double e = (a.s2 - s) + E.lo;
  dd r = fast_two_sum(E.hi, e);
  S2Eft o;
  o.ss = r.hi;
  o.ess = r.lo;
  double B = 0x1p-96 * (a.S2 + a.S3 * C.hi + (1.0 + C.hi) * a.side);
  o.sign = r.hi > B ? 1 : (r.hi < -B ? -1 : UNDECIDED);
  return o;
}

// sign(z0 - z/|x|) for one endpoint, or UNDECIDED (then the exact answer is
// sgn(z0) * sign(z0^2 |x|^2 - z^2)).  Only the same-sign case needs arithmetic:
// Stage 1: t = fl(C n2 - zz) (one FMA) with C = fl(z0^2), n2 = fl(|x|^2) (three products and
//          two sums: relative error <= 3.01 u), zz = fl(z^2): error <= 4.02 u C n2 + u zz +
//          u |t|; threshold 2^-49 (C n2 + zz) = 16 u (...).
// Stage 2: |x|^2 as s2 + L (TwoProducts of the squares, two TwoSums, the five small parts
//          summed: error <= 16 u^2 n2), then (C_hi + C_lo)(s2 + L) - z^2 with one TwoProduct
//          and one TwoSum for the leading terms and the small terms summed: error <=
//          49 u^2 (C n2 + zz) + u |t|; threshold 2^-92 (C n2 + zz) = 16384 u^2 (...).  At
//          arcs near a pole, where heights differ from z0 by a few ulps of 1, stage 1 leaves
//          a few percent of pairs open, and this stage settles them for a third of the cost
//          of a full compensated dot product.
// The endpoint's x and y are needed by stage 2 only; xy() supplies them (as {x, y}).
template <class XY>
__host__ __device__ __forceinline__ int height_cmp_xy(double z0, double z, double n2, double zz,
                                                      dd C, XY&& xy) {
  if (z0 == 0.0) return -sgn(z);
  if (z == 0.0 || ((z0 > 0.0) != (z > 0.0))) return sgn(z0);
  const double mag = C.hi * n2 + zz;
  const double t = __builtin_fma(C.hi, n2, -zz);
  if (__builtin_fabs(t) > 0x1p-49 * mag) return sgn(z0) * sgn(t);
  const dd e = xy();
  const double x = e.hi, y = e.lo;
  const dd X = two_prod(x, x), Y = two_prod(y, y), Z = two_prod(z, z);
  const dd s1 = two_sum(X.hi, Y.hi);
  const dd s2 = two_sum(s1.hi, Z.hi);
  const double L = (((s1.lo + s2.lo) + X.lo) + Y.lo) + Z.lo;
  const dd P = two_prod(C.hi, s2.hi);
  const double rest = (C.hi * L + C.lo * s2.hi) + C.lo * L;
  const dd h = two_sum(P.hi, -Z.hi);
  const double w = h.hi + (((h.lo + P.lo) - Z.lo) + rest);
  if (__builtin_fabs(w) > 0x1p-92 * mag) return sgn(z0) * sgn(w);
  return UNDECIDED;
}

__host__ __device__ __forceinline__ int height_cmp(double z0, double z, double n2, double zz,
                                                   double x, double y, dd C) {
  return height_cmp_xy(z0, z, n2, zz, C, [&] { return dd{x, y}; });
}

// Alg. 2 (CompDot) over six TwoProducts in Alg. 8's term order, split in two: the running
// sum over the first two terms (the z0 terms, the same for both roots) and the rest.
struct CdState {
  double p, s;
};

// The second term is e_F z0 with |e_F| <= 3.01 u |F| (F's pair comes from a TwoProduct and
// two products of renormalised parts), so FastTwoSum returns TwoSum's exact pair.
__host__ __device__ __forceinline__ CdState comp_dot_head(dd t0, dd t1) {
  const dd q = fast_two_sum(t0.hi, t1.hi);
  return {q.hi, t0.lo + (q.lo + t1.lo)};
}

// Continues the sum with sg * t2 ... sg * t5 (sg = +1 or -1; negating a TwoProduct's pair
// negates both parts exactly, so this equals CompDot over the negated products).
__host__ __device__ __forceinline__ double comp_dot_tail(CdState c, dd t2, dd t3, dd t4, dd t5,
                                                         double sg) {
  double p = c.p, s = c.s;
  dd q = two_sum(p, sg * t2.hi); p = q.hi; s = s + (q.lo + sg * t2.lo);
  q = two_sum(p, sg * t3.hi); p = q.hi; s = s + (q.lo + sg * t3.lo);
  q = two_sum(p, sg * t4.hi); p = q.hi; s = s + (q.lo + sg * t4.lo);
  q = two_sum(p, sg * t5.hi); p = q.hi; s = s + (q.lo + sg * t5.lo);
  return p + s;
}

// Alg. 8's numerators and divisions for the roots of a pair (o.count, o.r0, o.r1 set).  The
// lower-sign root is AccuX with (s, e_s) negated, so its TwoProducts are the exact negations
// of the upper root's: the products are formed once, with the sign of the first root, and a
// second root (always the other sign) reuses them negated.  The z0 terms open both CompDots.
// g(k) supplies the arc's terms when they are first needed: k = 0..7 for Fx, e_Fx, Fy, e_Fy,
// n_x, e_nx, n_y, e_ny.
template <class G>
__host__ __device__ __forceinline__ void points_eft_g(G&& g, double S2, double z0,
                                                      const S2Eft& s2, PairOut& o) {
  const dd sq = acc_sqrt(s2.ss, s2.ess);
  const Divider dv = divider(S2);
  const CdState hx = comp_dot_head(two_prod(g(0), z0), two_prod(g(1), z0));
  const CdState hy = comp_dot_head(two_prod(g(2), z0), two_prod(g(3), z0));
  const bool plus0 = o.r0 == ROOT_PLUS;
  const double sb = plus0 ? sq.hi : -sq.hi;
  const double es = plus0 ? sq.lo : -sq.lo;
  {  // x of both roots, then y: the eight TwoProducts of one coordinate live at a time
    const double ny = g(6), eny = g(7);
    const dd x2 = two_prod(ny, sb), x3 = two_prod(eny, sb);
    const dd x4 = two_prod(ny, es), x5 = two_prod(eny, es);
    o.px0 = -quot(dv, comp_dot_tail(hx, x2, x3, x4, x5, 1.0));
    if (o.count == 2) o.px1 = -quot(dv, comp_dot_tail(hx, x2, x3, x4, x5, -1.0));
  }
  {
    const double nx = g(4), enx = g(5);
    const dd y2 = two_prod(-nx, sb), y3 = two_prod(-enx, sb);
    const dd y4 = two_prod(-nx, es), y5 = two_prod(-enx, es);
    o.py0 = -quot(dv, comp_dot_tail(hy, y2, y3, y4, y5, 1.0));
    if (o.count == 2) o.py1 = -quot(dv, comp_dot_tail(hy, y2, y3, y4, y5, -1.0));
  }
}

__host__ __device__ __forceinline__ void points_eft(const ArcEft& a, double z0, const S2Eft& s2,
                                                    PairOut& o) {
  points_eft_g(
      [&](int k) {
        switch (k) {
          case 0: return a.Fx;
          case 1: return a.eFx;
          case 2: return a.Fy;
          case 3: return a.eFy;
          case 4: return a.nx;
          case 5: return a.enx;
          case 6: return a.ny;
          default: return a.eny;
        }
      },
      a.S2, z0, s2, o);
}

// ====================================================================== pair drivers

// The five decisions of one pair: the slopes d1, d2 (sign of dz/dt at the endpoints), the
// existence sign s2 (sign of s^2) and the height comparisons c1, c2 (sign(z0 - z_i/|x_i|));
// UNDECIDED where a filter could not decide.
struct Decisions {
  int d1, d2, s2, c1, c2;
};

// Replaces every UNDECIDED decision by its exact sign (exact_sign in the arena; a height
// comparison is undecided only when z0 and z_i are nonzero with the same sign, and then
// c_i = sgn(z0) * sign(z0^2 |x_i|^2 - z_i^2)).  Returns false if an expansion exceeded the
// arena (the sign is then taken as 0).
__host__ __device__ __forceinline__ bool resolve_exact(Decisions& d, double x1, double y1,
                                                       double z1, double x2, double y2,
                                                       double z2, double z0, double* arena) {
  bool ok = true;
  auto ex = [&](int which) {
    int r = exact_sign(which, x1, y1, z1, x2, y2, z2, z0, arena);
    if (r == 2) {
      ok = false;
      r = 0;
    }
    return r;
  };
  if (d.s2 == UNDECIDED) d.s2 = ex(PRED_S2);
  if (d.d1 == UNDECIDED) d.d1 = ex(PRED_D1);
  if (d.d2 == UNDECIDED) d.d2 = ex(PRED_D2);
  if (d.c1 == UNDECIDED) d.c1 = sgn(z0) * ex(PRED_H1);
  if (d.c2 == UNDECIDED) d.c2 = sgn(z0) * ex(PRED_H2);
  return ok;
}

// One pair in EFT mode.  FORCED == false: the decisions come from the floating-point filters
// and are stored in `dec`; if one cannot be decided (and the pair is not certainly without
// intersection), the result carries F_NEEDEXACT and nothing else of it is valid.
// FORCED == true: the decisions are taken from `dec` (all decided), so the result is final.
// Both evaluate the same AccuX arithmetic.
template <bool FORCED>
__host__ __device__ __forceinline__ PairOut eval_eft_core(bool valid, double x1, double y1,
                                                          double z1, double x2, double y2,
                                                          double z2, double z0, Decisions& dec) {
  PairOut o;
  o.count = 0;
  o.r0 = o.r1 = 0;
  o.px0 = o.py0 = o.px1 = o.py1 = 0.0;
  o.flags = 0;
  if (!valid) return o;
  ArcEft A;
  arc_eft(x1, y1, z1, x2, y2, z2, A);
  if (A.flags) {
    o.flags = A.flags;
    return o;
  }
  if (!finite(z0)) {
    o.flags = F_NONFINITE;
    return o;
  }
  const S2Eft S = s2_eft(A, z0);
  if (!FORCED) dec.s2 = S.sign;
  if (dec.s2 < 0) return o;  // certainly no intersection (UNDECIDED is positive)
  if (!FORCED) {
    dec.d1 = d_sign(A, x1, y1);
    dec.d2 = d_sign(A, x2, y2);
    const dd C = two_prod(z0, z0);
    dec.c1 = height_cmp(z0, A.z1, A.n21, A.zz1, x1, y1, C);
    dec.c2 = height_cmp(z0, A.z2, A.n22, A.zz2, x2, y2, C);
    if (dec.s2 == UNDECIDED || dec.d1 == UNDECIDED || dec.d2 == UNDECIDED ||
        dec.c1 == UNDECIDED || dec.c2 == UNDECIDED) {
      o.flags = F_NEEDEXACT;
      return o;
    }
  }
  const bool tangent = dec.s2 == 0;
  o.flags = F_EXISTS | (tangent ? F_TANGENT : 0u) | (FORCED ? F_FALLBACK : 0u);
  o.count = hit_rule(dec.d1, dec.d2, dec.c1, dec.c2, tangent, o.r0, o.r1);
  if (o.count) points_eft(A, z0, S, o);
  return o;
}

// EFT evaluation with exact decisions.  resolve(need, fn) must run fn() on every caller
// with need == true (the GPU runs them one lane at a time per wavefront; the CPU build runs
// them at once); all callers of one wavefront must reach the call.  The fast evaluation
// runs for every pair; a pair with undecided filters gets exact signs for exactly those
// decisions (in the arena) and a forced re-evaluation.
template <class Resolve>
__host__ __device__ __forceinline__ PairOut eval_eft(bool valid, double x1, double y1, double z1,
                                                     double x2, double y2, double z2, double z0,
                                                     double* arena, Resolve&& resolve) {
  Decisions dec = {0, 0, 0, 0, 0};
  PairOut o = eval_eft_core<false>(valid, x1, y1, z1, x2, y2, z2, z0, dec);
  const bool need = (o.flags & F_NEEDEXACT) != 0;
  bool ok = true;
  resolve(need, [&] { ok = resolve_exact(dec, x1, y1, z1, x2, y2, z2, z0, arena); });
  if (need) {
    o = eval_eft_core<true>(valid, x1, y1, z1, x2, y2, z2, z0, dec);
    if (!ok) o.flags |= F_INTERNAL;
  }
  return o;
}

// ====================================================== EFT mode, arc part shared
//
// In a CSR list an arc has several candidate latitudes, and everything of Alg. 8 before z0
// enters (the normal, its norms and the F pairs), as well as the slope signs d1, d2 of the
// containment rule, depends on the arc alone.  ArcDec and ArcPts hold what the z0-dependent
// steps read of an arc (the decisions, then the points); an arc's record is computed once
// (arc_shared, then exact signs for open slope filters) and every candidate of the arc is
// evaluated from it.  The result equals eval_eft on the pair's endpoints bit for bit and
// flag for flag: the same functions run on the same values, and a pair that the per-pair
// evaluation would send to the exact fallback (an open filter on a pair not certainly
// without intersection) takes the forced path here too.

struct ArcDec {
  double S2, s2, S3, s3, side;  // s^2 block (Alg. 8 lines 7-11) and its filter
  double z1, z2, n21, n22;      // height comparisons
  unsigned meta;                // arc flags (bits 0-7) and the ARC_* bits
};

struct ArcPts {
  double Fx, eFx, Fy, eFy;  // Alg. 8 lines 13-16 / 18-21
  double nx, enx, ny, eny;  // the root numerators' s terms
};

enum : unsigned {
  ARC_D1_SHIFT = 8,      // d1 + 1 in bits 8-9
  ARC_D2_SHIFT = 10,     // d2 + 1 in bits 10-11
  ARC_OPEN1 = 1u << 12,  // the d1 filter was open (d1 is the exact sign)
  ARC_OPEN2 = 1u << 13,
  ARC_XOVER = 1u << 14,  // an exact slope sign exceeded the arena (taken as 0)
};

// The shared part of one arc; d1, d2 come back from the filters (UNDECIDED where open).
__host__ __device__ __forceinline__ void arc_shared(double x1, double y1, double z1, double x2,
                                                    double y2, double z2, ArcDec& D, ArcPts& P,
                                                    int& d1, int& d2) {
  ArcEft A;
  arc_eft(x1, y1, z1, x2, y2, z2, A);
  d1 = d2 = 0;
  D.meta = A.flags;
  D.S2 = D.s2 = D.S3 = D.s3 = D.side = D.z1 = D.z2 = D.n21 = D.n22 = 0.0;
  P.Fx = P.eFx = P.Fy = P.eFy = P.nx = P.enx = P.ny = P.eny = 0.0;
  if (A.flags) return;
  D.S2 = A.S2; D.s2 = A.s2; D.S3 = A.S3; D.s3 = A.s3; D.side = A.side;
  D.z1 = A.z1; D.z2 = A.z2; D.n21 = A.n21; D.n22 = A.n22;
  P.Fx = A.Fx; P.eFx = A.eFx; P.Fy = A.Fy; P.eFy = A.eFy;
  P.nx = A.nx; P.enx = A.enx; P.ny = A.ny; P.eny = A.eny;
  d1 = d_sign(A, x1, y1);
  d2 = d_sign(A, x2, y2);
}

// The meta word once both slope signs are final.
__host__ __device__ __forceinline__ unsigned arc_meta(unsigned flags, int d1, int d2, bool open1,
                                                      bool open2, bool xover) {
  return (flags & 0xffu) | ((unsigned)(d1 + 1) << ARC_D1_SHIFT) |
         ((unsigned)(d2 + 1) << ARC_D2_SHIFT) | (open1 ? ARC_OPEN1 : 0u) |
         (open2 ? ARC_OPEN2 : 0u) | (xover ? ARC_XOVER : 0u);
}

__host__ __device__ __forceinline__ int arc_d(unsigned meta, int shift) {
  return (int)((meta >> shift) & 3u) - 1;
}

// Exact slope signs of an arc whose filters left them open (all six endpoint coordinates
// are finite and the arc is not degenerate, or arc_shared would have flagged it).
__host__ __device__ __forceinline__ unsigned arc_resolve(unsigned flags, int d1, int d2,
                                                         double x1, double y1, double z1,
                                                         double x2, double y2, double z2,
                                                         double* arena) {
  const bool o1 = d1 == UNDECIDED, o2 = d2 == UNDECIDED;
  bool xo = false;
  if (o1) {
    d1 = exact_sign(PRED_D1, x1, y1, z1, x2, y2, z2, 0.0, arena);
    if (d1 == 2) { xo = true; d1 = 0; }
  }
  if (o2) {
    d2 = exact_sign(PRED_D2, x1, y1, z1, x2, y2, z2, 0.0, arena);
    if (d2 == 2) { xo = true; d2 = 0; }
  }
  return arc_meta(flags, d1, d2, o1, o2, xo);
}

// Decisions and hit count of one pair from its arc's record (eval_eft_core without the
// points).  FORCED == false: filters (F_NEEDEXACT when one is open); FORCED == true: the
// decisions in `dec`.  S receives the s^2 pair the points use; xy(i) gives endpoint i's
// (x, y) for the second stage of a height comparison.
template <bool FORCED, class XY>
__host__ __device__ __forceinline__ PairOut decide_shared(bool valid, const ArcDec& D, double z0,
                                                          Decisions& dec, S2Eft& S, XY&& xy) {
  PairOut o;
  o.count = 0;
  o.r0 = o.r1 = 0;
  o.px0 = o.py0 = o.px1 = o.py1 = 0.0;
  o.flags = 0;
  S.ss = S.ess = 0.0;
  S.sign = 0;
  if (!valid) return o;
  const unsigned af = D.meta & 0xffu;
  if (af) {
    o.flags = af;
    return o;
  }
  if (!finite(z0)) {
    o.flags = F_NONFINITE;
    return o;
  }
  ArcEft A;
  A.S2 = D.S2; A.s2 = D.s2; A.S3 = D.S3; A.s3 = D.s3; A.side = D.side;
  S = s2_eft(A, z0);
  if (!FORCED) dec.s2 = S.sign;
  if (dec.s2 < 0) return o;
  if (!FORCED) {
    dec.d1 = (D.meta & ARC_OPEN1) ? UNDECIDED : arc_d(D.meta, ARC_D1_SHIFT);
    dec.d2 = (D.meta & ARC_OPEN2) ? UNDECIDED : arc_d(D.meta, ARC_D2_SHIFT);
    const dd C = two_prod(z0, z0);
    dec.c1 = height_cmp_xy(z0, D.z1, D.n21, D.z1 * D.z1, C, [&] { return xy(1); });
    dec.c2 = height_cmp_xy(z0, D.z2, D.n22, D.z2 * D.z2, C, [&] { return xy(2); });
    if (dec.s2 == UNDECIDED || dec.d1 == UNDECIDED || dec.d2 == UNDECIDED ||
        dec.c1 == UNDECIDED || dec.c2 == UNDECIDED) {
      o.flags = F_NEEDEXACT;
      return o;
    }
  }
  const bool tangent = dec.s2 == 0;
  o.flags = F_EXISTS | (tangent ? F_TANGENT : 0u) | (FORCED ? F_FALLBACK : 0u);
  o.count = hit_rule(dec.d1, dec.d2, dec.c1, dec.c2, tangent, o.r0, o.r1);
  return o;
}

// resolve_exact for a pair evaluated from its arc's record: s^2 and the heights from the
// endpoints, the slope signs from the record.
__host__ __device__ __forceinline__ bool resolve_exact_shared(Decisions& d, unsigned meta,
                                                              double x1, double y1, double z1,
                                                              double x2, double y2, double z2,
                                                              double z0, double* arena) {
  bool ok = true;
  auto ex = [&](int which) {
    int r = exact_sign(which, x1, y1, z1, x2, y2, z2, z0, arena);
    if (r == 2) {
      ok = false;
      r = 0;
    }
    return r;
  };
  if (d.s2 == UNDECIDED) d.s2 = ex(PRED_S2);
  if (d.d1 == UNDECIDED) {
    d.d1 = arc_d(meta, ARC_D1_SHIFT);
    if (meta & ARC_XOVER) ok = false;
  }
  if (d.d2 == UNDECIDED) {
    d.d2 = arc_d(meta, ARC_D2_SHIFT);
    if (meta & ARC_XOVER) ok = false;
  }
  if (d.c1 == UNDECIDED) d.c1 = sgn(z0) * ex(PRED_H1);
  if (d.c2 == UNDECIDED) d.c2 = sgn(z0) * ex(PRED_H2);
  return ok;
}


__host__ __device__ __forceinline__ PairOut eval_naive(bool valid, double x1, double y1,
                                                       double z1, double x2, double y2,
                                                       double z2, double z0) {
  PairOut o;
  o.count = 0;
  o.r0 = o.r1 = 0;
  o.px0 = o.py0 = o.px1 = o.py1 = 0.0;
  o.flags = 0;
  if (!valid) return o;
  ArcNaive A;
  arc_naive(x1, y1, z1, x2, y2, z2, A);
  return pair_naive(A, z0);
}

}  // namespace sphint
