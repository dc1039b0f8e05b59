// Intersection of two great-circle arcs, per pair (host and device).
//
// The next application the paper names for its accurate cross product (Sec. 1, Sec. 9): the
// great circles of A = a1 -> a2 and B = b1 -> b2 meet at +-p, p = (a1 x a2) x (b1 x b2)
// normalised ("three cross products and a normalisation").  With n_A = a1 x a2 and
// n_B = b1 x b2, the Binet-Cauchy identity turns "q = +-p lies on both closed minor arcs"
// into four orientation signs,
//     sa1 = sign(n_B . a1), sa2 = sign(n_B . a2), sb1 = sign(n_A . b1), sb2 = sign(n_A . b2):
// +p is the point iff sa1 >= 0 >= sa2 and sb2 >= 0 >= sb1, -p iff all four are reversed, and
// sa1 = sa2 = 0 means both arcs lie on one great circle (COPLANAR, no isolated point).
//
// EFT mode: n_A, n_B by AccuDOP (Alg. 4) renormalised by TwoSum; the signs certified by two
// filter stages and decided exactly (exact_orient) when both fail; each component of
// n_A x n_B by AccuDOP on the leading parts plus the trailing parts' first-order products;
// |X|^2 by SumOfSquares (Alg. 5); one binary64 square root and three divisions.  Naive mode: plain
// binary64 throughout (signs included).
#pragma once
#pragma clang fp contract(off)

#include "sphint_pair.hpp"

namespace sphint {

enum : unsigned {
  AA_HIT = 1u,
  AA_DEGEN = 4u,     // an arc with a zero normal (coincident or antipodal endpoints)
  AA_COPLANAR = 8u,  // both arcs on one great circle
  AA_NONFINITE = 16u,
  AA_EXACT = 32u,     // diagnostic: an exact orientation decided this pair
  AA_INTERNAL = 64u,  // an exact evaluation exceeded its arena
};

struct AAOut {
  double px, py, pz;
  int count;
  unsigned flags;
};

// n = u x v as renormalised AccuDOP pairs, with the magnitudes m_i = |p1_i| + |p2_i| of the
// two products (the pair is within 3.01 u^2 m_i of the exact component); zero is exact.
struct NormalPairs {
  double n[3], e[3], m[3];
  bool zero;
};

__host__ __device__ __forceinline__ NormalPairs normal_pairs(double ux, double uy, double uz,
                                                             double vx, double vy, double vz) {
  NormalPairs r;
  const dop3 c[3] = {accu_dop(uy, vz, uz, vy), accu_dop(uz, vx, ux, vz), accu_dop(ux, vy, uy, vx)};
  bool zero = true;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    zero = zero && c[i].zero;
    r.n[i] = c[i].hi;
    r.e[i] = c[i].lo;
    r.m[i] = c[i].mag;
  }
  r.zero = zero;
  return r;
}

// sign(n . w) for the exact normal n of a NormalPairs, or UNDECIDED.
// Stage 1 (binary64 over the leading parts): error <= 4.02 u sum|n_i w_i| + 3.01 u^2 sum m_i
// |w_i|; threshold 2^-49 and 2^-96 times those sums.  Stage 2 (CompDotC over the six products
// of both parts, Alg. 1): error <= u |w| + 37 u^2 sum|terms| + 3.01 u^2 sum m_i |w_i|;
// threshold 2^-96 = 128 u^2 times the sum of both magnitudes (a margin above 3).
__host__ __device__ __forceinline__ int orient_sign(const NormalPairs& N, double wx, double wy,
                                                    double wz) {
  const double t0 = N.n[0] * wx, t1 = N.n[1] * wy, t2 = N.n[2] * wz;
  const double w0 = (t0 + t1) + t2;
  const double mag = __builtin_fabs(t0) + __builtin_fabs(t1) + __builtin_fabs(t2);
  const double side = N.m[0] * __builtin_fabs(wx) + N.m[1] * __builtin_fabs(wy) +
                      N.m[2] * __builtin_fabs(wz);
  if (__builtin_fabs(w0) > 0x1p-49 * mag + 0x1p-96 * side) return sgn(w0);
  dd p = two_prod(N.n[0], wx);
  double ph = p.hi, s = p.lo;
  const double xs[5] = {N.n[1], N.n[2], N.e[0], N.e[1], N.e[2]};
  const double ws[5] = {wy, wz, wx, wy, wz};
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const dd h = two_prod(xs[i], ws[i]);
    const dd q = two_sum(ph, h.hi);
    ph = q.hi;
    s = s + (q.lo + h.lo);
  }
  const double w = ph + s;
  if (__builtin_fabs(w) > 0x1p-96 * (mag + side)) return sgn(w);
  return UNDECIDED;
}

// The decision rule on four signs; returns the point's sign (+1, -1) or 0, and flags.
__host__ __device__ __forceinline__ int aa_rule(int sa1, int sa2, int sb1, int sb2,
                                                unsigned& flags) {
  if (sa1 == 0 && sa2 == 0) {
    flags = AA_COPLANAR;
    return 0;
  }
  if (sa1 >= 0 && sa2 <= 0 && sb2 >= 0 && sb1 <= 0) {
    flags = AA_HIT;
    return 1;
  }
  if (sa1 <= 0 && sa2 >= 0 && sb2 <= 0 && sb1 >= 0) {
    flags = AA_HIT;
    return -1;
  }
  flags = 0;
  return 0;
}

__host__ __device__ __forceinline__ bool finite12(double a, double b, double c, double d, double e,
                                                  double f, double g, double h, double i,
                                                  double j, double k, double l) {
  return finite(a) && finite(b) && finite(c) && finite(d) && finite(e) && finite(f) &&
         finite(g) && finite(h) && finite(i) && finite(j) && finite(k) && finite(l);
}

__host__ __device__ __forceinline__ bool same3(const double* u, const double* v) {
  return u[0] == v[0] && u[1] == v[1] && u[2] == v[2];
}

// EFT evaluation of one pair.  resolve(need, fn) as for eval_eft: fn() computes the exact
// signs of the open decisions in the arena.
template <class Resolve>
__host__ __device__ __forceinline__ AAOut eval_aa_eft(bool valid, const double* a1,
                                                      const double* a2, const double* b1,
                                                      const double* b2, double* arena,
                                                      Resolve&& resolve) {
  AAOut o;
  o.px = o.py = o.pz = 0.0;
  o.count = 0;
  o.flags = 0;
  const bool fin = valid && finite12(a1[0], a1[1], a1[2], a2[0], a2[1], a2[2], b1[0], b1[1],
                                     b1[2], b2[0], b2[1], b2[2]);
  const NormalPairs A = normal_pairs(a1[0], a1[1], a1[2], a2[0], a2[1], a2[2]);
  const NormalPairs B = normal_pairs(b1[0], b1[1], b1[2], b2[0], b2[1], b2[2]);
  int sa1 = orient_sign(B, a1[0], a1[1], a1[2]);
  int sa2 = orient_sign(B, a2[0], a2[1], a2[2]);
  int sb1 = orient_sign(A, b1[0], b1[1], b1[2]);
  int sb2 = orient_sign(A, b2[0], b2[1], b2[2]);
  // A shared endpoint (a mesh vertex) makes two orientations determinants with a repeated
  // row, exactly zero: decided here without expansion arithmetic.
  const bool e11 = same3(a1, b1), e12 = same3(a1, b2), e21 = same3(a2, b1), e22 = same3(a2, b2);
  if (sa1 == UNDECIDED && (e11 || e12)) sa1 = 0;
  if (sa2 == UNDECIDED && (e21 || e22)) sa2 = 0;
  if (sb1 == UNDECIDED && (e11 || e21)) sb1 = 0;
  if (sb2 == UNDECIDED && (e12 || e22)) sb2 = 0;
  const bool live = fin && !A.zero && !B.zero;
  const bool need = live && (sa1 == UNDECIDED || sa2 == UNDECIDED || sb1 == UNDECIDED ||
                             sb2 == UNDECIDED);
  bool ok = true;
  resolve(need, [&] {
    auto ex = [&](const double* u, const double* v, const double* w) {
      int r = exact_orient(u[0], u[1], u[2], v[0], v[1], v[2], w[0], w[1], w[2], arena);
      if (r == 2) {
        ok = false;
        r = 0;
      }
      return r;
    };
    if (sa1 == UNDECIDED) sa1 = ex(a1, b1, b2);  // n_B . a1 = a1 . (b1 x b2)
    if (sa2 == UNDECIDED) sa2 = ex(a2, b1, b2);
    if (sb1 == UNDECIDED) sb1 = ex(b1, a1, a2);  // n_A . b1 = b1 . (a1 x a2)
    if (sb2 == UNDECIDED) sb2 = ex(b2, a1, a2);
  });
  if (!valid) return o;
  if (!fin) {
    o.flags = AA_NONFINITE;
    return o;
  }
  if (A.zero || B.zero) {
    o.flags = AA_DEGEN;
    return o;
  }
  unsigned fl;
  const int sg = aa_rule(sa1, sa2, sb1, sb2, fl);
  o.flags = fl | (need ? AA_EXACT : 0u) | (ok ? 0u : AA_INTERNAL);
  if (sg == 0) return o;
  o.count = 1;
  // X = n_A x n_B: component c = nA_i nB_j - nA_j nB_i, (i, j) = (1,2), (2,0), (0,1), by
  // AccuDOP on the leading parts with the trailing parts' first-order products (one
  // multiplication, three FMAs) added to its error term; the second-order products are
  // below u^2 of the result.
  double X[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int i = (c + 1) % 3, j = (c + 2) % 3;
    const dd p1 = two_prod(A.n[i], B.n[j]), p2 = two_prod(A.n[j], B.n[i]);
    const dd d = two_sum(p1.hi, -p2.hi);
    const double err = d.lo + (p1.lo - p2.lo);
    double t = A.n[i] * B.e[j];
    t = __builtin_fma(A.e[i], B.n[j], t);
    t = __builtin_fma(-A.n[j], B.e[i], t);
    t = __builtin_fma(-A.e[j], B.n[i], t);
    X[c] = d.hi + (err + t);
  }
  dd S = two_prod(X[0], X[0]);  // SumOfSquares (Alg. 5)
  S = sum_non_neg(S, two_prod(X[1], X[1]));
  S = sum_non_neg(S, two_prod(X[2], X[2]));
  const double r = __builtin_sqrt(S.hi);
  o.px = (sg * X[0]) / r;
  o.py = (sg * X[1]) / r;
  o.pz = (sg * X[2]) / r;
  return o;
}

__host__ __device__ __forceinline__ AAOut eval_aa_naive(bool valid, const double* a1,
                                                        const double* a2, const double* b1,
                                                        const double* b2) {
  AAOut o;
  o.px = o.py = o.pz = 0.0;
  o.count = 0;
  o.flags = 0;
  if (!valid) return o;
  if (!finite12(a1[0], a1[1], a1[2], a2[0], a2[1], a2[2], b1[0], b1[1], b1[2], b2[0], b2[1],
                b2[2])) {
    o.flags = AA_NONFINITE;
    return o;
  }
  const double na[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                        a1[0] * a2[1] - a1[1] * a2[0]};
  const double nb[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2],
                        b1[0] * b2[1] - b1[1] * b2[0]};
  if ((na[0] == 0.0 && na[1] == 0.0 && na[2] == 0.0) ||
      (nb[0] == 0.0 && nb[1] == 0.0 && nb[2] == 0.0)) {
    o.flags = AA_DEGEN;
    return o;
  }
  auto dot = [](const double* u, const double* v) { return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]; };
  unsigned fl;
  const int sg = aa_rule(sgn(dot(nb, a1)), sgn(dot(nb, a2)), sgn(dot(na, b1)), sgn(dot(na, b2)), fl);
  o.flags = fl;
  if (sg == 0) return o;
  o.count = 1;
  const double X[3] = {na[1] * nb[2] - na[2] * nb[1], na[2] * nb[0] - na[0] * nb[2],
                       na[0] * nb[1] - na[1] * nb[0]};
  const double r = __builtin_sqrt((X[0] * X[0] + X[1] * X[1]) + X[2] * X[2]);
  o.px = (sg * X[0]) / r;
  o.py = (sg * X[1]) / r;
  o.pz = (sg * X[2]) / r;
  return o;
}

}  // namespace sphint
