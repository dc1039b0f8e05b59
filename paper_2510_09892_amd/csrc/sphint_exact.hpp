// Exact sign predicates by floating-point expansion arithmetic (Shewchuk 1997, "Adaptive
// precision floating-point arithmetic and fast robust geometric predicates", cited by the
// paper in Sec. 1.1 for adaptive exact predicates).
//
// The paper's Sec. 2 says candidate points must still be checked to lie between x1 and x2
// and that two points exist iff |n_xy|^2 > |n|^2 z0^2.  Those decisions are signs of
// polynomials in the binary64 inputs.  The hit kernels decide them with floating-point
// filters; the rare inputs no filter can certify (exact ties, or values within ~2^-90 of
// zero relative to their terms) come here, where each polynomial is evaluated exactly as a
// nonoverlapping expansion (a sum of doubles in increasing magnitude) and its sign is the
// sign of its largest component.
//
// This code runs one lane at a time per wavefront on a per-wavefront LDS arena (see
// resolve_exact in the kernels), so it holds no private arrays and needs no scratch.
// Valid without overflow or underflow, i.e. for nonzero input magnitudes roughly within
// [2^-150, 2^150].
#pragma once
#pragma clang fp contract(off)

#include "sphint_eft.hpp"

namespace sphint {
namespace xp {

constexpr int CAP = 64;        // doubles per arena buffer
constexpr int NBUF = 8;        // buffers per arena
constexpr int ARENA = CAP * NBUF;

// h = e + b (Grow-Expansion with zero elimination); h may alias e.
__host__ __device__ inline int grow(int elen, const double* e, double b, double* h) {
  double Q = b;
  int k = 0;
  for (int i = 0; i < elen; ++i) {
    dd t = two_sum(Q, e[i]);
    Q = t.hi;
    if (t.lo != 0.0) h[k++] = t.lo;
  }
  if (Q != 0.0 || k == 0) h[k++] = Q;
  return k;
}

// e += f, in place, by repeated Grow-Expansion (nonoverlapping output for nonoverlapping
// inputs).  Returns the new length, or -1 if it could exceed CAP.
__host__ __device__ inline int add_into(int elen, double* e, int flen, const double* f) {
  if (elen + flen > CAP) return -1;
  for (int j = 0; j < flen; ++j) elen = grow(elen, e, f[j], e);
  return elen;
}

// h = b * e (Scale-Expansion with zero elimination); h must not alias e.
__host__ __device__ inline int scale(int elen, const double* e, double b, double* h) {
  if (2 * elen > CAP) return -1;
  dd p = two_prod(e[0], b);
  int k = 0;
  if (p.lo != 0.0) h[k++] = p.lo;
  double Q = p.hi;
  for (int i = 1; i < elen; ++i) {
    dd t = two_prod(e[i], b);
    dd s = two_sum(Q, t.lo);
    if (s.lo != 0.0) h[k++] = s.lo;
    dd f = fast_two_sum(t.hi, s.hi);
    Q = f.hi;
    if (f.lo != 0.0) h[k++] = f.lo;
  }
  if (Q != 0.0 || k == 0) h[k++] = Q;
  return k;
}

// Compress (Shewchuk's two sweeps): an equal, nonadjacent expansion, usually much shorter;
// in place.
__host__ __device__ inline int compress(int elen, double* e) {
  if (elen <= 1) return elen;
  int bottom = elen - 1;
  double Q = e[bottom];
  for (int i = elen - 2; i >= 0; --i) {
    dd t = fast_two_sum(Q, e[i]);
    if (t.lo != 0.0) {
      e[bottom--] = t.hi;
      Q = t.lo;
    } else {
      Q = t.hi;
    }
  }
  e[bottom] = Q;
  int top = 0;
  for (int i = bottom + 1; i < elen; ++i) {
    dd t = fast_two_sum(e[i], Q);
    if (t.lo != 0.0) e[top++] = t.lo;
    Q = t.hi;
  }
  e[top++] = Q;
  return top;
}

__host__ __device__ inline int sign_of(int elen, const double* e) { return elen > 0 ? sgn(e[elen - 1]) : 0; }

__host__ __device__ inline void negate(int elen, double* e) {
  for (int i = 0; i < elen; ++i) e[i] = -e[i];
}

// h = a * b for expansions (sum of Scale-Expansions), compressed; tmp is scratch.
__host__ __device__ inline int mul(int alen, const double* a, int blen, const double* b, double* h,
                          double* tmp) {
  if (alen < 0 || blen < 0) return -1;
  int hlen = scale(alen, a, b[0], h);
  if (hlen < 0) return -1;
  hlen = compress(hlen, h);
  for (int j = 1; j < blen; ++j) {
    int tlen = scale(alen, a, b[j], tmp);
    if (tlen < 0) return -1;
    hlen = add_into(hlen, h, tlen, tmp);
    if (hlen < 0) return -1;
    hlen = compress(hlen, h);
  }
  return hlen;
}

// Expansion of a*b - c*d from the four exact parts of two TwoProducts.
__host__ __device__ inline int diff_of_products(double a, double b, double c, double d, double* h) {
  dd p1 = two_prod(a, b);
  dd p2 = two_prod(c, d);
  int k = grow(0, h, p1.lo, h);
  k = grow(k, h, p1.hi, h);
  k = grow(k, h, -p2.lo, h);
  k = grow(k, h, -p2.hi, h);
  return compress(k, h);
}

// Expansion of x^2 + y^2 + z^2 (exact).
__host__ __device__ inline int sum_sq3(double x, double y, double z, double* h) {
  dd a = two_prod(x, x), b = two_prod(y, y), c = two_prod(z, z);
  int k = grow(0, h, a.lo, h);
  k = grow(k, h, a.hi, h);
  k = grow(k, h, b.lo, h);
  k = grow(k, h, b.hi, h);
  k = grow(k, h, c.lo, h);
  k = grow(k, h, c.hi, h);
  return compress(k, h);
}

}  // namespace xp

// Exact sign of the determinant u . (v x w) (an orientation of three vectors from the
// origin), in the caller's arena (xp::ARENA doubles).  Returns 2 if an expansion would
// overflow the arena (never for inputs in the documented range).
__host__ __device__ __noinline__ inline int exact_orient(double ux, double uy, double uz,
                                                          double vx, double vy, double vz,
                                                          double wx, double wy, double wz,
                                                          double* arena) {
  using namespace xp;
  double* B0 = arena;
  double* B1 = arena + CAP;
  double* B2 = arena + 2 * CAP;
  double* B3 = arena + 3 * CAP;
  int l0 = diff_of_products(vy, wz, vz, wy, B0);  // (v x w)_x
  int t = scale(l0, B0, ux, B1);
  if (t < 0) return 2;
  int l1 = diff_of_products(vz, wx, vx, wz, B0);  // (v x w)_y
  int t2 = scale(l1, B0, uy, B2);
  if (t2 < 0) return 2;
  t = add_into(t, B1, t2, B2);
  if (t < 0) return 2;
  int l2 = diff_of_products(vx, wy, vy, wx, B0);  // (v x w)_z
  t2 = scale(l2, B0, uz, B3);
  if (t2 < 0) return 2;
  t = add_into(t, B1, t2, B3);
  if (t < 0) return 2;
  return sign_of(compress(t, B1), B1);
}

// Which predicate exact_sign evaluates.
enum : int {
  PRED_S2 = 0,  // sign(|n_xy|^2 - |n|^2 z0^2)              (Sec. 2 existence test)
  PRED_D1 = 1,  // sign(n_x y1 - n_y x1) = sign(dz/dt at x1)  (direction of travel)
  PRED_D2 = 2,  // sign(n_x y2 - n_y x2)
  PRED_H1 = 3,  // sign(z0^2 |x1|^2 - z1^2)                    (|z0| vs |z1|/|x1|)
  PRED_H2 = 4,  // sign(z0^2 |x2|^2 - z2^2)
};

// Exact sign of predicate `which` for the inputs (x1, y1, z1, x2, y2, z2, z0), computed in
// the caller's LDS arena (xp::ARENA doubles).  Returns 2 if an expansion would overflow
// the arena (never for inputs in the documented range; callers flag it as an error).
__host__ __device__ __noinline__ inline int exact_sign(int which, double x1, double y1, double z1, double x2,
                                       double y2, double z2, double z0, double* arena) {
  using namespace xp;
  double* B0 = arena;
  double* B1 = arena + CAP;
  double* B2 = arena + 2 * CAP;
  double* B3 = arena + 3 * CAP;
  double* B4 = arena + 4 * CAP;
  double* B5 = arena + 5 * CAP;
  double* B6 = arena + 6 * CAP;
  double* T = arena + 7 * CAP;
  if (which == PRED_D1 || which == PRED_D2) {
    const double xa = which == PRED_D1 ? x1 : x2;
    const double ya = which == PRED_D1 ? y1 : y2;
    int nxl = diff_of_products(y1, z2, z1, y2, B0);  // n_x
    int nyl = diff_of_products(z1, x2, x1, z2, B1);  // n_y
    int al = scale(nxl, B0, ya, B2);
    int bl = scale(nyl, B1, -xa, B3);
    if (al < 0 || bl < 0) return 2;
    al = add_into(al, B2, bl, B3);
    if (al < 0) return 2;
    return sign_of(compress(al, B2), B2);
  }
  if (which == PRED_H1 || which == PRED_H2) {
    const double xa = which == PRED_H1 ? x1 : x2;
    const double ya = which == PRED_H1 ? y1 : y2;
    const double za = which == PRED_H1 ? z1 : z2;
    int nl = sum_sq3(xa, ya, za, B0);          // |x|^2
    int czl = grow(0, B2, two_prod(z0, z0).lo, B2);
    czl = grow(czl, B2, z0 * z0, B2);           // z0^2 = C + eC exactly
    int pl = mul(nl, B0, czl, B2, B1, T);      // z0^2 |x|^2
    if (pl < 0 || pl + 2 > CAP) return 2;
    dd zz = two_prod(za, za);
    pl = grow(pl, B1, -zz.lo, B1);
    pl = grow(pl, B1, -zz.hi, B1);
    if (pl > CAP) return 2;
    return sign_of(compress(pl, B1), B1);
  }
  // PRED_S2: |n_xy|^2 (1 - z0^2) - n_z^2 z0^2, i.e. S2 - S3 z0^2 with the exact normal.
  int nxl = diff_of_products(y1, z2, z1, y2, B0);
  int nyl = diff_of_products(z1, x2, x1, z2, B1);
  int nzl = diff_of_products(x1, y2, y1, x2, B2);
  int s2l = mul(nxl, B0, nxl, B0, B3, T);        // n_x^2
  int tl = mul(nyl, B1, nyl, B1, B4, T);         // n_y^2
  if (s2l < 0 || tl < 0) return 2;
  s2l = add_into(s2l, B3, tl, B4);               // S2
  if (s2l < 0) return 2;
  s2l = compress(s2l, B3);
  int zl = mul(nzl, B2, nzl, B2, B4, T);         // n_z^2
  if (zl < 0) return 2;
  for (int i = 0; i < s2l; ++i) B5[i] = B3[i];
  int s3l = add_into(s2l, B5, zl, B4);           // S3
  if (s3l < 0) return 2;
  s3l = compress(s3l, B5);
  int czl = grow(0, B4, two_prod(z0, z0).lo, B4);
  czl = grow(czl, B4, z0 * z0, B4);              // z0^2 = C + eC exactly
  int dl = mul(s3l, B5, czl, B4, B6, T);         // S3 z0^2
  if (dl < 0) return 2;
  negate(dl, B6);
  s2l = add_into(s2l, B3, dl, B6);               // S2 - S3 z0^2
  if (s2l < 0) return 2;
  return sign_of(compress(s2l, B3), B3);
}

}  // namespace sphint
