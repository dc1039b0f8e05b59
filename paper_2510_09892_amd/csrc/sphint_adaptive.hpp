// Adaptive evaluation of one arc-latitude pair (host and device): the direct binary64
// evaluation of Eq. 2.2 carrying a running bound on its own rounding error, accepted when
// the bound certifies every decision and keeps each point within tol * 2^-53 (max-norm) of
// the exact intersection, and otherwise left to the EFT evaluation (AccuX, Alg. 8, with
// exact decisions).  The paper names such filtered switching as future work (Sec. 9) and
// expects no gain from it for CPU batches, where the branch breaks vectorisation; here the
// pairs that fail the filter are queued and evaluated by a second kernel, so no wavefront
// runs both paths.
//
// Certified decisions are the exact ones of the EFT mode: the slope signs d_i = n_x y_i -
// n_y x_i of the exact normal, the sign of s^2 (a tangency is never certified), and the
// comparisons of z0 with the normalised endpoint heights z_i / |x_i|.  The point is the
// naive mode's Eq. 2.2 arithmetic, operation for operation.
//
// Error bounds (first order, standard model |fl(a op b) - a op b| <= u |fl(a op b)| with
// u = 2^-53, products of two error bounds kept where they can matter): every bound is
// inflated by 2^-10 before it is compared, which covers the dropped second-order terms and
// the rounding of the bound arithmetic itself (both below 100 u relative).
#pragma once
#pragma clang fp contract(off)

#include "sphint_pair.hpp"

namespace sphint {

constexpr double ADAPT_U = 0x1p-53;
constexpr double ADAPT_K = 1.0 + 0x1p-10;

// fl(a - b) of two rounded products p = fl(a b), q = fl(c d) and its error bound:
// |(p - q)(1 + d3) + a b d1 - c d d2 - computed| <= u (|p| + |q| + |p - q|) (1 + u).
struct BoundedDiff {
  double v, e;
};

__host__ __device__ __forceinline__ BoundedDiff bounded_dop(double a, double b, double c,
                                                           double d) {
  const double p = a * b, q = c * d;
  const double v = p - q;
  return {v, ADAPT_U * ((__builtin_fabs(p) + __builtin_fabs(q)) + __builtin_fabs(v))};
}

// Pass 1 of the adaptive evaluation.  Returns true and fills o (the naive point arithmetic
// with certified decisions) when every decision is certified and each point's bound is at
// most tol * 2^-53; returns false otherwise (o is then unspecified).
__host__ __device__ __forceinline__ bool adaptive_pass1(double x1, double y1, double z1,
                                                        double x2, double y2, double z2,
                                                        double z0, double tol, PairOut& o) {
  o.count = 0;
  o.r0 = ROOT_PLUS;
  o.r1 = ROOT_MINUS;
  o.px0 = o.py0 = o.px1 = o.py1 = 0.0;
  o.flags = 0;
  if (!(finite(x1) && finite(y1) && finite(z1) && finite(x2) && finite(y2) && finite(z2) &&
        finite(z0))) {
    o.flags = F_NONFINITE;
    return true;
  }
  const double u = ADAPT_U;
  // normal n = x1 x x2, each component with its bound
  const BoundedDiff nx = bounded_dop(y1, z2, z1, y2);
  const BoundedDiff ny = bounded_dop(z1, x2, x1, z2);
  const BoundedDiff nz = bounded_dop(x1, y2, y1, x2);
  const double ax_ = __builtin_fabs(nx.v), ay_ = __builtin_fabs(ny.v), az_ = __builtin_fabs(nz.v);
  // S2 = nx^2 + ny^2, S3 = S2 + nz^2 (naive order)
  const double S2 = nx.v * nx.v + ny.v * ny.v;
  const double S3 = S2 + nz.v * nz.v;
  const double eS2 = (nx.e * (2.0 * ax_ + nx.e) + ny.e * (2.0 * ay_ + ny.e)) + 2.0 * u * S2;
  const double eS3 = (eS2 + nz.e * (2.0 * az_ + nz.e)) + 2.0 * u * S3;
  if (!(S2 > ADAPT_K * eS2)) return false;  // n_xy (or n) possibly zero: not certified
  // s^2 = S2 - S3 z0^2
  const double Z = z0 * z0;
  const double T = S3 * Z;
  const double s2 = S2 - T;
  const double es2 = ((eS2 + eS3 * Z) + 2.0 * u * T) + u * __builtin_fabs(s2);
  if (s2 < 0.0) {
    if (-s2 > ADAPT_K * es2) return true;  // certainly no intersection
    return false;
  }
  if (!(s2 > 2.0 * ADAPT_K * es2)) return false;  // tangency or too close to decide
  o.flags = F_EXISTS;
  // slope signs at the endpoints
  const double d1a = nx.v * y1, d1b = ny.v * x1, d1 = d1a - d1b;
  const double d2a = nx.v * y2, d2b = ny.v * x2, d2 = d2a - d2b;
  const double ed1 = (__builtin_fabs(y1) * nx.e + __builtin_fabs(x1) * ny.e) +
                     u * ((__builtin_fabs(d1a) + __builtin_fabs(d1b)) + __builtin_fabs(d1));
  const double ed2 = (__builtin_fabs(y2) * nx.e + __builtin_fabs(x2) * ny.e) +
                     u * ((__builtin_fabs(d2a) + __builtin_fabs(d2b)) + __builtin_fabs(d2));
  if (!(__builtin_fabs(d1) > ADAPT_K * ed1) || !(__builtin_fabs(d2) > ADAPT_K * ed2)) return false;
  // heights of the normalised endpoints: |h - z/|x|| <= 4 u |h| (the squared norm within
  // 3 u, its square root within 1.5 u + u, the division u: 3.5 u, taken as 4 u)
  const double h1 = z1 / __builtin_sqrt((x1 * x1 + y1 * y1) + z1 * z1);
  const double h2 = z2 / __builtin_sqrt((x2 * x2 + y2 * y2) + z2 * z2);
  const double g1 = z0 - h1, g2 = z0 - h2;
  if (!(__builtin_fabs(g1) > ADAPT_K * (4.0 * u * __builtin_fabs(h1) + u * __builtin_fabs(g1))) ||
      !(__builtin_fabs(g2) > ADAPT_K * (4.0 * u * __builtin_fabs(h2) + u * __builtin_fabs(g2))))
    return false;
  o.count = hit_rule(sgn(d1), sgn(d2), sgn(g1), sgn(g2), false, o.r0, o.r1);
  if (o.count == 0) return true;
  // points, Eq. 2.2 in the naive mode's operation order
  const double s = __builtin_sqrt(s2);
  // s2 > 2 es2: |s - s*| <= es2 / (sqrt(s2) + sqrt(s2 - es2)) + u s <= 0.6 es2 / s + u s
  const double es = 0.6 * es2 / s + u * s;
  const double nxz = nx.v * nz.v, nyz = ny.v * nz.v;
  const double ax = nxz * z0, bx = s * ny.v, ay = nyz * z0, by = s * nx.v;
  const double az0 = __builtin_fabs(z0);
  const double eax = az0 * ((az_ * nx.e + ax_ * nz.e) + nx.e * nz.e) + 2.0 * u * __builtin_fabs(ax);
  const double eay = az0 * ((az_ * ny.e + ay_ * nz.e) + ny.e * nz.e) + 2.0 * u * __builtin_fabs(ay);
  const double ebx = (ay_ * es + s * ny.e) + es * ny.e + u * __builtin_fabs(bx);
  const double eby = (ax_ * es + s * nx.e) + es * nx.e + u * __builtin_fabs(by);
  const double xp = -((ax + bx) / S2), yp = -((ay - by) / S2);  // upper signs
  const double xm = -((ax - bx) / S2), ym = -((ay + by) / S2);  // lower signs
  // |N/S2 - N*/S2*| <= eN / S2 + (|N| + eN) eS2 / (S2 (S2 - eS2)), plus the division's u |P|
  const double inv = 1.0 / S2, rel = eS2 / (S2 - eS2);
  auto ebound = [&](double num, double enum_, double p) {
    return (enum_ + u * __builtin_fabs(num)) * inv +
           ((__builtin_fabs(num) + enum_) * inv) * rel + u * __builtin_fabs(p);
  };
  const double exn = eax + ebx, eyn = eay + eby;
  const double lim = tol * u;
  const bool plus = o.r0 == ROOT_PLUS || (o.count == 2 && o.r1 == ROOT_PLUS);
  const bool minus = o.r0 == ROOT_MINUS || (o.count == 2 && o.r1 == ROOT_MINUS);
  if (plus && !(ADAPT_K * ebound(ax + bx, exn, xp) <= lim &&
                ADAPT_K * ebound(ay - by, eyn, yp) <= lim))
    return false;
  if (minus && !(ADAPT_K * ebound(ax - bx, exn, xm) <= lim &&
                 ADAPT_K * ebound(ay + by, eyn, ym) <= lim))
    return false;
  o.px0 = o.r0 == ROOT_PLUS ? xp : xm;
  o.py0 = o.r0 == ROOT_PLUS ? yp : ym;
  if (o.count == 2) {
    o.px1 = o.r1 == ROOT_PLUS ? xp : xm;
    o.py1 = o.r1 == ROOT_PLUS ? yp : ym;
  }
  return true;
}

}  // namespace sphint
