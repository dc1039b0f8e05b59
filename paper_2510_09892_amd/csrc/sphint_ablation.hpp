// Alternative binary64 formulas for the arc-latitude points (host and device), for accuracy
// comparisons with the method's AccuX: the paper's Eq. (2.2) evaluated directly, Eq. (2.1)
// on the unit normal, Eq. (7.1) (Eq. (2.1) with the denominator 1 - n^z^2, which cancels
// for great circles near the equator) and Eq. (2.2) with Kahan's DiffOfProd (Alg. 3) for the
// normal (Sec. S2).  Each returns both intersection points of the great circle with the
// latitude circle, upper signs (PLUS) first; no containment test.  Operation order:
//
//   |n|^2 = (nx nx + ny ny) + nz nz,  r = sqrt(|n|^2),  n^ = (nx / r, ny / r, nz / r)
//   Eq. (2.1): T = n^x n^x + n^y n^y,   Eq. (7.1): T = 1 - n^z n^z,   s2 = T - z0 z0
//   Eq. (2.2): T = S2 = nx nx + ny ny,  s2 = S2 - (S2 + nz nz) (z0 z0)
//   ax = (a_x a_z) z0, bx = s a_y, ay = (a_y a_z) z0, by = s a_x   (a = n^ or n)
//   P+ = (-((ax + bx) / T), -((ay - by) / T)),  P- = (-((ax - bx) / T), -((ay + by) / T))
//
// A pair whose denominator is not positive or whose s2 is negative gets no points.
#pragma once
#pragma clang fp contract(off)

#include "sphint_pair.hpp"

namespace sphint {

enum : int { ABL_EQ22 = 0, ABL_EQ21 = 1, ABL_EQ71 = 2, ABL_KAHAN = 3, ABL_ACCUX = 4 };

struct CirclePoints {
  double xp, yp, xm, ym;
  bool ok;
};

// a*d - b*c by Kahan's algorithm (Alg. 3 as printed).
__host__ __device__ __forceinline__ double kahan_dop(double a, double d, double b, double c) {
  const double bc = b * c;
  const double err = __builtin_fma(-b, c, bc);
  return __builtin_fma(a, d, -bc) + err;
}

template <int VARIANT>
__host__ __device__ __forceinline__ CirclePoints circle_points(double x1, double y1, double z1,
                                                               double x2, double y2, double z2,
                                                               double z0) {
  CirclePoints o{0.0, 0.0, 0.0, 0.0, false};
  double nx, ny, nz;
  if constexpr (VARIANT == ABL_KAHAN) {
    nx = kahan_dop(y1, z2, z1, y2);
    ny = kahan_dop(z1, x2, x1, z2);
    nz = kahan_dop(x1, y2, y1, x2);
  } else {
    nx = y1 * z2 - z1 * y2;
    ny = z1 * x2 - x1 * z2;
    nz = x1 * y2 - y1 * x2;
  }
  double T, s2, a0, a1, a2;
  if constexpr (VARIANT == ABL_EQ21 || VARIANT == ABL_EQ71) {
    const double r = __builtin_sqrt((nx * nx + ny * ny) + nz * nz);
    if (!(r > 0.0)) return o;
    a0 = nx / r;
    a1 = ny / r;
    a2 = nz / r;
    T = VARIANT == ABL_EQ21 ? a0 * a0 + a1 * a1 : 1.0 - a2 * a2;
    s2 = T - z0 * z0;
  } else {
    a0 = nx;
    a1 = ny;
    a2 = nz;
    T = nx * nx + ny * ny;
    s2 = T - (T + nz * nz) * (z0 * z0);
  }
  if (!(T > 0.0) || !(s2 >= 0.0)) return o;
  const double s = __builtin_sqrt(s2);
  const double ax = (a0 * a2) * z0, bx = s * a1, ay = (a1 * a2) * z0, by = s * a0;
  o.xp = -((ax + bx) / T);
  o.yp = -((ay - by) / T);
  o.xm = -((ax - bx) / T);
  o.ym = -((ay + by) / T);
  o.ok = true;
  return o;
}

}  // namespace sphint
