// Candidate latitudes of an arc: the step before the intersection path (building the CSR
// arc -> latitude lists that a regridding-shaped call takes).
//
// A latitude z0 can meet the minor arc x1 -> x2 only inside the closed height interval the
// arc covers: between the heights of its normalised endpoints, widened to the top (bottom)
// of its great circle when that point lies inside the arc, which the slope signs at the
// endpoints tell (z rises at x1 and falls at x2: the top is inside; the reverse: the
// bottom).  This is the containment rule of Sec. 2 read as a range query.  The bounds are
// computed in binary64 with a relative error of a few units of 2^-53; the interval is then
// widened by `pad` + 2^-46, which covers that error, so every latitude the arc actually meets
// is a candidate (a few extra candidates at the edges are harmless: the intersection step
// gives them zero hits).  A slope sign the filters cannot certify counts as both signs.
#pragma once
#pragma clang fp contract(off)

#include "sphint_pair.hpp"

namespace sphint {

constexpr double ZRANGE_SLACK = 0x1p-46;

struct ZRange {
  double lo, hi;  // empty when lo > hi
};

__host__ __device__ __forceinline__ ZRange arc_zrange(double x1, double y1, double z1, double x2,
                                                      double y2, double z2, double pad) {
  ArcEft A;
  arc_eft(x1, y1, z1, x2, y2, z2, A);  // degenerate arcs stop early: use A only when flags == 0
  if (A.flags & F_NONFINITE) return {1.0, -1.0};
  const double h1 = z1 / __builtin_sqrt((x1 * x1 + y1 * y1) + z1 * z1);
  const double h2 = z2 / __builtin_sqrt((x2 * x2 + y2 * y2) + z2 * z2);
  double lo = h1 < h2 ? h1 : h2;
  double hi = h1 < h2 ? h2 : h1;
  if (A.flags == 0) {  // S2 > 0: the great circle has a top and a bottom
    const int d1 = d_sign(A, x1, y1), d2 = d_sign(A, x2, y2);
    const bool up1 = d1 != -1, down1 = d1 != 1;  // UNDECIDED allows both
    const bool up2 = d2 != -1, down2 = d2 != 1;
    const double zmax = __builtin_sqrt((A.S2 + A.s2) / (A.S3 + A.s3));
    if (up1 && down2) hi = hi > zmax ? hi : zmax;
    if (down1 && up2) lo = lo < -zmax ? lo : -zmax;
  }
  const double eps = pad + ZRANGE_SLACK;
  return {lo - eps, hi + eps};
}

// First index k of the ascending table z[0..n) with z[k] >= v (n if none).
__host__ __device__ __forceinline__ int32_t lower_index(const double* z, int32_t n, double v) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (z[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// First index k of the ascending table z[0..n) with z[k] > v (n if none).
__host__ __device__ __forceinline__ int32_t upper_index(const double* z, int32_t n, double v) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (z[mid] <= v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The arc's candidates: latitudes [first, first + count) of the ascending table.
__host__ __device__ __forceinline__ void arc_candidates(double x1, double y1, double z1, double x2,
                                                        double y2, double z2, const double* lat_z,
                                                        int32_t n_lat, double pad,
                                                        int32_t& first, int32_t& count) {
  const ZRange r = arc_zrange(x1, y1, z1, x2, y2, z2, pad);
  if (!(r.lo <= r.hi)) {
    first = 0;
    count = 0;
    return;
  }
  first = lower_index(lat_z, n_lat, r.lo);
  const int32_t end = upper_index(lat_z, n_lat, r.hi);
  count = end > first ? end - first : 0;
}

}  // namespace sphint
