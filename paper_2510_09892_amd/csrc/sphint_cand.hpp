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

// Both ends of the candidate range in the ascending table z[0..n), n >= 1: first = the
// first index k with z[k] >= lo, end = the first index k with z[k] > hi (n if none).  The two
// binary searches run in lockstep with a fixed number of halvings (ceil(log2 n)), so their
// loads are independent and every lane of a wavefront takes the same trip count.
__host__ __device__ __forceinline__ void candidate_span(const double* z, int32_t n, double lo,
                                                        double hi, int32_t& first,
                                                        int32_t& end) {
  int32_t b1 = 0, b2 = 0, len = n;  // the answers lie in [b, b + len]
  while (len > 1) {
    const int32_t half = len >> 1;
    b1 = z[b1 + half] < lo ? b1 + half : b1;
    b2 = z[b2 + half] <= hi ? b2 + half : b2;
    len -= half;
  }
  first = b1 + (z[b1] < lo ? 1 : 0);
  end = b2 + (z[b2] <= hi ? 1 : 0);
}

// The arc's candidates: latitudes [first, first + count) of the ascending table.
__host__ __device__ __forceinline__ void arc_candidates(double x1, double y1, double z1, double x2,
                                                        double y2, double z2, const double* lat_z,
                                                        int32_t n_lat, double pad,
                                                        int32_t& first, int32_t& count) {
  const ZRange r = arc_zrange(x1, y1, z1, x2, y2, z2, pad);
  if (!(r.lo <= r.hi) || n_lat <= 0) {
    first = 0;
    count = 0;
    return;
  }
  int32_t end;
  candidate_span(lat_z, n_lat, r.lo, r.hi, first, end);
  count = end > first ? end - first : 0;
}

}  // namespace sphint
