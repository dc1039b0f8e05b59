// CPU build of the per-pair arithmetic, for tests only (never a product path: the library's
// entry points run on the GPU and nothing in the package loads this object).  It compiles
// the same header the kernels use, so the CPU tests exercise the exact operation sequence
// of the GPU evaluation; undecided predicates are resolved immediately instead of one lane
// at a time.
#include "sphint_ablation.hpp"
#include "sphint_adaptive.hpp"
#include "sphint_arcarc.hpp"
#include "sphint_cand.hpp"
#include "sphint_pair.hpp"

extern "C" int sphint_hostcheck_eval(int mode, int64_t n, const double* x1, const double* y1,
                                     const double* z1, const double* x2, const double* y2,
                                     const double* z2, const double* z0, int32_t* count,
                                     int32_t* flags, int32_t* r0, int32_t* r1, double* px0,
                                     double* py0, double* px1, double* py1) {
  using namespace sphint;
  static thread_local double arena[xp::ARENA];
  for (int64_t i = 0; i < n; ++i) {
    PairOut o;
    if (mode == 1)
      o = eval_eft(true, x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i], arena,
                   [](bool need, auto&& fn) {
                     if (need) fn();
                   });
    else
      o = eval_naive(true, x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i]);
    count[i] = o.count;
    flags[i] = (int32_t)o.flags;
    r0[i] = o.r0;
    r1[i] = o.r1;
    px0[i] = o.px0;
    py0[i] = o.py0;
    px1[i] = o.px1;
    py1[i] = o.py1;
  }
  return 0;
}

// Exact sign of one predicate (sphint::PRED_*), for tests of the expansion arithmetic.
extern "C" int sphint_hostcheck_exact_sign(int which, double x1, double y1, double z1, double x2,
                                           double y2, double z2, double z0) {
  static thread_local double arena[sphint::xp::ARENA];
  return sphint::exact_sign(which, x1, y1, z1, x2, y2, z2, z0, arena);
}

// Candidate latitudes of each arc (first index and count in the ascending table lat_z).
extern "C" int sphint_hostcheck_candidates(int64_t n, const double* x1, const double* y1,
                                           const double* z1, const double* x2, const double* y2,
                                           const double* z2, const double* lat_z, int32_t n_lat,
                                           double pad, int32_t* first, int32_t* count) {
  for (int64_t i = 0; i < n; ++i)
    sphint::arc_candidates(x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], lat_z, n_lat, pad, first[i],
                           count[i]);
  return 0;
}

// Arc x arc intersections, direct pairs: a = (ax1..az2)[i], b = (bx1..bz2)[i].
extern "C" int sphint_hostcheck_arcarc(int mode, int64_t n, const double* const* a,
                                       const double* const* b, double* px, double* py,
                                       double* pz, int32_t* count, int32_t* flags) {
  using namespace sphint;
  static thread_local double arena[xp::ARENA];
  for (int64_t i = 0; i < n; ++i) {
    const double a1[3] = {a[0][i], a[1][i], a[2][i]}, a2[3] = {a[3][i], a[4][i], a[5][i]};
    const double b1[3] = {b[0][i], b[1][i], b[2][i]}, b2[3] = {b[3][i], b[4][i], b[5][i]};
    AAOut o;
    if (mode == 1)
      o = eval_aa_eft(true, a1, a2, b1, b2, arena, [](bool need, auto&& fn) {
        if (need) fn();
      });
    else
      o = eval_aa_naive(true, a1, a2, b1, b2);
    px[i] = o.px;
    py[i] = o.py;
    pz[i] = o.pz;
    count[i] = o.count;
    flags[i] = (int32_t)o.flags;
  }
  return 0;
}

// Exact sign of u . (v x w).
extern "C" int sphint_hostcheck_orient(const double* u, const double* v, const double* w) {
  static thread_local double arena[sphint::xp::ARENA];
  return sphint::exact_orient(u[0], u[1], u[2], v[0], v[1], v[2], w[0], w[1], w[2], arena);
}

// The adaptive evaluation: pass 1, and the EFT evaluation for the pairs it does not accept
// (cert[i] = 1 when pass 1 accepted pair i).
extern "C" int sphint_hostcheck_adaptive(int64_t n, const double* x1, const double* y1,
                                         const double* z1, const double* x2, const double* y2,
                                         const double* z2, const double* z0, double tol,
                                         int32_t* count, int32_t* flags, int32_t* r0,
                                         int32_t* r1, double* px0, double* py0, double* px1,
                                         double* py1, int32_t* cert) {
  using namespace sphint;
  static thread_local double arena[xp::ARENA];
  for (int64_t i = 0; i < n; ++i) {
    PairOut o;
    const bool c = adaptive_pass1(x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i], tol, o);
    if (!c)
      o = eval_eft(true, x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i], arena,
                   [](bool need, auto&& fn) {
                     if (need) fn();
                   });
    count[i] = o.count;
    flags[i] = (int32_t)(o.flags & 127u);
    r0[i] = o.count ? o.r0 : 0;
    r1[i] = o.count == 2 ? o.r1 : 0;
    px0[i] = o.count ? o.px0 : 0.0;
    py0[i] = o.count ? o.py0 : 0.0;
    px1[i] = o.count == 2 ? o.px1 : 0.0;
    py1[i] = o.count == 2 ? o.py1 : 0.0;
    cert[i] = c;
  }
  return 0;
}

// Both circle points of each pair by one alternative formula (SPHINT_FORMULA_EQ22..KAHAN).
extern "C" int sphint_hostcheck_circle(int formula, int64_t n, const double* x1, const double* y1,
                                       const double* z1, const double* x2, const double* y2,
                                       const double* z2, const double* z0, double* ox, double* oy,
                                       int32_t* ok) {
  using namespace sphint;
  for (int64_t i = 0; i < n; ++i) {
    CirclePoints c;
    switch (formula) {
      case ABL_EQ22: c = circle_points<ABL_EQ22>(x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i]); break;
      case ABL_EQ21: c = circle_points<ABL_EQ21>(x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i]); break;
      case ABL_EQ71: c = circle_points<ABL_EQ71>(x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i]); break;
      default: c = circle_points<ABL_KAHAN>(x1[i], y1[i], z1[i], x2[i], y2[i], z2[i], z0[i]); break;
    }
    ox[2 * i] = c.xp;
    oy[2 * i] = c.yp;
    ox[2 * i + 1] = c.xm;
    oy[2 * i + 1] = c.ym;
    ok[i] = c.ok;
  }
  return 0;
}
