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

// CSR lists in EFT mode with the arc part shared, as the batched kernels' shared path
// evaluates them: each arc's record once (exact slope signs where the filters are open),
// then every candidate from its arc's record; the points run for every pair and are kept
// where there are hits.  lat_idx entries outside [0, n_lat) give z0 = NaN.  *open_arcs
// receives the number of arcs whose slope filters left a sign open.
extern "C" int sphint_hostcheck_eval_shared(int64_t n_arcs, const double* x1, const double* y1,
                                            const double* z1, const double* x2,
                                            const double* y2, const double* z2,
                                            const double* lat_z, int64_t n_lat,
                                            const int64_t* off, const int32_t* idx,
                                            int32_t* count, int32_t* flags, int32_t* r0,
                                            int32_t* r1, double* px0, double* py0, double* px1,
                                            double* py1, int64_t* open_arcs) {
  using namespace sphint;
  static thread_local double arena[xp::ARENA];
  int64_t opened = 0;
  for (int64_t a = 0; a < n_arcs; ++a) {
    ArcDec D;
    ArcPts P;
    int d1, d2;
    arc_shared(x1[a], y1[a], z1[a], x2[a], y2[a], z2[a], D, P, d1, d2);
    if (d1 == UNDECIDED || d2 == UNDECIDED) {
      ++opened;
      D.meta = arc_resolve(D.meta, d1, d2, x1[a], y1[a], z1[a], x2[a], y2[a], z2[a], arena);
    } else {
      D.meta = arc_meta(D.meta, d1, d2, false, false, false);
    }
    auto xy = [&](int e) { return e == 1 ? dd{x1[a], y1[a]} : dd{x2[a], y2[a]}; };
    for (int64_t k = off[a]; k < off[a + 1]; ++k) {
      const int32_t li = idx[k];
      const double z0 = li >= 0 && li < n_lat ? lat_z[li] : __builtin_nan("");
      Decisions dec = {0, 0, 0, 0, 0};
      S2Eft S;
      PairOut o = decide_shared<false>(true, D, z0, dec, S, xy);
      if (o.flags & F_NEEDEXACT) {
        const bool ok = resolve_exact_shared(dec, D.meta, x1[a], y1[a], z1[a], x2[a], y2[a],
                                             z2[a], z0, arena);
        o = decide_shared<true>(true, D, z0, dec, S, xy);
        if (!ok) o.flags |= F_INTERNAL;
      }
      PairOut q = o;
      points_eft_g(
          [&](int t) {
            switch (t) {
              case 0: return P.Fx;
              case 1: return P.eFx;
              case 2: return P.Fy;
              case 3: return P.eFy;
              case 4: return P.nx;
              case 5: return P.enx;
              case 6: return P.ny;
              default: return P.eny;
            }
          },
          D.S2, z0, S, q);
      if (o.count) o = q;
      count[k] = o.count;
      flags[k] = (int32_t)o.flags;
      r0[k] = o.r0;
      r1[k] = o.r1;
      px0[k] = o.px0;
      py0[k] = o.py0;
      px1[k] = o.px1;
      py1[k] = o.py1;
    }
  }
  if (open_arcs) *open_arcs = opened;
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
