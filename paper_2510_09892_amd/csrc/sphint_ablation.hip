// C-ABI entry point for the alternative point formulas (include/sphint.h): one lane per
// pair over a grid-stride loop, both circle-intersection points per pair, written densely.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "sphint.h"
#include "sphint_ablation.hpp"
#include "sphint_host.hpp"

using namespace sphint;

namespace {

constexpr int AB_BLOCK = 256;
constexpr int64_t AB_MAX_BLOCKS = 1 << 16;

struct AbArgs {
  const double *x1, *y1, *z1, *x2, *y2, *z2, *z0;
  int64_t n;
  double *ox, *oy;
  uint8_t* ok;
};

template <int VARIANT>
__device__ __forceinline__ CirclePoints variant_points(double x1, double y1, double z1, double x2,
                                                       double y2, double z2, double z0) {
  if constexpr (VARIANT == ABL_ACCUX) {
    CirclePoints c{0.0, 0.0, 0.0, 0.0, false};
    ArcEft A;
    arc_eft(x1, y1, z1, x2, y2, z2, A);
    if (A.flags) return c;
    const S2Eft S = s2_eft(A, z0);
    if (!(S.ss >= 0.0)) return c;
    PairOut o;
    o.count = 2;
    o.r0 = ROOT_PLUS;
    o.r1 = ROOT_MINUS;
    points_eft(A, z0, S, o);
    return {o.px0, o.py0, o.px1, o.py1, true};
  } else {
    return circle_points<VARIANT>(x1, y1, z1, x2, y2, z2, z0);
  }
}

template <int VARIANT>
__global__ __launch_bounds__(AB_BLOCK) void k_circle(AbArgs g) {
  const int64_t stride = (int64_t)gridDim.x * AB_BLOCK;
  for (int64_t k = (int64_t)blockIdx.x * AB_BLOCK + threadIdx.x; k < g.n; k += stride) {
    const CirclePoints c =
        variant_points<VARIANT>(g.x1[k], g.y1[k], g.z1[k], g.x2[k], g.y2[k], g.z2[k], g.z0[k]);
    g.ox[2 * k] = c.xp;
    g.oy[2 * k] = c.yp;
    g.ox[2 * k + 1] = c.xm;
    g.oy[2 * k + 1] = c.ym;
    g.ok[k] = c.ok ? 1 : 0;
  }
}

template <int VARIANT>
hipError_t launch_circle(const AbArgs& g, hipStream_t st) {
  int64_t blocks = (g.n + AB_BLOCK - 1) / AB_BLOCK;
  if (blocks > AB_MAX_BLOCKS) blocks = AB_MAX_BLOCKS;
  hipLaunchKernelGGL(k_circle<VARIANT>, dim3((unsigned)blocks), dim3(AB_BLOCK), 0, st, g);
  return hipGetLastError();
}

}  // namespace

extern "C" sphint_status sphint_circle_points(int64_t n, sphint_pts_soa p1, sphint_pts_soa p2,
                                              const double* z0, int formula, double* out_x,
                                              double* out_y, uint8_t* out_ok, void* stream) {
  if (n < 0 || formula < SPHINT_FORMULA_EQ22 || formula > SPHINT_FORMULA_ACCUX)
    return SPHINT_E_INVAL;
  if (n == 0) return SPHINT_OK;
  if (!p1.x || !p1.y || !p1.z || !p2.x || !p2.y || !p2.z || !z0 || !out_x || !out_y || !out_ok)
    return SPHINT_E_INVAL;
  const AbArgs g{p1.x, p1.y, p1.z, p2.x, p2.y, p2.z, z0, n, out_x, out_y, out_ok};
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  switch (formula) {
    case SPHINT_FORMULA_EQ22: e = launch_circle<ABL_EQ22>(g, st); break;
    case SPHINT_FORMULA_EQ21: e = launch_circle<ABL_EQ21>(g, st); break;
    case SPHINT_FORMULA_EQ71: e = launch_circle<ABL_EQ71>(g, st); break;
    case SPHINT_FORMULA_KAHAN: e = launch_circle<ABL_KAHAN>(g, st); break;
    default: e = launch_circle<ABL_ACCUX>(g, st); break;
  }
  return e == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}
