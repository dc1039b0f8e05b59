// C-ABI entry point for arc x arc intersections (include/sphint.h).
//
// One lane per pair.  Pairs either pair arc k of A with arc k of B (direct) or gather both
// arcs by int32 index (indexed); every output is written densely, one entry per pair, with
// per-lane consecutive (coalesced) stores.  The work per pair is a few hundred binary64
// operations and 122 bytes of traffic in the direct form, so both modes sit near the
// HBM roofline at full occupancy; nothing here needs a workspace or a device-wide
// ordering.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "sphint.h"
#include "sphint_arcarc.hpp"
#include "sphint_exact.hpp"
#include "sphint_host.hpp"

using namespace sphint;

namespace {

constexpr int AA_BLOCK = 256;
constexpr int64_t AA_MAX_BLOCKS = 1 << 16;  // beyond this the grid loops

struct AAArgs {
  const double *ax1, *ay1, *az1, *ax2, *ay2, *az2;
  const double *bx1, *by1, *bz1, *bx2, *by2, *bz2;
  const int32_t *ia, *ib;
  int64_t n, n_a, n_b;
  double *ox, *oy, *oz;
  uint8_t *ocount, *oflags;
};

struct AAIn {
  double a1[3], a2[3], b1[3], b2[3];
};

// Loads one side's arc i; an index outside [0, n) reads nothing and gives NaN (the pair is
// then reported NONFINITE).
__device__ __forceinline__ void load_arc(const double* x1, const double* y1, const double* z1,
                                         const double* x2, const double* y2, const double* z2,
                                         int64_t i, bool ok, double* p, double* q) {
  const double nan = __builtin_nan("");
  p[0] = ok ? x1[i] : nan;
  p[1] = ok ? y1[i] : nan;
  p[2] = ok ? z1[i] : nan;
  q[0] = ok ? x2[i] : nan;
  q[1] = ok ? y2[i] : nan;
  q[2] = ok ? z2[i] : nan;
}

// Pair k's four endpoints (nothing is read when k >= n).
template <bool IDX>
__device__ __forceinline__ void load_pair(const AAArgs& g, int64_t k, AAIn& in) {
  const bool valid = k < g.n;
  int64_t i = k, j = k;
  if (IDX) {
    if (valid && g.ia) i = g.ia[k];
    if (valid && g.ib) j = g.ib[k];
  }
  const bool oka = valid && i >= 0 && i < g.n_a;
  const bool okb = valid && j >= 0 && j < g.n_b;
  load_arc(g.ax1, g.ay1, g.az1, g.ax2, g.ay2, g.az2, i, oka, in.a1, in.a2);
  load_arc(g.bx1, g.by1, g.bz1, g.bx2, g.by2, g.bz2, j, okb, in.b1, in.b2);
}

// One lane per pair over a block-uniform grid-stride loop (the exact fallback's ballot sees
// whole wavefronts).  Loads are not software-pipelined: with the wavefronts this register
// budget allows resident, a prefetch of the next chunk measured slower.
template <int MODE, bool IDX>
__global__ __launch_bounds__(AA_BLOCK) void k_arc_arc(AAArgs g) {
  const int64_t stride = (int64_t)gridDim.x * AA_BLOCK;
  for (int64_t k0 = (int64_t)blockIdx.x * AA_BLOCK; k0 < g.n; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    const bool valid = k < g.n;
    AAIn in;
    load_pair<IDX>(g, k, in);
    AAOut o;
    if constexpr (MODE == SPHINT_EFT_FP64) {
      __shared__ double arena[AA_BLOCK / 64][xp::ARENA];
      o = eval_aa_eft(valid, in.a1, in.a2, in.b1, in.b2, arena[threadIdx.x >> 6],
                      [](bool need, auto&& fn) { resolve_serial(need, fn); });
    } else {
      o = eval_aa_naive(valid, in.a1, in.a2, in.b1, in.b2);
    }
    if (valid) {
      g.ox[k] = o.px;
      g.oy[k] = o.py;
      g.oz[k] = o.pz;
      g.ocount[k] = (uint8_t)o.count;
      if (g.oflags) g.oflags[k] = (uint8_t)o.flags;
    }
  }
}

template <int MODE, bool IDX>
hipError_t launch_aa(const AAArgs& g, hipStream_t st) {
  int64_t blocks = (g.n + AA_BLOCK - 1) / AA_BLOCK;
  if (blocks > AA_MAX_BLOCKS) blocks = AA_MAX_BLOCKS;
  hipLaunchKernelGGL((k_arc_arc<MODE, IDX>), dim3((unsigned)blocks), dim3(AA_BLOCK), 0, st, g);
  return hipGetLastError();
}

bool soa_ok(const sphint_pts_soa& p) { return p.x && p.y && p.z; }

}  // namespace

extern "C" sphint_status sphint_arc_arc(int64_t n_pairs, sphint_pts_soa a1, sphint_pts_soa a2,
                                        int64_t n_a, sphint_pts_soa b1, sphint_pts_soa b2,
                                        int64_t n_b, const int32_t* ia, const int32_t* ib,
                                        sphint_pts_out out, uint8_t* out_count,
                                        uint8_t* out_flags, int mode, void* stream) {
  if (n_pairs < 0 || n_a < 0 || n_b < 0) return SPHINT_E_INVAL;
  if (mode != SPHINT_NAIVE_FP64 && mode != SPHINT_EFT_FP64) return SPHINT_E_INVAL;
  if ((!ia && n_a != n_pairs) || (!ib && n_b != n_pairs)) return SPHINT_E_INVAL;
  if (n_pairs == 0) return SPHINT_OK;
  if (!out.x || !out.y || !out.z || !out_count) return SPHINT_E_INVAL;
  if ((n_a > 0 && (!soa_ok(a1) || !soa_ok(a2))) || (n_b > 0 && (!soa_ok(b1) || !soa_ok(b2))))
    return SPHINT_E_INVAL;
  AAArgs g{a1.x, a1.y, a1.z, a2.x, a2.y, a2.z, b1.x, b1.y, b1.z, b2.x, b2.y, b2.z,
           ia,   ib,   n_pairs, n_a, n_b, out.x, out.y, out.z, out_count, out_flags};
  hipStream_t st = (hipStream_t)stream;
  const bool idx = ia || ib;
  hipError_t e;
  if (mode == SPHINT_EFT_FP64) e = idx ? launch_aa<1, true>(g, st) : launch_aa<1, false>(g, st);
  else e = idx ? launch_aa<0, true>(g, st) : launch_aa<0, false>(g, st);
  return e == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}
