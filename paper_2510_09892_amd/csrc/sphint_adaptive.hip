// C-ABI entry point for the adaptive evaluation (include/sphint.h).
//
// Three launches on one stream:
//   k_adapt_init   clears the queue length;
//   k_adapt_pass1  one lane per pair: the direct evaluation with its running error bound
//                  (adaptive_pass1); a certified pair writes its dense outputs, the others
//                  are appended to one of NQ queues (chosen by the 256-pair chunk; one
//                  atomic per wavefront on that queue's counter, lanes placed by popcount).
//                  One shared counter serialised pass 1 on its atomics (1.9 ms for 1e7
//                  pairs); NQ counters on separate cache lines take the contention away;
//   k_adapt_pass2  one lane per queued pair: the EFT evaluation (eval_eft, exact decisions,
//                  serialised exact fallbacks in an LDS arena), flagged RECOMPUTED.
// The queue keeps the two paths in separate wavefronts: pass 2's grid walks only the queued
// pairs, so its cost follows the queue length and not the batch size.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "sphint.h"
#include "sphint_adaptive.hpp"
#include "sphint_host.hpp"

using namespace sphint;

namespace {

constexpr int AD_BLOCK = 256;
constexpr int64_t AD_MAX_BLOCKS = 1 << 16;
constexpr int NQ = 64;             // queues
constexpr size_t COUNTER_STRIDE = 16;  // counters 128 bytes apart (in 8-byte words)
constexpr size_t AD_HEADER = NQ * COUNTER_STRIDE * 8;

// Entries per queue: queue q takes the chunks c with c % NQ == q.
int64_t queue_region(int64_t n) {
  const int64_t chunks = (n + AD_BLOCK - 1) / AD_BLOCK;
  return ((chunks + NQ - 1) / NQ) * AD_BLOCK;
}

struct AdArgs {
  const double *x1, *y1, *z1, *x2, *y2, *z2, *z0;
  int64_t n;
  double tol;
  double *ox, *oy;
  uint8_t *oroot, *ocount, *oflags;
  unsigned long long* qlen;  // NQ queue lengths, COUNTER_STRIDE words apart
  uint32_t* queue;           // NQ regions of `region` pair indices
  int64_t region;
  int64_t* recomputed;       // optional copy of the queue length
};

__device__ __forceinline__ void write_pair(const AdArgs& g, int64_t k, const PairOut& o,
                                           unsigned extra) {
  const bool two = o.count == 2;
  g.ox[2 * k] = o.count ? o.px0 : 0.0;
  g.oy[2 * k] = o.count ? o.py0 : 0.0;
  g.ox[2 * k + 1] = two ? o.px1 : 0.0;
  g.oy[2 * k + 1] = two ? o.py1 : 0.0;
  if (g.oroot) {
    g.oroot[2 * k] = (uint8_t)(o.count ? o.r0 : 0);
    g.oroot[2 * k + 1] = (uint8_t)(two ? o.r1 : 0);
  }
  g.ocount[k] = (uint8_t)o.count;
  if (g.oflags) g.oflags[k] = (uint8_t)((o.flags & 127u) | extra);
}

__global__ void k_adapt_init(unsigned long long* qlen) {
  if (threadIdx.x < NQ) qlen[threadIdx.x * COUNTER_STRIDE] = 0;
}

__global__ __launch_bounds__(AD_BLOCK) void k_adapt_pass1(AdArgs g) {
  const int64_t stride = (int64_t)gridDim.x * AD_BLOCK;
  const int lane = __lane_id();
  for (int64_t k0 = (int64_t)blockIdx.x * AD_BLOCK; k0 < g.n; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    const bool valid = k < g.n;
    PairOut o;
    bool cert = false;
    if (valid)
      cert = adaptive_pass1(g.x1[k], g.y1[k], g.z1[k], g.x2[k], g.y2[k], g.z2[k], g.z0[k],
                            g.tol, o);
    if (valid && cert) write_pair(g, k, o, 0u);
    const bool q = valid && !cert;
    const unsigned long long m = __ballot(q);
    if (m) {  // wavefront-uniform
      const int64_t qi = (k0 / AD_BLOCK) % NQ;
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(g.qlen + qi * COUNTER_STRIDE, (unsigned long long)__popcll(m));
      base = __shfl(base, 0, 64);
      if (q) {
        const unsigned long long below = lane ? (m & ((1ull << lane) - 1)) : 0ull;
        g.queue[qi * g.region + (int64_t)(base + __popcll(below))] = (uint32_t)k;
      }
    }
  }
}

__global__ __launch_bounds__(AD_BLOCK) void k_adapt_pass2(AdArgs g) {
  __shared__ double arena[AD_BLOCK / 64][xp::ARENA];
  __shared__ int64_t start[NQ + 1];  // exclusive prefix of the queue lengths
  if (threadIdx.x < 64) {  // the first wavefront scans the NQ lengths (written by pass 1)
    const int64_t c = (int64_t)g.qlen[threadIdx.x * COUNTER_STRIDE];
    int64_t inc = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t v = __shfl_up(inc, o, 64);
      if (threadIdx.x >= o) inc += v;
    }
    start[threadIdx.x] = inc - c;
    if (threadIdx.x == 63) start[NQ] = inc;
  }
  __syncthreads();
  const int64_t len = start[NQ];
  if (blockIdx.x == 0 && threadIdx.x == 0 && g.recomputed) *g.recomputed = len;
  const int64_t stride = (int64_t)gridDim.x * AD_BLOCK;
  for (int64_t j0 = (int64_t)blockIdx.x * AD_BLOCK; j0 < len; j0 += stride) {  // block-uniform
    const int64_t j = j0 + threadIdx.x;
    const bool valid = j < len;
    int q = 0;  // the queue holding position j: the last q with start[q] <= j
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1)
      if (q + step < NQ && start[q + step] <= j) q += step;
    const int64_t k = valid ? (int64_t)g.queue[q * g.region + (j - start[q])] : 0;
    const bool ok = valid && k < g.n;  // the queue holds indices below n by construction
    double x1 = 0, y1 = 0, z1 = 0, x2 = 0, y2 = 0, z2 = 0, z0 = 0;
    if (ok) {
      x1 = g.x1[k]; y1 = g.y1[k]; z1 = g.z1[k];
      x2 = g.x2[k]; y2 = g.y2[k]; z2 = g.z2[k];
      z0 = g.z0[k];
    }
    const PairOut o = eval_eft(ok, x1, y1, z1, x2, y2, z2, z0, arena[threadIdx.x >> 6],
                               [](bool need, auto&& fn) { resolve_serial(need, fn); });
    if (ok) write_pair(g, k, o, SPHINT_F_RECOMPUTED);
  }
}

int64_t ad_blocks(int64_t n) {
  int64_t b = (n + AD_BLOCK - 1) / AD_BLOCK;
  return b > AD_MAX_BLOCKS ? AD_MAX_BLOCKS : b;
}

}  // namespace

extern "C" size_t sphint_adaptive_workspace_size(int64_t n) {
  if (n < 0) n = 0;
  return AD_HEADER + 4 * (size_t)NQ * (size_t)queue_region(n);
}

extern "C" sphint_status sphint_arc_constlat_adaptive(int64_t n, sphint_pts_soa p1,
                                                      sphint_pts_soa p2, const double* z0,
                                                      double tol, sphint_dense_out out,
                                                      int64_t* out_recomputed, void* workspace,
                                                      size_t workspace_bytes, void* stream) {
  if (n < 0 || n > 0xffffffffLL || !(tol >= 0.0) || !workspace || !aligned256(workspace) ||
      workspace_bytes < sphint_adaptive_workspace_size(n))
    return SPHINT_E_INVAL;
  if (n > 0 && (!p1.x || !p1.y || !p1.z || !p2.x || !p2.y || !p2.z || !z0 || !out.x || !out.y ||
                !out.count))
    return SPHINT_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  AdArgs g{p1.x, p1.y, p1.z, p2.x, p2.y, p2.z, z0, n, tol, out.x, out.y, out.root, out.count,
           out.flags, (unsigned long long*)workspace,
           (uint32_t*)((char*)workspace + AD_HEADER), queue_region(n), out_recomputed};
  hipLaunchKernelGGL(k_adapt_init, dim3(1), dim3(NQ), 0, st, g.qlen);
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  if (n == 0) {
    if (out_recomputed) {  // keep the contract: the count is written on every call
      hipLaunchKernelGGL(k_adapt_pass2, dim3(1), dim3(AD_BLOCK), 0, st, g);
      if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
    }
    return SPHINT_OK;
  }
  const ProfileEvents& pe = profile_events();
  if (pe.start && hipEventRecord(pe.start, st) != hipSuccess) return SPHINT_E_HIP;
  hipLaunchKernelGGL(k_adapt_pass1, dim3((unsigned)ad_blocks(n)), dim3(AD_BLOCK), 0, st, g);
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  if (pe.stop && hipEventRecord(pe.stop, st) != hipSuccess) return SPHINT_E_HIP;
  // pass 2: a grid the device holds at once, walking the queue
  int64_t b2 = (int64_t)4 * device_cus();
  const int64_t bn = ad_blocks(n);
  if (b2 > bn) b2 = bn;
  hipLaunchKernelGGL(k_adapt_pass2, dim3((unsigned)b2), dim3(AD_BLOCK), 0, st, g);
  return hipGetLastError() == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}
