// C-ABI entry points of libsphint (declared in include/sphint.h).
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "sphint.h"
#include "sphint_host.hpp"

using namespace sphint;

namespace {

// Clears the tile states, counter and error word; writes *ototal = 0 for empty calls; for
// CSR calls (off != NULL) also writes the pair-to-arc table (one launch for both).
__global__ __launch_bounds__(INIT_BLOCK) void k_init(uint32_t* ws, uint64_t* status,
                                                     int64_t ntiles, int64_t* ototal, int64_t nnz,
                                                     const int64_t* __restrict__ off,
                                                     int64_t n_arcs,
                                                     uint32_t* __restrict__ parc) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ws[0] = 0u;
    ws[1] = 0u;
    if (nnz == 0) *ototal = 0;
  }
  for (int64_t k = t; k < ntiles; k += (int64_t)gridDim.x * blockDim.x) status[k] = 0ull;
  __shared__ uint32_t win[INIT_BLOCK / 64][FILL_W];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (off && nnz > 0)
    fill_pair_arcs(off, n_arcs, nnz, parc, (int64_t)blockIdx.x * (INIT_BLOCK / 64) + wave,
                   (int64_t)gridDim.x * (INIT_BLOCK / 64), win[wave]);
}

// Copies a call's error bits (the workspace header's error word) to a caller's device word.
__global__ __launch_bounds__(64) void k_error_out(const uint32_t* ws, int32_t* out_error) {
  if (threadIdx.x == 0) *out_error = (int32_t)ws[1];
}

// Pairs per lane of single calls: the EFT evaluation is compute-heavy and gains from four
// resident waves per SIMD, which its 3-row tiles (192 pairs, 31.75 KB of LDS per
// workgroup) allow; the memory-bound naive evaluation does better with fewer, larger
// 4-row tiles (256 pairs).
template <int MODE>
constexpr int wppt_single() {
  return MODE ? 3 : 4;
}
constexpr int WG_PER_CU_SINGLE = 4;  // resident workgroups per CU of the persistent grid


// EFT calls over CSR lists share each arc's z0-free part among the arc's candidates (arc
// records in registers, as the batched kernel's shared schedules) when the lists hold at
// least 2.5 candidates per arc on average; sparser lists (the cubed sphere holds 0.48) keep
// the per-pair evaluation, since a row then spans more arcs than a window holds.  Results
// are the same either way.
inline bool share_arcs(int64_t nnz, int64_t n_arcs) { return 2 * nnz >= 5 * n_arcs; }

// Workgroups of k_intersect_w<MODE, wppt_single<MODE>(), CSR, SHARE> one CU holds at once
// (queried once).
template <int MODE, bool CSR, bool SHARE>
int resident_per_cu() {
  static std::atomic<int> cached{0};  // calls may come from several host threads
  int b = cached.load(std::memory_order_relaxed);
  if (!b) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &b, k_intersect_w<MODE, wppt_single<MODE>(), CSR, SHARE>, BLOCK, 0) != hipSuccess ||
        b <= 0)
      b = 1;
    cached.store(b, std::memory_order_relaxed);
  }
  return b;
}

template <int MODE, bool CSR, bool SHARE = false>
hipError_t launch_main(const KArgs& k, hipStream_t st) {
  int per_cu = resident_per_cu<MODE, CSR, SHARE>();
  if (per_cu > WG_PER_CU_SINGLE) per_cu = WG_PER_CU_SINGLE;
  int64_t grid = (int64_t)per_cu * device_cus();
  const int64_t need = (k.ntiles + 1 + NWAVE - 1) / NWAVE;  // + the scanner wavefront
  if (grid > need) grid = need;
  hipLaunchKernelGGL((k_intersect_w<MODE, wppt_single<MODE>(), CSR, SHARE>), dim3((unsigned)grid),
                     dim3(BLOCK), 0, st, k);
  return hipGetLastError();
}

}  // namespace

extern "C" size_t sphint_workspace_size(int64_t nnz) { return workspace_bytes_for(nnz); }

// The body of sphint_arc_constlat and sphint_arc_constlat_noalloc: arguments validated,
// `ws_base` points at workspace_bytes_for(nnz) (dense calls: the header and tile states
// only) bytes of device memory, 256-byte aligned.
static sphint_status arc_constlat_on(int64_t n_arcs, const sphint_pts_soa& p1,
                                     const sphint_pts_soa& p2, const double* lat_z,
                                     int64_t n_lat, const int64_t* lat_offsets,
                                     const int32_t* lat_idx, int64_t nnz, const sphint_hits& out,
                                     uint8_t* out_count, uint8_t* out_flags, int64_t* out_total,
                                     sphint_mode mode, void* ws_base, int64_t ntiles,
                                     hipStream_t st, int32_t* out_error) {
  uint32_t* ws = (uint32_t*)ws_base;
  uint64_t* status = (uint64_t*)((char*)ws_base + WS_HEADER);

  LaunchChain chain;
  if (chain.begin(st) != hipSuccess) return SPHINT_E_HIP;
  uint32_t* parc = (uint32_t*)((char*)ws_base + WS_HEADER + 8 * status_words_for(nnz));
  int64_t init_blocks = (ntiles + INIT_BLOCK - 1) / INIT_BLOCK;  // one lane per tile state
  if (init_blocks > 8192) init_blocks = 8192;
  if (lat_offsets && nnz > 0 && fill_blocks(n_arcs) > init_blocks)
    init_blocks = fill_blocks(n_arcs);
  if (init_blocks < 1) init_blocks = 1;
  hipLaunchKernelGGL(k_init, dim3((unsigned)init_blocks), dim3(INIT_BLOCK), 0, st, ws, status,
                     ntiles, out_total, nnz, lat_offsets, n_arcs, parc);
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  hipError_t e = hipSuccess;
  if (nnz > 0) {
    KArgs k = make_args(n_arcs, p1, p2, lat_z, n_lat, lat_offsets, lat_idx, nnz, out, out_count,
                        out_flags, out_total, ws, status, ntiles, parc);
    if (profile_events().start && hipEventRecord(profile_events().start, st) != hipSuccess)
      return SPHINT_E_HIP;
    const bool csr = lat_offsets != nullptr;
    if (mode == SPHINT_EFT_FP64)
      e = !csr ? launch_main<1, false>(k, st)
          : share_arcs(nnz, n_arcs) ? launch_main<1, true, true>(k, st)
                                    : launch_main<1, true>(k, st);
    else
      e = csr ? launch_main<0, true>(k, st) : launch_main<0, false>(k, st);
    if (e == hipSuccess && profile_events().stop) e = hipEventRecord(profile_events().stop, st);
  }
  if (e == hipSuccess && out_error) {
    hipLaunchKernelGGL(k_error_out, dim3(1), dim3(64), 0, st, (const uint32_t*)ws, out_error);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = chain.end();
  return e == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}

// Number of tiles of one call, or -1 when there would be too many for the launch.
static int64_t call_tiles(int64_t nnz, sphint_mode mode) {
  const int64_t ntiles =
      wave_tiles_for(nnz, mode == SPHINT_EFT_FP64 ? wppt_single<1>() : wppt_single<0>());
  return ntiles > 0x7fffffffLL ? -1 : ntiles;
}

extern "C" sphint_status sphint_arc_constlat(int64_t n_arcs, sphint_pts_soa p1,
                                             sphint_pts_soa p2, const double* lat_z,
                                             int64_t n_lat, const int64_t* lat_offsets,
                                             const int32_t* lat_idx, int64_t nnz,
                                             sphint_hits out, uint8_t* out_count,
                                             uint8_t* out_flags, int64_t* out_total,
                                             sphint_mode mode, void* workspace,
                                             size_t workspace_bytes, void* stream) {
  if (mode != SPHINT_NAIVE_FP64 && mode != SPHINT_EFT_FP64) return SPHINT_E_INVAL;
  sphint_status v = validate(n_arcs, p1, p2, lat_z, n_lat, lat_offsets, lat_idx, nnz, out,
                             out_count, out_total);
  if (v != SPHINT_OK) return v;
  if (!workspace || !aligned256(workspace) || workspace_bytes < sphint_workspace_size(nnz))
    return SPHINT_E_INVAL;
  const int64_t ntiles = call_tiles(nnz, mode);
  if (ntiles < 0) return SPHINT_E_INVAL;
  return arc_constlat_on(n_arcs, p1, p2, lat_z, n_lat, lat_offsets, lat_idx, nnz, out,
                         out_count, out_flags, out_total, mode, workspace, ntiles,
                         (hipStream_t)stream, nullptr);
}

// ------------------------------------------------------------ allocation-free variant
//
// The workspace of sphint_arc_constlat_noalloc lives in this array: one copy per device
// (each device that runs the library holds it until the process ends).  Host code never
// uses the array's name as a device address: its address on each device comes from
// hipGetSymbolAddress, taken once per device (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[SPHINT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

// Device address of `scratch` on the current device, or nullptr if it cannot be had.
static void* scratch_on_current_device() {
  static std::atomic<void*> ptrs[MAX_DEVICES];
  static std::mutex m;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  void* p = ptrs[dev].load(std::memory_order_acquire);
  if (p) return p;
  std::lock_guard<std::mutex> g(m);
  p = ptrs[dev].load(std::memory_order_relaxed);
  if (!p) {
    void* q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return nullptr;
    ptrs[dev].store(q, std::memory_order_release);
    p = q;
  }
  return p;
}

// Scratch bytes a call over nnz pairs takes: the header and the tile states, and for the
// CSR form the pair-to-arc table.
static size_t noalloc_bytes(int64_t nnz, bool csr) {
  return csr ? workspace_bytes_for(nnz) : WS_HEADER + 8 * status_words_for(nnz);
}

extern "C" sphint_status sphint_arc_constlat_noalloc(int64_t n_arcs, sphint_pts_soa p1,
                                                     sphint_pts_soa p2, const double* lat_z,
                                                     int64_t n_lat, const int64_t* lat_offsets,
                                                     const int32_t* lat_idx, int64_t nnz,
                                                     sphint_hits out, uint8_t* out_count,
                                                     uint8_t* out_flags, int64_t* out_total,
                                                     int32_t* out_error, sphint_mode mode,
                                                     void* stream) {
  if (mode != SPHINT_NAIVE_FP64 && mode != SPHINT_EFT_FP64) return SPHINT_E_INVAL;
  sphint_status v = validate(n_arcs, p1, p2, lat_z, n_lat, lat_offsets, lat_idx, nnz, out,
                             out_count, out_total);
  if (v != SPHINT_OK) return v;
  if (noalloc_bytes(nnz, lat_offsets != nullptr) > SPHINT_NOALLOC_SCRATCH_BYTES)
    return SPHINT_E_INVAL;
  const int64_t ntiles = call_tiles(nnz, mode);
  if (ntiles < 0) return SPHINT_E_INVAL;
  void* ws = scratch_on_current_device();
  if (!ws) return SPHINT_E_HIP;
  return arc_constlat_on(n_arcs, p1, p2, lat_z, n_lat, lat_offsets, lat_idx, nnz, out,
                         out_count, out_flags, out_total, mode, ws, ntiles, (hipStream_t)stream,
                         out_error);
}

extern "C" sphint_status sphint_set_wait_limit(double seconds) {
  if (!(seconds >= 0.0 && seconds <= 3600.0)) return SPHINT_E_INVAL;
  wait_ticks_setting().store((uint64_t)(seconds * 1e8), std::memory_order_relaxed);
  return SPHINT_OK;
}

extern "C" sphint_status sphint_set_profile_events(void* start, void* stop) {
  if ((start == nullptr) != (stop == nullptr)) return SPHINT_E_INVAL;
  profile_events().start = (hipEvent_t)start;
  profile_events().stop = (hipEvent_t)stop;
  return SPHINT_OK;
}

extern "C" sphint_status sphint_check(const void* workspace, int64_t host_total,
                                      int64_t capacity) {
  if (!workspace) return SPHINT_E_INVAL;
  uint32_t hdr[2] = {0, 0};
  if (hipMemcpy(hdr, workspace, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess)
    return SPHINT_E_HIP;
  if (hdr[1]) return SPHINT_E_DEVICE;
  if (host_total > capacity) return SPHINT_E_CAPACITY;
  return SPHINT_OK;
}

extern "C" const char* sphint_status_string(sphint_status s) {
  switch (s) {
    case SPHINT_OK: return "ok";
    case SPHINT_E_INVAL: return "invalid argument";
    case SPHINT_E_CAPACITY: return "hit output capacity exceeded";
    case SPHINT_E_HIP: return "HIP runtime error";
    case SPHINT_E_NOMEM: return "out of memory";
    case SPHINT_E_DEVICE: return "kernel reported an internal limit";
  }
  return "unknown status";
}

extern "C" const char* sphint_version(void) { return "sphint 0.1 gfx950"; }
