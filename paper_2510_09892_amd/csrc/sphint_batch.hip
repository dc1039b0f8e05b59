// Batched meshes: many independent CSR (or dense) calls in one persistent launch.
//
// The tiles of all meshes form one sequence (mesh 0's tiles, then mesh 1's, ...).  A
// persistent grid no larger than what the device holds at once walks that sequence in a
// static order (compute wavefront c takes tiles c, c + W, ...); each tile belongs to one mesh
// and runs the single-call tile routine on that mesh's arguments, with the mesh's own slice
// of tile states, so every mesh's outputs equal those of a sphint_arc_constlat call on that
// mesh alone.  The scanner wavefront publishes the in-order prefixes of mesh 0's tiles, then
// mesh 1's, and so on.
//
// Schedule parameters: pairs per lane (wavefront tile = 64 * ppt pairs), the number of
// resident workgroups per CU, and how tiles learn their output offsets (the scanner
// wavefront, or decoupled look-back by every wavefront, which lets small tiles run without
// waiting on one scanner); sphint_batch_autotune times the candidates and keeps the
// fastest.  The init kernel and the persistent kernel are captured once into a HIP graph and
// replayed.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <new>
#include <string>
#include <vector>

#include "sphint_host.hpp"

using namespace sphint;

template <int MODE, int PPT, bool CSR, bool LB, bool SHARE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(const KArgs* __restrict__ args,
                                                 const int64_t* __restrict__ tile_base,
                                                 int n_meshes, int64_t total_tiles) {
  __shared__ WgShared<MODE, PPT, CSR> sh;
  if (threadIdx.x == 0) sh.lock = 0;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int64_t gw = (int64_t)blockIdx.x * NWAVE + wave;
  const int64_t W = (int64_t)gridDim.x * NWAVE - (LB ? 0 : 1);
  if (!LB && gw == W) {  // the scanner follows the global tile order: mesh after mesh
    __builtin_amdgcn_s_setprio(3);  // ahead of the compute wavefronts on its SIMD
    for (int m = 0; m < n_meshes; ++m) {
      const KArgs a = args[m];
      scan_tiles<scan_k<PPT>()>(a.status, a.ntiles, a.ototal, a.ws, a.wait_ticks,
                                reinterpret_cast<uint64_t*>(&sh.stage[wave]));
    }
    return;
  }
  int64_t t = gw;
  int mesh = 0;  // tiles only increase, so the mesh index only moves forward
  wave_loop<MODE, PPT, CSR, flush_at<MODE, PPT, SHARE>(), LB, SHARE>(args, sh, [&](int& m, int64_t& tile) {
    if (t >= total_tiles) return false;
    while (mesh + 1 < n_meshes && tile_base[mesh + 1] <= t) ++mesh;
    m = mesh;
    tile = t - tile_base[mesh];
    t += W;
    return true;
  });
}

// Clears the header and tile states, zeroes the totals of empty meshes and, for CSR plans,
// fills every mesh's pair-to-arc table in the same launch (every wavefront takes part in
// every mesh's fill, as in the one-shot launch's init).
__global__ __launch_bounds__(INIT_BLOCK) void k_batch_init(uint32_t* ws, uint64_t* status,
                                                           int64_t total_tiles,
                                                           const KArgs* __restrict__ args,
                                                           int n_meshes, int csr) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ws[0] = 0u;
    ws[1] = 0u;
  }
  if (t < n_meshes && args[t].nnz == 0) *args[t].ototal = 0;
  for (int64_t k = t; k < total_tiles; k += (int64_t)gridDim.x * blockDim.x) status[k] = 0ull;
  if (!csr) return;
  __shared__ uint32_t win[INIT_BLOCK / 64][FILL_W];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int m = 0; m < n_meshes; ++m) {
    const KArgs& a = args[m];
    if (a.nnz > 0)
      fill_pair_arcs(a.off, a.n_arcs, a.nnz, const_cast<uint32_t*>(a.parc),
                     (int64_t)blockIdx.x * (INIT_BLOCK / 64) + wave,
                     (int64_t)gridDim.x * (INIT_BLOCK / 64), win[wave]);
  }
}

struct sphint_plan {
  sphint_mode mode = SPHINT_EFT_FP64;
  std::vector<sphint_mesh_desc> meshes;
  int device = 0;
  int cus = 1;
  // schedule
  int ppt = 1;
  int wg_per_cu = 0;  // resident workgroups per CU (0: as many as fit)
  bool lookback = false;  // tile offsets by decoupled look-back instead of the scanner
  bool share = false;     // EFT over CSR lists: arc records shared by a tile's rows
  // device state
  KArgs* d_args = nullptr;
  int64_t* d_tile_base = nullptr;
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<int64_t> tile_base;
  int64_t total_tiles = 0;
  bool csr = false;  // every mesh of a plan has the same form
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

template <int MODE, int PPT, bool CSR, bool LB = false, bool SHARE = false>
int max_resident() {
  static std::atomic<int> cached{0};  // queried once; calls may come from several threads
  int blocks = cached.load(std::memory_order_relaxed);
  if (blocks) return blocks;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<MODE, PPT, CSR, LB, SHARE>,
                                                   BLOCK, 0) !=
          hipSuccess ||
      blocks <= 0)
    blocks = 1;
  cached.store(blocks, std::memory_order_relaxed);
  return blocks;
}

template <bool CSR, bool LB>
int resident_per_cu_form(sphint_mode mode, int ppt) {
  if (mode == SPHINT_EFT_FP64) {
    if (ppt == 1) return max_resident<1, 1, CSR, LB>();
    if (ppt == 2) return max_resident<1, 2, CSR, LB>();
    if (ppt == 3) return max_resident<1, 3, CSR, LB>();
    return max_resident<1, 4, CSR, LB>();
  }
  if (ppt == 1) return max_resident<0, 1, CSR, LB>();
  if (ppt == 2) return max_resident<0, 2, CSR, LB>();
  if (ppt == 3) return max_resident<0, 3, CSR, LB>();
  return max_resident<0, 4, CSR, LB>();
}

// Arc records are shared in EFT mode over CSR lists only; five pairs per lane exist with
// them only.
constexpr int PPT_SHARED_MAX = 5;
bool can_share(const sphint_plan* p) { return p->mode == SPHINT_EFT_FP64 && p->csr; }

void drop_graph(sphint_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  p->exec = nullptr;
}

// (Re)lays out tiles for the plan's ppt and uploads the per-mesh arguments.
sphint_status layout(sphint_plan* p) {
  drop_graph(p);
  const int n = (int)p->meshes.size();
  p->tile_base.assign(n + 1, 0);
  for (int m = 0; m < n; ++m)
    p->tile_base[m + 1] = p->tile_base[m] + wave_tiles_for(p->meshes[m].nnz, p->ppt);
  p->total_tiles = p->tile_base[n];
  if (p->total_tiles > 0x7fffffffLL) return SPHINT_E_INVAL;
  int64_t nnz_all = 0;
  for (int m = 0; m < n; ++m) nnz_all += p->meshes[m].nnz;
  const size_t status_words = (size_t)(p->total_tiles > 0 ? p->total_tiles : 1);
  const size_t need = WS_HEADER + 8 * status_words + (p->csr ? 4 * (size_t)nnz_all : 0);
  if (need > p->ws_bytes) {
    if (p->d_ws) (void)hipFree(p->d_ws);
    p->d_ws = nullptr;
    if (hipMalloc(&p->d_ws, need) != hipSuccess) return SPHINT_E_HIP;
    p->ws_bytes = need;
  }
  uint32_t* ws = (uint32_t*)p->d_ws;
  uint64_t* status = (uint64_t*)((char*)p->d_ws + WS_HEADER);
  uint32_t* parc = (uint32_t*)((char*)p->d_ws + WS_HEADER + 8 * status_words);
  std::vector<KArgs> h(n);
  for (int m = 0; m < n; ++m) {
    const sphint_mesh_desc& d = p->meshes[m];
    h[m] = make_args(d.n_arcs, d.p1, d.p2, d.lat_z, d.n_lat, d.lat_offsets, d.lat_idx, d.nnz,
                     d.out, d.out_count, d.out_flags, d.out_total, ws,
                     status + p->tile_base[m], p->tile_base[m + 1] - p->tile_base[m], parc);
    if (p->csr) parc += d.nnz;
  }
  if (hipMemcpy(p->d_args, h.data(), sizeof(KArgs) * n, hipMemcpyHostToDevice) != hipSuccess)
    return SPHINT_E_HIP;
  if (hipMemcpy(p->d_tile_base, p->tile_base.data(), sizeof(int64_t) * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess)
    return SPHINT_E_HIP;
  return SPHINT_OK;
}

template <bool LB>
int resident_per_cu_share(int ppt) {
  if (ppt == 1) return max_resident<1, 1, true, LB, true>();
  if (ppt == 2) return max_resident<1, 2, true, LB, true>();
  if (ppt == 3) return max_resident<1, 3, true, LB, true>();
  if (ppt == 4) return max_resident<1, 4, true, LB, true>();
  return max_resident<1, PPT_SHARED_MAX, true, LB, true>();
}

int resident_per_cu(const sphint_plan* p, int ppt, bool lb, bool share) {
  if (share) return lb ? resident_per_cu_share<true>(ppt) : resident_per_cu_share<false>(ppt);
  if (lb)
    return p->csr ? resident_per_cu_form<true, true>(p->mode, ppt)
                  : resident_per_cu_form<false, true>(p->mode, ppt);
  return p->csr ? resident_per_cu_form<true, false>(p->mode, ppt)
                : resident_per_cu_form<false, false>(p->mode, ppt);
}

template <int MODE, int PPT, bool LB>
void launch_batch_lb(const sphint_plan* p, unsigned grid, hipStream_t st) {
  if (MODE == 1 && p->csr && p->share)
    hipLaunchKernelGGL((k_batch<1, PPT, true, LB, true>), dim3(grid), dim3(BLOCK), 0, st,
                       p->d_args, p->d_tile_base, (int)p->meshes.size(), p->total_tiles);
  else if (p->csr)
    hipLaunchKernelGGL((k_batch<MODE, PPT, true, LB>), dim3(grid), dim3(BLOCK), 0, st, p->d_args,
                       p->d_tile_base, (int)p->meshes.size(), p->total_tiles);
  else
    hipLaunchKernelGGL((k_batch<MODE, PPT, false, LB>), dim3(grid), dim3(BLOCK), 0, st, p->d_args,
                       p->d_tile_base, (int)p->meshes.size(), p->total_tiles);
}

// Five-row tiles exist with shared arc records only (one window fill serves five rows; the
// LDS already limits four-row EFT tiles to three workgroups per CU, and five still fit three).
template <bool LB>
void launch_batch_shared5(const sphint_plan* p, unsigned grid, hipStream_t st) {
  hipLaunchKernelGGL((k_batch<1, PPT_SHARED_MAX, true, LB, true>), dim3(grid), dim3(BLOCK), 0, st,
                     p->d_args, p->d_tile_base, (int)p->meshes.size(), p->total_tiles);
}

template <int MODE, int PPT>
void launch_batch(const sphint_plan* p, unsigned grid, hipStream_t st) {
  if (p->lookback) launch_batch_lb<MODE, PPT, true>(p, grid, st);
  else launch_batch_lb<MODE, PPT, false>(p, grid, st);
}

// Enqueues init + persistent kernel on st (no graph).
sphint_status enqueue(const sphint_plan* p, hipStream_t st) {
  LaunchChain chain;  // no-op while st is being captured
  if (chain.begin(st) != hipSuccess) return SPHINT_E_HIP;
  uint32_t* ws = (uint32_t*)p->d_ws;
  uint64_t* status = (uint64_t*)((char*)p->d_ws + WS_HEADER);
  const int n = (int)p->meshes.size();
  int64_t work = p->total_tiles > n ? p->total_tiles : n;
  int64_t ib = (work + INIT_BLOCK - 1) / INIT_BLOCK;
  if (ib > 1024) ib = 1024;
  if (p->csr)
    for (int m = 0; m < n; ++m)
      if (p->meshes[m].nnz > 0 && fill_blocks(p->meshes[m].n_arcs) > ib)
        ib = fill_blocks(p->meshes[m].n_arcs);
  if (ib < 1) ib = 1;
  hipLaunchKernelGGL(k_batch_init, dim3((unsigned)ib), dim3(INIT_BLOCK), 0, st, ws, status,
                     p->total_tiles, p->d_args, n, p->csr ? 1 : 0);
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  if (p->total_tiles > 0) {
    // every wavefront of the grid must be resident at once (see k_batch)
    const int res = resident_per_cu(p, p->ppt, p->lookback, p->share);
    const int per_cu = p->wg_per_cu > 0 && p->wg_per_cu < res ? p->wg_per_cu : res;
    int64_t grid = (p->total_tiles + (p->lookback ? 0 : 1) + NWAVE - 1) / NWAVE;  // + scanner
    if ((int64_t)per_cu * p->cus < grid) grid = (int64_t)per_cu * p->cus;
    const bool eft = p->mode == SPHINT_EFT_FP64;
    if (p->ppt == 1) eft ? launch_batch<1, 1>(p, (unsigned)grid, st) : launch_batch<0, 1>(p, (unsigned)grid, st);
    else if (p->ppt == 2) eft ? launch_batch<1, 2>(p, (unsigned)grid, st) : launch_batch<0, 2>(p, (unsigned)grid, st);
    else if (p->ppt == 3) eft ? launch_batch<1, 3>(p, (unsigned)grid, st) : launch_batch<0, 3>(p, (unsigned)grid, st);
    else if (p->ppt == 4) eft ? launch_batch<1, 4>(p, (unsigned)grid, st) : launch_batch<0, 4>(p, (unsigned)grid, st);
    else if (p->lookback) launch_batch_shared5<true>(p, (unsigned)grid, st);  // shared only
    else launch_batch_shared5<false>(p, (unsigned)grid, st);
  }
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  return chain.end() == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}

std::string plan_key(const sphint_plan* p) {
  int64_t nnz = 0, arcs = 0;
  for (const auto& m : p->meshes) {
    nnz += m.nnz;
    arcs += m.n_arcs;
  }
  char buf[160];
  snprintf(buf, sizeof(buf), "mode=%d meshes=%zu arcs=%lld nnz=%lld cus=%d", (int)p->mode,
           p->meshes.size(), (long long)arcs, (long long)nnz, p->cus);
  return buf;
}

}  // namespace

extern "C" sphint_status sphint_batch_plan_create(const sphint_mesh_desc* meshes, int n_meshes,
                                                  sphint_mode mode, sphint_plan** plan) {
  if (!plan || n_meshes <= 0 || !meshes) return SPHINT_E_INVAL;
  if (mode != SPHINT_NAIVE_FP64 && mode != SPHINT_EFT_FP64) return SPHINT_E_INVAL;
  *plan = nullptr;
  for (int m = 0; m < n_meshes; ++m) {
    const sphint_mesh_desc& d = meshes[m];
    sphint_status v = validate(d.n_arcs, d.p1, d.p2, d.lat_z, d.n_lat, d.lat_offsets,
                               d.lat_idx, d.nnz, d.out, d.out_count, d.out_total);
    if (v != SPHINT_OK) return v;
    if ((d.lat_offsets != nullptr) != (meshes[0].lat_offsets != nullptr)) return SPHINT_E_INVAL;
  }
  sphint_plan* p = new (std::nothrow) sphint_plan();
  if (!p) return SPHINT_E_NOMEM;
  p->mode = mode;
  p->csr = meshes[0].lat_offsets != nullptr;
  p->meshes.assign(meshes, meshes + n_meshes);
  (void)hipGetDevice(&p->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) p->cus = prop.multiProcessorCount;
  if (hipMalloc((void**)&p->d_args, sizeof(KArgs) * n_meshes) != hipSuccess ||
      hipMalloc((void**)&p->d_tile_base, sizeof(int64_t) * (n_meshes + 1)) != hipSuccess) {
    sphint_plan_destroy(p);
    return SPHINT_E_HIP;
  }
  p->ppt = 4;
  p->wg_per_cu = 0;
  sphint_status s = layout(p);
  if (s != SPHINT_OK) {
    sphint_plan_destroy(p);
    return s;
  }
  *plan = p;
  return SPHINT_OK;
}

extern "C" sphint_status sphint_batch_launch(sphint_plan* p, void* stream) {
  if (!p) return SPHINT_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!p->exec) {
    if (!p->capture_stream &&
        hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)
      return SPHINT_E_HIP;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return SPHINT_E_HIP;
    sphint_status s = enqueue(p, p->capture_stream);
    hipError_t e = hipStreamEndCapture(p->capture_stream, &g);
    if (s != SPHINT_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return SPHINT_E_HIP;
    }
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->exec = nullptr;
      return SPHINT_E_HIP;
    }
  }
  LaunchChain chain;
  if (chain.begin(st) != hipSuccess || hipGraphLaunch(p->exec, st) != hipSuccess ||
      chain.end() != hipSuccess)
    return SPHINT_E_HIP;
  return SPHINT_OK;
}

extern "C" sphint_status sphint_batch_autotune(sphint_plan* p, const char* cache_path,
                                               void* stream) {
  if (!p) return SPHINT_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const std::string key = plan_key(p);
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[512];
      while (fgets(line, sizeof(line), f)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        if (key == line) {
          int ppt = 0, wg = -1, lb = 0, sh = 0;
          if (sscanf(bar + 1, "%d %d %d %d", &ppt, &wg, &lb, &sh) >= 2 && ppt >= 1 &&
              (ppt <= 4 || (ppt == PPT_SHARED_MAX && sh == 1)) && wg >= 0 &&
              (lb == 0 || lb == 1) && (sh == 0 || (sh == 1 && can_share(p)))) {
            fclose(f);
            p->ppt = ppt;
            p->wg_per_cu = wg;
            p->lookback = lb == 1;
            p->share = sh == 1;
            return layout(p);
          }
        }
      }
      fclose(f);
    }
  }
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess)
    return SPHINT_E_HIP;
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  float best = 1e30f;
  int best_ppt = 1, best_wg = 0;
  bool best_lb = false, best_share = false;
  // candidates: pairs per lane 1-4 x {scanner, look-back}; with shared arc records (EFT over
  // CSR lists) also pairs per lane 2-5 (one-row tiles share nothing across rows)
  struct Cand {
    int ppt;
    bool lb, share;
  };
  std::vector<Cand> cands;
  for (int lb = 0; lb < 2; ++lb)
    for (int ppt = 1; ppt <= 4; ++ppt) cands.push_back({ppt, lb == 1, false});
  if (can_share(p))
    for (int lb = 0; lb < 2; ++lb)
      for (int ppt = 2; ppt <= PPT_SHARED_MAX; ++ppt) cands.push_back({ppt, lb == 1, true});
  for (const Cand& c : cands) {
    const int ppt = c.ppt;
    const bool lb = c.lb, share = c.share;
    const int res = resident_per_cu(p, ppt, lb, share);
    const int wgs[4] = {res, res > 1 ? res - 1 : 1, res > 2 ? res / 2 : 1, 1};
    for (int wi = 0; wi < 4; ++wi) {
      if (wi > 0 && wgs[wi] == wgs[wi - 1]) continue;
      p->ppt = ppt;
      p->wg_per_cu = wgs[wi];
      p->lookback = lb;
      p->share = share;
      sphint_status s = layout(p);
      if (s != SPHINT_OK) return s;
      if (enqueue(p, st) != SPHINT_OK) return SPHINT_E_HIP;  // warm-up
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 3; ++r)
        if (enqueue(p, st) != SPHINT_OK) return SPHINT_E_HIP;
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) return SPHINT_E_HIP;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        best_ppt = ppt;
        best_wg = wgs[wi];
        best_lb = lb;
        best_share = share;
      }
    }
  }
  p->ppt = best_ppt;
  p->wg_per_cu = best_wg;
  p->lookback = best_lb;
  p->share = best_share;
  sphint_status s = layout(p);
  if (s == SPHINT_OK && cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%s|%d %d %d %d\n", key.c_str(), best_ppt, best_wg, best_lb ? 1 : 0,
              best_share ? 1 : 0);
      fclose(f);
    }
  }
  return s;
}

extern "C" sphint_status sphint_batch_params(const sphint_plan* p, int* pairs_per_thread,
                                             int* wg_per_cu) {
  if (!p) return SPHINT_E_INVAL;
  if (pairs_per_thread) *pairs_per_thread = p->ppt;
  if (wg_per_cu) *wg_per_cu = p->wg_per_cu;
  return SPHINT_OK;
}

extern "C" sphint_status sphint_batch_set_params(sphint_plan* p, int pairs_per_thread,
                                                 int wg_per_cu) {
  if (!p || pairs_per_thread < 1 || wg_per_cu < 0 ||
      pairs_per_thread > (p->share ? PPT_SHARED_MAX : 4))
    return SPHINT_E_INVAL;
  p->ppt = pairs_per_thread;
  p->wg_per_cu = wg_per_cu;
  return layout(p);
}

extern "C" sphint_status sphint_batch_scan(const sphint_plan* p, int* lookback) {
  if (!p || !lookback) return SPHINT_E_INVAL;
  *lookback = p->lookback ? 1 : 0;
  return SPHINT_OK;
}

extern "C" sphint_status sphint_batch_set_scan(sphint_plan* p, int lookback) {
  if (!p || (lookback != 0 && lookback != 1)) return SPHINT_E_INVAL;
  p->lookback = lookback == 1;
  return layout(p);
}

extern "C" sphint_status sphint_batch_share(const sphint_plan* p, int* share) {
  if (!p || !share) return SPHINT_E_INVAL;
  *share = p->share ? 1 : 0;
  return SPHINT_OK;
}

extern "C" sphint_status sphint_batch_set_share(sphint_plan* p, int share) {
  if (!p || (share != 0 && share != 1) || (share == 1 && !can_share(p)) ||
      (share == 0 && p->ppt > 4))
    return SPHINT_E_INVAL;
  p->share = share == 1;
  return layout(p);
}

extern "C" sphint_status sphint_batch_check(const sphint_plan* p) {
  if (!p || !p->d_ws) return SPHINT_E_INVAL;
  uint32_t hdr[2] = {0, 0};
  if (hipMemcpy(hdr, p->d_ws, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess)
    return SPHINT_E_HIP;
  if (hdr[1]) return SPHINT_E_DEVICE;
  for (const auto& m : p->meshes) {
    int64_t t = 0;
    if (hipMemcpy(&t, m.out_total, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess)
      return SPHINT_E_HIP;
    if (t > m.out.capacity) return SPHINT_E_CAPACITY;
  }
  return SPHINT_OK;
}

extern "C" void sphint_plan_destroy(sphint_plan* p) {
  if (!p) return;
  drop_graph(p);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->d_args) (void)hipFree(p->d_args);
  if (p->d_tile_base) (void)hipFree(p->d_tile_base);
  if (p->d_ws) (void)hipFree(p->d_ws);
  delete p;
}

// ------------------------------------------------------------ one-shot batched launch
//
// Continuous batching changes the set of meshes on every launch, so a plan (device tables,
// a captured graph) would be rebuilt each time.  sphint_batch_run instead passes the
// meshes' arguments to an init kernel by value; the init kernel writes them into the
// caller's workspace, clears the tile states and fills the CSR pair-to-arc tables, and the
// same persistent batched kernel as a plan's runs behind it.  Two launches, no allocation,
// no host synchronisation.

namespace {

constexpr int RUN_MAX = SPHINT_BATCH_RUN_MAX;

struct RunTable {
  KArgs m[RUN_MAX];
  int64_t tile_base[RUN_MAX + 1];
};
static_assert(sizeof(RunTable) <= 3584, "the table travels as a kernel argument");

constexpr size_t RUN_ARGS_BYTES = (sizeof(KArgs) * RUN_MAX + 255) / 256 * 256;
constexpr size_t RUN_BASE_BYTES = (sizeof(int64_t) * (RUN_MAX + 1) + 255) / 256 * 256;

// Workspace layout: header (counter, error word) | argument table | tile bases | tile
// states (one word per 64 pairs of each mesh, at most) | CSR pair-to-arc tables.
size_t run_status_words(int n_meshes, int64_t total_nnz) {
  return (size_t)((total_nnz + 63) / 64 + n_meshes + 1);
}
size_t run_workspace_bytes(int n_meshes, int64_t total_nnz) {
  return WS_HEADER + RUN_ARGS_BYTES + RUN_BASE_BYTES + 8 * run_status_words(n_meshes, total_nnz) +
         4 * (size_t)total_nnz;
}

__global__ __launch_bounds__(INIT_BLOCK) void k_batch_run_init(const RunTable tbl, int n_meshes,
                                                               KArgs* __restrict__ d_args,
                                                               int64_t* __restrict__ d_base,
                                                               uint64_t* __restrict__ status,
                                                               int64_t total_tiles,
                                                               uint32_t* __restrict__ ws,
                                                               int csr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ws[0] = 0u;
    ws[1] = 0u;
  }
  if (t < n_meshes) {
    d_args[t] = tbl.m[t];
    if (tbl.m[t].nnz == 0) *tbl.m[t].ototal = 0;
  }
  if (t <= n_meshes) d_base[t] = tbl.tile_base[t];
  for (int64_t k = t; k < total_tiles; k += (int64_t)gridDim.x * blockDim.x) status[k] = 0ull;
  if (!csr) return;
  __shared__ uint32_t win[INIT_BLOCK / 64][FILL_W];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int m = 0; m < n_meshes; ++m) {  // every wavefront takes part in every mesh's fill
    const KArgs& a = tbl.m[m];
    if (a.nnz > 0)
      fill_pair_arcs(a.off, a.n_arcs, a.nnz, const_cast<uint32_t*>(a.parc),
                     (int64_t)blockIdx.x * (INIT_BLOCK / 64) + wave,
                     (int64_t)gridDim.x * (INIT_BLOCK / 64), win[wave]);
  }
}

// Pairs per lane of a one-shot batch: those of single calls.
constexpr int run_ppt(sphint_mode mode) { return mode == SPHINT_EFT_FP64 ? 3 : 4; }

// SHARE: EFT over CSR lists holding at least 2.5 candidates per arc in all (the single
// call's rule), arc records shared among a tile's rows.
template <int MODE, bool CSR, bool SHARE = false>
void launch_run(const KArgs* d_args, const int64_t* d_base, int n, int64_t total_tiles,
                hipStream_t st) {
  constexpr int PPT = MODE ? 3 : 4;
  const int per_cu = max_resident<MODE, PPT, CSR, false, SHARE>();
  int64_t grid = (total_tiles + 1 + NWAVE - 1) / NWAVE;  // + the scanner
  if ((int64_t)per_cu * device_cus() < grid) grid = (int64_t)per_cu * device_cus();
  hipLaunchKernelGGL((k_batch<MODE, PPT, CSR, false, SHARE>), dim3((unsigned)grid), dim3(BLOCK),
                     0, st, d_args, d_base, n, total_tiles);
}

}  // namespace

extern "C" size_t sphint_batch_run_workspace_size(int n_meshes, int64_t total_nnz) {
  if (n_meshes < 0 || total_nnz < 0) return 0;
  return run_workspace_bytes(n_meshes, total_nnz);
}

extern "C" sphint_status sphint_batch_run(const sphint_mesh_desc* meshes, int n_meshes,
                                          sphint_mode mode, void* workspace,
                                          size_t workspace_bytes, void* stream) {
  if (!meshes || n_meshes < 1 || n_meshes > RUN_MAX) return SPHINT_E_INVAL;
  if (mode != SPHINT_NAIVE_FP64 && mode != SPHINT_EFT_FP64) return SPHINT_E_INVAL;
  const bool csr = meshes[0].lat_offsets != nullptr;
  int64_t total_nnz = 0, total_arcs = 0;
  for (int m = 0; m < n_meshes; ++m) {
    const sphint_mesh_desc& d = meshes[m];
    sphint_status v = validate(d.n_arcs, d.p1, d.p2, d.lat_z, d.n_lat, d.lat_offsets, d.lat_idx,
                               d.nnz, d.out, d.out_count, d.out_total);
    if (v != SPHINT_OK) return v;
    if ((d.lat_offsets != nullptr) != csr) return SPHINT_E_INVAL;
    total_nnz += d.nnz;
    total_arcs += d.n_arcs;
  }
  if (total_nnz > ((int64_t)1 << 40)) return SPHINT_E_INVAL;
  if (!workspace || !aligned256(workspace) ||
      workspace_bytes < run_workspace_bytes(n_meshes, total_nnz))
    return SPHINT_E_INVAL;
  const int ppt = run_ppt(mode);
  RunTable tbl;
  memset(&tbl, 0, sizeof(tbl));
  char* w = (char*)workspace;
  uint32_t* ws = (uint32_t*)w;
  KArgs* d_args = (KArgs*)(w + WS_HEADER);
  int64_t* d_base = (int64_t*)(w + WS_HEADER + RUN_ARGS_BYTES);
  uint64_t* status = (uint64_t*)(w + WS_HEADER + RUN_ARGS_BYTES + RUN_BASE_BYTES);
  uint32_t* parc = (uint32_t*)(status + run_status_words(n_meshes, total_nnz));
  int64_t max_arcs = 0;
  for (int m = 0; m < n_meshes; ++m) {
    const sphint_mesh_desc& d = meshes[m];
    const int64_t nt = wave_tiles_for(d.nnz, ppt);
    tbl.tile_base[m + 1] = tbl.tile_base[m] + nt;
    tbl.m[m] = make_args(d.n_arcs, d.p1, d.p2, d.lat_z, d.n_lat, d.lat_offsets, d.lat_idx, d.nnz,
                         d.out, d.out_count, d.out_flags, d.out_total, ws,
                         status + tbl.tile_base[m], nt, csr ? parc : nullptr);
    if (csr) parc += d.nnz;
    if (d.n_arcs > max_arcs) max_arcs = d.n_arcs;
  }
  for (int m = n_meshes; m < RUN_MAX; ++m) tbl.tile_base[m + 1] = tbl.tile_base[n_meshes];
  const int64_t total_tiles = tbl.tile_base[n_meshes];
  if (total_tiles > 0x7fffffffLL) return SPHINT_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  LaunchChain chain;
  if (chain.begin(st) != hipSuccess) return SPHINT_E_HIP;
  int64_t ib = (total_tiles + INIT_BLOCK - 1) / INIT_BLOCK;
  if (csr && fill_blocks(max_arcs) > ib) ib = fill_blocks(max_arcs);
  if (ib > 8192) ib = 8192;
  if (ib < 1) ib = 1;
  hipLaunchKernelGGL(k_batch_run_init, dim3((unsigned)ib), dim3(INIT_BLOCK), 0, st, tbl, n_meshes,
                     d_args, d_base, status, total_tiles, ws, (int)csr);
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  if (total_tiles > 0) {
    const bool eft = mode == SPHINT_EFT_FP64;
    if (csr) eft ? (2 * total_nnz >= 5 * total_arcs
                        ? launch_run<1, true, true>(d_args, d_base, n_meshes, total_tiles, st)
                        : launch_run<1, true>(d_args, d_base, n_meshes, total_tiles, st))
                 : launch_run<0, true>(d_args, d_base, n_meshes, total_tiles, st);
    else eft ? launch_run<1, false>(d_args, d_base, n_meshes, total_tiles, st)
             : launch_run<0, false>(d_args, d_base, n_meshes, total_tiles, st);
    if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  }
  return chain.end() == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}
