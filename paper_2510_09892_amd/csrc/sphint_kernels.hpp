// gfx950 kernels for the arc x constant-latitude intersection (Sec. 2, Eq. 2.2; Alg. 8).
//
// One lane per arc-latitude pair, 256-lane workgroups (four wave64s).  Each workgroup takes
// a tile of consecutive pairs, evaluates them (naive or EFT), then writes its hits into one
// dense output in pair order: a ballot/popcount scan inside each wavefront, a four-entry
// scan across wavefronts, and a single-pass decoupled look-back across tiles (tile ids are
// taken from an atomic counter in start order, so every tile waited on is already
// running).  Rare undecided exact predicates are resolved one lane at a time per wavefront
// in an LDS arena (exact_sign), keeping private arrays and scratch out of the kernel.
#pragma once
#pragma clang fp contract(off)

#include "sphint_pair.hpp"

namespace sphint {

constexpr int BLOCK = 256;
constexpr int NWAVE = BLOCK / 64;
constexpr size_t WS_HEADER = 256;  // counter + error word, padded
constexpr uint64_t ST_AGG = 1, ST_PREFIX = 2;
constexpr long SPIN_LIMIT = 1L << 24;  // bounded wait: ~seconds, far beyond any real wait
enum : uint32_t { ERR_SPIN = 1u, ERR_EXACT = 2u };

struct KArgs {
  int64_t n_arcs, n_lat, nnz;
  const double *x1, *y1, *z1, *x2, *y2, *z2;
  const double* lat_z;
  const int64_t* off;
  const int32_t* idx;
  double *ox, *oy;
  int64_t* opair;
  uint8_t* oroot;
  int64_t cap;
  uint8_t* ocount;
  uint8_t* oflags;
  int64_t* ototal;
  uint32_t* ws;      // [0] tile counter, [1] error bits
  uint64_t* status;  // one word per tile: (value << 2) | state
  int64_t ntiles;
};

// Runs fn() for every lane of the wavefront with need == true, one lane at a time.
template <class F>
__device__ __forceinline__ void resolve_serial(bool need, F&& fn) {
  unsigned long long m = __ballot(need);
  const int lane = __lane_id();
  while (m) {
    int l = __ffsll(m) - 1;
    if (lane == l) fn();
    m &= m - 1;
  }
}

// Largest a in [lo, hi] with off[a] <= k: the arc owning CSR entry k.
__device__ __forceinline__ int64_t find_arc(const int64_t* __restrict__ off, int64_t lo,
                                            int64_t hi, int64_t k) {
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Single-pass decoupled look-back: publish this tile's aggregate, sum predecessors until
// one with an inclusive prefix, publish the inclusive prefix.  Returns the exclusive prefix.
__device__ __forceinline__ int64_t look_back(uint64_t* status, int64_t tile, int64_t agg,
                                             uint32_t* ws) {
  if (tile == 0) {
    __hip_atomic_store(status, ((uint64_t)agg << 2) | ST_PREFIX, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  __hip_atomic_store(status + tile, ((uint64_t)agg << 2) | ST_AGG, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  int64_t excl = 0;
  int64_t j = tile - 1;
  long spins = 0;
  while (j >= 0) {
    uint64_t w = __hip_atomic_load(status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t st = w & 3u;
    if (st == 0) {
      if (++spins > SPIN_LIMIT) {
        atomicOr(ws + 1, ERR_SPIN);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += (int64_t)(w >> 2);
    if (st == ST_PREFIX) break;
    --j;
  }
  __hip_atomic_store(status + tile, ((uint64_t)(excl + agg) << 2) | ST_PREFIX,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Shared state of one workgroup while it processes a tile.
template <int MODE, int PPT>
struct TileShared {
  double arena[MODE ? NWAVE : 1][MODE ? xp::ARENA : 1];
  int64_t prefix, arc_lo, arc_hi;
  int wtot[PPT][NWAVE];
};

// Evaluates pairs [tile * BLOCK * PPT, +BLOCK * PPT) of call `a` and writes their counts,
// flags and compacted hits.  Pair base + j * BLOCK + tid goes to thread tid (coalesced
// loads), so hits are ordered row j by row j.  All threads of the workgroup must call it.
template <int MODE, int PPT>
__device__ __forceinline__ void run_tile(const KArgs& a, int64_t tile, TileShared<MODE, PPT>& sh) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const bool csr = a.off != nullptr;
  const int64_t base = tile * (int64_t)(BLOCK * PPT);
  if (csr) {
    if (tid == 0) sh.arc_lo = find_arc(a.off, 0, a.n_arcs - 1, base);
    if (tid == BLOCK - 1) {
      int64_t last = base + BLOCK * PPT - 1 < a.nnz ? base + BLOCK * PPT - 1 : a.nnz - 1;
      sh.arc_hi = find_arc(a.off, 0, a.n_arcs - 1, last);
    }
    __syncthreads();
  }
  PairOut o[PPT];
  int woff[PPT];
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t i = base + (int64_t)j * BLOCK + tid;
    const bool valid = i < a.nnz;
    int64_t arc = i;
    double z0 = 0.0;
    if (csr) {
      arc = valid ? find_arc(a.off, sh.arc_lo, sh.arc_hi, i) : 0;
      if (valid) {
        int32_t li = a.idx[i];
        z0 = (li >= 0 && li < a.n_lat) ? a.lat_z[li] : __builtin_nan("");
      }
    } else if (valid) {
      z0 = a.lat_z[i];
    }
    double x1 = 0, y1 = 0, z1 = 0, x2 = 0, y2 = 0, z2 = 0;
    if (valid) {
      x1 = a.x1[arc]; y1 = a.y1[arc]; z1 = a.z1[arc];
      x2 = a.x2[arc]; y2 = a.y2[arc]; z2 = a.z2[arc];
    }
    if (MODE) {
      o[j] = eval_eft(valid, x1, y1, z1, x2, y2, z2, z0, &sh.arena[MODE ? wave : 0][0],
                      [](bool need, auto&& fn) { resolve_serial(need, fn); });
      if (o[j].flags & F_INTERNAL) atomicOr(a.ws + 1, ERR_EXACT);
    } else {
      o[j] = eval_naive(valid, x1, y1, z1, x2, y2, z2, z0);
    }
    const int cnt = valid ? o[j].count : 0;
    o[j].count = cnt;
    const unsigned long long b1 = __ballot(cnt >= 1);
    const unsigned long long b2 = __ballot(cnt >= 2);
    woff[j] = __popcll(b1 & lt) + __popcll(b2 & lt);
    if (lane == 0) sh.wtot[j][wave] = __popcll(b1) + __popcll(b2);
  }
  __syncthreads();
  int boff[PPT];
  int agg = 0;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    boff[j] = agg;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
      int t = sh.wtot[j][w];
      boff[j] += w < wave ? t : 0;
      agg += t;
    }
  }
  if (tid == 0) sh.prefix = look_back(a.status, tile, agg, a.ws);
  __syncthreads();
  const int64_t prefix = sh.prefix;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t i = base + (int64_t)j * BLOCK + tid;
    const int cnt = o[j].count;
    const int64_t pos = prefix + boff[j] + woff[j];
    if (i < a.nnz) {
      a.ocount[i] = (uint8_t)cnt;
      if (a.oflags) a.oflags[i] = (uint8_t)o[j].flags;
    }
    if (cnt >= 1 && pos < a.cap) {
      a.ox[pos] = o[j].px0;
      a.oy[pos] = o[j].py0;
      a.opair[pos] = i;
      a.oroot[pos] = (uint8_t)o[j].r0;
    }
    if (cnt >= 2 && pos + 1 < a.cap) {
      a.ox[pos + 1] = o[j].px1;
      a.oy[pos + 1] = o[j].py1;
      a.opair[pos + 1] = i;
      a.oroot[pos + 1] = (uint8_t)o[j].r1;
    }
  }
  if (tid == 0 && tile == a.ntiles - 1) *a.ototal = prefix + agg;
}

// One workgroup per tile; tile ids in start order from the workspace counter.
template <int MODE, int PPT>
__global__ __launch_bounds__(BLOCK) void k_intersect(KArgs a) {
  __shared__ TileShared<MODE, PPT> sh;
  __shared__ int64_t s_tile;
  if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(a.ws, 1u);
  __syncthreads();
  run_tile<MODE, PPT>(a, s_tile, sh);
}

}  // namespace sphint
