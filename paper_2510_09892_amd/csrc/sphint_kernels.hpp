// gfx950 kernels for the arc x constant-latitude intersection (Sec. 2, Eq. 2.2; Alg. 8).
//
// One lane per arc-latitude pair.  A wavefront owns tiles of 64 * WPPT consecutive pairs
// (row j of a tile is pairs base + 64 j + lane) and evaluates them (naive or EFT), writing
// per-pair counts and flags at once.  Hits go into one dense output in pair order: a
// ballot/popcount scan inside the wavefront gives in-tile offsets, the wavefront publishes
// its tile's hit count, and one scanner wavefront per launch turns the counts into
// exclusive prefixes in tile order.  The grid is persistent and never larger than what the
// device holds at once, with a static tile order, so every tile the scanner waits for
// belongs to a running wavefront.  Hits wait in LDS until their tile's prefix is known and
// are then copied out in contiguous runs.  Rare undecided exact predicates are resolved one
// lane at a time per wavefront in an LDS arena (exact_sign).
#pragma once
#pragma clang fp contract(off)

#include "sphint_pair.hpp"

namespace sphint {

constexpr int BLOCK = 256;
constexpr int NWAVE = BLOCK / 64;
constexpr size_t WS_HEADER = 256;  // counter + error word, padded
constexpr uint64_t ST_AGG = 1, ST_PREFIX = 2;  // tile states (value << 2) | state
// Bounded waits: a wait gives up after KArgs::wait_ticks of the 100 MHz real-time counter
// (by default WAIT_TICKS = 2 s, far beyond any real wait; sphint_set_wait_limit changes it),
// sets ERR_SPIN, and every later wait of the launch gives up at once, so a launch always
// ends (with the error reported by sphint_check).
constexpr uint64_t WAIT_TICKS = 200000000ull;
enum : uint32_t { ERR_SPIN = 1u, ERR_EXACT = 2u };

struct KArgs {
  int64_t n_arcs, n_lat, nnz;
  const double *x1, *y1, *z1, *x2, *y2, *z2;
  const double* lat_z;
  const int64_t* off;
  const int32_t* idx;
  const uint32_t* parc;  // CSR: arc of each pair (in the workspace)
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
  uint64_t wait_ticks;  // limit of every bounded wait (real-time counter ticks)
};

// The same pointer in the global address space: argument pointers read from memory (the
// batched kernel's per-mesh tables) are otherwise generic, and generic (flat) accesses
// are slower and share a wait counter with scalar loads.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

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


// Ordered offsets across tiles.  A compute wavefront publishes its tile's hit count
// (aggregate) and later reads its exclusive prefix; one scanner wavefront per launch walks the
// tile states in order, up to K * 64 tiles per pass, and publishes the prefix of every tile
// whose predecessors have all reported; waiting wavefronts read only their own word.

// True when this wait must give up (timed out, or another wait of the launch did).
__device__ __forceinline__ bool wait_expired(uint64_t t0, unsigned& polls, uint32_t* ws,
                                             uint64_t ticks) {
  if ((++polls & 63u) == 0 &&
      (__hip_atomic_load(ws + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_SPIN))
    return true;
  if (__builtin_amdgcn_s_memrealtime() - t0 >= ticks) {
    atomicOr(ws + 1, ERR_SPIN);
    return true;
  }
  return false;
}

// Waits (lane 0 polls, bounded) until the scanner has published the tile's exclusive prefix.
__device__ __forceinline__ int64_t wait_prefix(uint64_t* status, int64_t tile, uint32_t* ws,
                                              uint64_t ticks) {
  const int lane = __lane_id();
  uint64_t w = 0;
  if (lane == 0) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    unsigned polls = 0;
    for (;;) {
      w = __hip_atomic_load(status + tile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((w & 3u) == ST_PREFIX) break;
      if (wait_expired(t0, polls, ws, ticks)) {
        w = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  w = __shfl(w, 0, 64);
  return (int64_t)(w >> 2);
}

// Decoupled look-back, the scanner's alternative (tile order is prefix order; a tile's state
// word goes 0 -> ST_AGG (its hit count) -> ST_INCL (its inclusive prefix)).  The exclusive
// prefix of `tile` is read from its predecessors: lane l of a window reads tile pos - l
// (tiles before 0 count as an inclusive prefix of 0); aggregates are summed up to the
// nearest inclusive prefix, which ends the walk, else the window moves 64 tiles back.  A
// window in which a tile before that point has not reported yet is read again (bounded
// wait, as wait_prefix).  The tile's own inclusive prefix is then published.  Every tile
// looked at belongs to a running wavefront that publishes its count without waiting for a
// later tile, so the walk ends.
constexpr uint64_t ST_INCL = 3;

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int64_t lookback_prefix(uint64_t* status, int64_t tile, int agg,
                                                   uint32_t* ws, uint64_t ticks) {
  const int lane = __lane_id();
  int64_t excl = 0;
  int64_t pos = tile - 1;
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  unsigned polls = 0;
  while (pos >= 0) {  // wavefront-uniform
    const int64_t j = pos - lane;
    const uint64_t w = j >= 0 ? __hip_atomic_load(status + j, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : ST_INCL;
    const unsigned st = (unsigned)(w & 3u);
    const unsigned long long incl = __ballot(st == ST_INCL);
    const int stop = incl ? __ffsll(incl) - 1 : 64;  // nearest inclusive prefix, if any
    const unsigned long long upto = stop >= 63 ? ~0ull : ((1ull << (stop + 1)) - 1);
    if (__ballot(st == 0u) & upto) {  // a tile before it has not reported yet
      bool quit = false;
      if (lane == 0) quit = wait_expired(t0, polls, ws, ticks);
      if (__shfl((int)quit, 0, 64)) {
        excl = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    excl += wave_sum(lane <= stop ? (int64_t)(w >> 2) : 0);
    if (stop < 64) break;
    pos -= 64;
    t0 = __builtin_amdgcn_s_memrealtime();
  }
  if (lane == 0)
    __hip_atomic_store(status + tile, ((uint64_t)(excl + agg) << 2) | ST_INCL, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// The scanner (one whole wavefront) for tiles [0, ntiles) of one call: publishes each tile's
// exclusive prefix in place of its aggregate and finally the call's total.  A pass reads
// K * 64 consecutive tile states with contiguous 512-byte loads, transposes them through
// `lds` (64 * (K + 1) words, padded against bank conflicts) so that lane l holds tiles
// t + K l ... t + K l + K - 1, sums within lanes, scans the 64 lane sums once, and writes
// the prefixes back the same way.
template <int K>
__device__ __forceinline__ int64_t lane_scan(int64_t v) {  // inclusive scan over the wave
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

template <int K>
__device__ __forceinline__ void scan_tiles(uint64_t* status, int64_t ntiles, int64_t* ototal,
                                           uint32_t* ws, uint64_t ticks, uint64_t* lds) {
  const int lane = __lane_id();
  constexpr int P = K + 1;  // padded row length of the transposed layout
  int64_t t = 0, run = 0;   // first tile without a prefix, hits before it
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  unsigned polls = 0;
  while (t < ntiles) {
    // coalesced loads, all issued before the first is used (no branch around them: indices
    // past the end read the last state, and are zeroed); word k * 64 + lane of the window
    // goes to lds[(q / K) * P + q % K]
    uint64_t wv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t j = t + k * 64 + lane;
      wv[k] = __hip_atomic_load(status + (j < ntiles ? j : ntiles - 1), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = k * 64 + lane;
      lds[(q / K) * P + q % K] = t + q < ntiles ? wv[k] : 0ull;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int ready = 0;  // leading entries of this lane that have reported
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t w = lds[lane * P + k];
      if (ready == k && (w & 3u) == ST_AGG) {
        ++ready;
        sum += (int64_t)(w >> 2);
      }
    }
    const unsigned long long full = __ballot(ready == K);
    const int L = full == ~0ull ? 64 : __ffsll(~full) - 1;  // first incomplete lane
    const int64_t v = lane <= L ? sum : 0;
    const int64_t inc = lane_scan<K>(v);
    int64_t ex = run + inc - v;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < K; ++k) {  // prefixes (state 0 = not published) back into lds
      const uint64_t w = lds[lane * P + k];
      uint64_t outw = 0;
      if (lane <= L && k < ready) {
        outw = ((uint64_t)ex << 2) | ST_PREFIX;
        ex += (int64_t)(w >> 2);
      }
      lds[lane * P + k] = outw;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = k * 64 + lane;
      const uint64_t w = lds[(q / K) * P + q % K];
      if (w) __hip_atomic_store(status + t + q, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int rL = __shfl(ready, L < 64 ? L : 63, 64);
    const int64_t advance = (int64_t)K * L + (L < 64 ? rL : 0);
    run += __shfl(inc, L < 64 ? L : 63, 64);
    __builtin_amdgcn_wave_barrier();
    if (advance == 0) {
      bool quit = false;
      if (lane == 0) quit = wait_expired(t0, polls, ws, ticks);
      if (__shfl((int)quit, 0, 64)) break;
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    t0 = __builtin_amdgcn_s_memrealtime();
    t += advance;
  }
  if (lane == 0) *ototal = run;
}

// ---------------------------------------------------------------- wavefront tiles
//
// A tile of WPPT * 64 consecutive pairs belongs to one wavefront: row j holds pairs
// base + 64 j + lane.  The wavefront evaluates the tile (writing counts and flags at once),
// publishes its hit count, and only then writes out the hits of its PREVIOUS tile, whose
// offset has had a whole tile's evaluation to arrive; those hits wait in an LDS buffer of
// the wavefront, from which they are copied to the output in contiguous (coalesced) runs.

// Hits of one pending tile, compacted in pair order.
template <int WPPT>
struct WaveStage {
  double x[2 * 64 * WPPT];
  double y[2 * 64 * WPPT];
  uint16_t pair[2 * 64 * WPPT];  // pair offset within the tile (bits 0-9), root (bit 15)
};

// Tiles per scanner lane per pass: the scanner borrows its own (unused) staging buffer.
template <int WPPT>
constexpr int scan_k() {
  return (int)(sizeof(WaveStage<WPPT>) / (64 * sizeof(uint64_t))) - 1;
}

// Workgroup LDS: one staging buffer per wavefront and one exact-arithmetic arena shared by
// the workgroup's wavefronts under a lock (exact evaluations are rare, and the arena's short
// dependent accesses want LDS latency).
template <int MODE, int WPPT, bool CSR>
struct WgShared {
  WaveStage<WPPT> stage[NWAVE];
  double arena[MODE ? xp::ARENA : 1];
  int lock;
};

__device__ __forceinline__ void lds_lock(int* l) {
  while (atomicCAS(l, 0, 1) != 0) __builtin_amdgcn_s_sleep(1);
}
__device__ __forceinline__ void lds_unlock(int* l) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  atomicExch(l, 0);
}

// Results of the tile being evaluated, held in registers.
template <int WPPT>
struct TileRegs {
  PairOut o[WPPT];
  int woff[WPPT];
  int agg;
  bool err;  // an exact sign overflowed its arena (reported once per tile)
};

// Inputs of one row (64 pairs, one per lane) of a tile; `o` is the pair's offset in the
// tile (the pair is tile base + o).
struct RowIn {
  double x1, y1, z1, x2, y2, z2, z0;
  int64_t arc;  // CSR: the pair's arc (clamped); rows evaluated from shared arc records
                // load only this, not the endpoints
  uint32_t o, oc;  // offset in the tile, offset read (the last pair's for lanes past the end)
  bool valid;
};

// Per-tile context for loading rows: the tile's first pair (wavefront-uniform, so that
// per-tile array bases live in scalar registers and lanes add 32-bit offsets).
struct TileCtx {
  int64_t base;
};

template <int WPPT, bool CSR>
__device__ __forceinline__ TileCtx tile_ctx(const KArgs& a, int64_t tile) {
  TileCtx c;
  c.base = tile * (int64_t)(64 * WPPT);
  return c;
}

// A row's slot: lane l holds pair j * 64 + l of the tile; lanes past the end read the last
// pair (and are marked invalid), so every load is unconditional and the compiler can count
// outstanding loads exactly.  Offsets stay below 1024 (a tile has at most 1024 pairs); the
// mask tells the compiler so, which lets it address from a scalar base plus a 32-bit lane
// offset.
struct RowSlot {
  uint32_t o, oc;  // offset in the tile, offset read
  bool valid;
};

__device__ __forceinline__ RowSlot row_slot(const KArgs& a, const TileCtx& c, int j) {
  RowSlot s;
  s.o = (uint32_t)(j * 64 + __lane_id()) & 1023u;
  s.valid = c.base + (int64_t)s.o < a.nnz;
  s.oc = (s.valid ? s.o : (uint32_t)(a.nnz - 1 - c.base)) & 1023u;
  return s;
}

// First level of a CSR row's loads: each pair's arc, from the pair-to-arc table that the
// init launch wrote, and its latitude index.  The gathers that depend on them (latitude,
// endpoints) are the second level, load_row; splitting the two lets a wavefront issue a
// row's first level one row before its second, so neither waits on the other.
struct RowIdx {
  uint32_t arc;
  int32_t li;
};

template <bool CSR>
__device__ __forceinline__ RowIdx load_idx(const KArgs& a, const TileCtx& c, int j) {
  RowIdx x = {0u, 0};
  if (CSR) {
    const RowSlot s = row_slot(a, c, j);
    x.arc = gptr(a.parc + c.base)[s.oc];
    x.li = gptr(a.idx + c.base)[s.oc];
  }
  return x;
}

// Loads one row (CSR: the second level, from the row's first-level values x; both are
// clamped, so malformed offsets or indices cannot send a read out of bounds).
template <bool CSR, bool SHARE = false>
__device__ __forceinline__ RowIn load_row(const KArgs& a, const TileCtx& c, int j,
                                          const RowIdx& x) {
  RowIn r;
  const RowSlot s = row_slot(a, c, j);
  r.o = s.o;
  r.oc = s.oc;
  r.valid = s.valid;
  if (CSR) {
    const int64_t pa = (int64_t)x.arc;
    const int64_t arc = pa < a.n_arcs ? pa : a.n_arcs - 1;
    const int32_t li = x.li;
    const bool ok = li >= 0 && li < a.n_lat;
    const double z = gptr(a.lat_z)[ok ? li : 0];
    r.z0 = ok ? z : __builtin_nan("");
    r.arc = arc;
    if (!SHARE) {
      r.x1 = gptr(a.x1)[arc]; r.y1 = gptr(a.y1)[arc]; r.z1 = gptr(a.z1)[arc];
      r.x2 = gptr(a.x2)[arc]; r.y2 = gptr(a.y2)[arc]; r.z2 = gptr(a.z2)[arc];
    }
  } else {
    const uint32_t oc = s.oc;
    r.z0 = gptr(a.lat_z + c.base)[oc];
    r.x1 = gptr(a.x1 + c.base)[oc]; r.y1 = gptr(a.y1 + c.base)[oc];
    r.z1 = gptr(a.z1 + c.base)[oc]; r.x2 = gptr(a.x2 + c.base)[oc];
    r.y2 = gptr(a.y2 + c.base)[oc]; r.z2 = gptr(a.z2 + c.base)[oc];
  }
  return r;
}

template <bool CSR, bool SHARE = false>
__device__ __forceinline__ RowIn load_row(const KArgs& a, const TileCtx& c, int j) {
  return load_row<CSR, SHARE>(a, c, j, load_idx<CSR>(a, c, j));
}

// CSR pair-to-arc table: parc[k] = the arc owning entry k.  Wavefront w of nw takes
// FILL_G * 64 consecutive arcs at a time and issues all their offset loads together
// (coalesced), so a wavefront waits for memory once per FILL_G groups of 64 arcs.  The
// entries of one group form one run [lo, hi); a window of FILL_W entries moves along it:
// every lane writes its own arc's entries inside the window into the wavefront's LDS
// buffer `win`, and the wavefront copies the window out with coalesced stores.  With
// monotone offsets the lanes' entries tile the window exactly.  Stores stay inside
// [lo, hi), clamped to [0, nnz), and LDS indices inside the window, so malformed
// offsets leave wrong arc ids in the table (clamped where they are read) but never
// reach outside either buffer.
constexpr int FILL_G = 4;    // groups of 64 arcs per load batch
constexpr int FILL_W = 512;  // window entries per wavefront (2 KB of LDS)

__device__ __forceinline__ void fill_pair_arcs(const int64_t* __restrict__ off, int64_t n_arcs,
                                               int64_t nnz, uint32_t* __restrict__ parc,
                                               int64_t w, int64_t nw, uint32_t* win) {
  const int lane = __lane_id();
  for (int64_t a0 = w * 64 * FILL_G; a0 < n_arcs; a0 += nw * 64 * FILL_G) {  // uniform
    int64_t b[FILL_G], e[FILL_G];
#pragma unroll
    for (int g = 0; g < FILL_G; ++g) {  // n_arcs >= 1 here, so the clamped index is valid
      const int64_t a = a0 + g * 64 + lane;
      const int64_t ac = a < n_arcs ? a : n_arcs - 1;
      b[g] = off[ac];
      e[g] = off[ac + 1];
    }
#pragma unroll
    for (int g = 0; g < FILL_G; ++g) {
      const int64_t ga = a0 + g * 64;
      if (ga >= n_arcs) break;  // wavefront-uniform
      const int64_t a = ga + lane;
      const bool ok = a < n_arcs;
      int64_t bb = ok ? b[g] : nnz, ee = ok ? e[g] : nnz;
      bb = bb < 0 ? 0 : (bb > nnz ? nnz : bb);
      ee = ee < bb ? bb : (ee > nnz ? nnz : ee);
      const int last = n_arcs - ga < 64 ? (int)(n_arcs - ga) - 1 : 63;
      const int64_t lo = __shfl(bb, 0, 64);
      const int64_t hi = __shfl(ee, last, 64);
      for (int64_t w0 = lo; w0 < hi; w0 += FILL_W) {  // wavefront-uniform
        const int64_t w1 = hi - w0 < FILL_W ? hi : w0 + FILL_W;
        const int64_t s = bb > w0 ? bb : w0;
        const int64_t t = ee < w1 ? ee : w1;
        for (int64_t q = s; q < t; ++q) win[(uint32_t)(q - w0) & (FILL_W - 1)] = (uint32_t)a;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int n = (int)(w1 - w0);
        for (int k = lane; k < n; k += 64) parc[w0 + k] = win[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
}

// Writes a row's counts and flags.  Every lane stores, so that the compiler can count the
// row's memory operations exactly and later waits for loads need not wait for these stores:
// a lane past the end holds the last pair (read at its slot `oc`), evaluated like the lane
// that owns it, so it writes the same bytes there.  Without a flags array the flags go to the
// count's byte first, and the count overwrites them (one lane's stores to one address stay
// in program order).
__device__ __forceinline__ void store_row(const KArgs& a, const TileCtx& c, const RowIn& in,
                                          const PairOut& o) {
  uint8_t* const fl = a.oflags ? a.oflags : a.ocount;
  gptr(fl + c.base)[in.oc] = (uint8_t)o.flags;
  gptr(a.ocount + c.base)[in.oc] = (uint8_t)o.count;
}

// Evaluates one row already loaded, writes its counts and flags, and accumulates the
// tile's in-order hit offsets.
template <int MODE, int WPPT, class Shared>
__device__ __forceinline__ void eval_row(const KArgs& a, const TileCtx& c, const RowIn& in, int j,
                                         TileRegs<WPPT>& r, Shared& sh) {
  const int lane = __lane_id();
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  PairOut& o = r.o[j];
  if (MODE) {
    o = eval_eft(true, in.x1, in.y1, in.z1, in.x2, in.y2, in.z2, in.z0, sh.arena,
                 [&](bool need, auto&& fn) {
                   resolve_serial(need, [&] {
                     lds_lock(&sh.lock);
                     fn();
                     lds_unlock(&sh.lock);
                   });
                 });
  } else {
    o = eval_naive(true, in.x1, in.y1, in.z1, in.x2, in.y2, in.z2, in.z0);
  }
  store_row(a, c, in, o);
  const int cnt = in.valid ? o.count : 0;
  o.count = cnt;
  const unsigned long long b1 = __ballot(cnt >= 1);
  const unsigned long long b2 = __ballot(cnt >= 2);
  const bool err = (o.flags & F_INTERNAL) != 0;
  r.err = j == 0 ? err : r.err || err;
  if (j == 0) r.agg = 0;
  r.woff[j] = r.agg + __popcll(b1 & lt) + __popcll(b2 & lt);
  r.agg += __popcll(b1) + __popcll(b2);
}

// ------------------------------------------------------ arc records shared in registers
//
// CSR lists hold an arc's candidates next to each other, so a few rows of a tile share a
// few dozen arcs.  With the arc part shared (EFT mode), a wavefront keeps a window of 64
// consecutive arcs of one mesh, lane l holding the record (ArcDec, ArcPts) of arc
// base + l, computed once by the whole wavefront; each lane of a row fetches its arc's
// record from the lane that holds it (ds_bpermute) instead of recomputing it from the
// endpoints.  A row whose arcs are not all in the window gets a new window starting at its
// first arc.  A row spanning more than 64 arc ids (arcs without candidates between its
// pairs) cannot share: every lane then computes its own arc's record into the window
// registers (the per-pair cost), and the next row starts a new window.

struct ArcWin {
  ArcDec d;
  ArcPts p;
  int64_t base;  // wavefront-uniform
  int mesh;      // mesh of the window (-1: none)
};

__device__ __forceinline__ double bperm_d(int addr, double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// addr = 4 * source lane; every lane of the wavefront must be active.
__device__ __forceinline__ ArcDec fetch_dec(const ArcDec& s, int addr) {
  ArcDec d;
  d.S2 = bperm_d(addr, s.S2); d.s2 = bperm_d(addr, s.s2);
  d.S3 = bperm_d(addr, s.S3); d.s3 = bperm_d(addr, s.s3);
  d.side = bperm_d(addr, s.side);
  d.z1 = bperm_d(addr, s.z1); d.z2 = bperm_d(addr, s.z2);
  d.n21 = bperm_d(addr, s.n21); d.n22 = bperm_d(addr, s.n22);
  d.meta = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)s.meta);
  return d;
}

__device__ __forceinline__ ArcPts fetch_pts(const ArcPts& s, int addr) {
  ArcPts p;
  p.Fx = bperm_d(addr, s.Fx); p.eFx = bperm_d(addr, s.eFx);
  p.Fy = bperm_d(addr, s.Fy); p.eFy = bperm_d(addr, s.eFy);
  p.nx = bperm_d(addr, s.nx); p.enx = bperm_d(addr, s.enx);
  p.ny = bperm_d(addr, s.ny); p.eny = bperm_d(addr, s.eny);
  return p;
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Each lane computes the record of arc `arc` (< a.n_arcs) into the window registers; open
// slope filters get exact signs one lane at a time.
template <class Shared>
__device__ __forceinline__ void fill_window(const KArgs& a, int64_t arc, ArcWin& w, Shared& sh) {
  const double x1 = gptr(a.x1)[arc], y1 = gptr(a.y1)[arc], z1 = gptr(a.z1)[arc];
  const double x2 = gptr(a.x2)[arc], y2 = gptr(a.y2)[arc], z2 = gptr(a.z2)[arc];
  int d1, d2;
  arc_shared(x1, y1, z1, x2, y2, z2, w.d, w.p, d1, d2);
  const bool open = d1 == UNDECIDED || d2 == UNDECIDED;
  unsigned meta = arc_meta(w.d.meta, d1, d2, false, false, false);
  resolve_serial(open, [&] {
    lds_lock(&sh.lock);
    meta = arc_resolve(w.d.meta, d1, d2, x1, y1, z1, x2, y2, z2, sh.arena);
    lds_unlock(&sh.lock);
  });
  w.d.meta = meta;
}

// eval_row for rows evaluated from arc records (EFT mode, CSR lists) of mesh m.
template <int WPPT, class Shared>
__device__ __forceinline__ void eval_row_shared(const KArgs& a, int m, const TileCtx& c,
                                                const RowIn& in, int j, TileRegs<WPPT>& r,
                                                Shared& sh, ArcWin& w) {
  const int lane = __lane_id();
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const unsigned long long vm = __ballot(in.valid);
  int64_t d = in.arc - w.base;
  if (__ballot(in.valid && w.mesh == m && d >= 0 && d < 64) != vm) {  // wavefront-uniform
    // the row's first arc (a row holds at least one valid pair)
    const int64_t b = readlane64(in.arc, __ffsll(vm) - 1);
    d = in.arc - b;
    if (__ballot(in.valid && d >= 0 && d < 64) == vm) {  // a new window holds the row
      const int64_t arc = b + lane;
      fill_window(a, arc < a.n_arcs ? arc : a.n_arcs - 1, w, sh);
      w.base = b;
      w.mesh = m;
    } else {  // every lane its own arc
      fill_window(a, in.arc, w, sh);
      d = lane;
      w.mesh = -1;
    }
  }
  int src = ((int)d & 63) << 2;
  auto xy = [&](int e) {
    return e == 1 ? dd{gptr(a.x1)[in.arc], gptr(a.y1)[in.arc]}
                  : dd{gptr(a.x2)[in.arc], gptr(a.y2)[in.arc]};
  };
  Decisions dec = {0, 0, 0, 0, 0};
  S2Eft S;
  PairOut& o = r.o[j];
  ArcDec D = fetch_dec(w.d, src);
  o = decide_shared<false>(in.valid, D, in.z0, dec, S, xy);
  const bool need = (o.flags & F_NEEDEXACT) != 0;
  if (__ballot(need)) {  // rare
    // Exact signs for the open decisions.  The window is made again afterwards (every lane
    // its own arc), so none of its registers has to survive the expansion arithmetic.
    bool ok = true;
    const unsigned meta = D.meta;
    resolve_serial(need, [&] {
      const int64_t k = in.arc;
      lds_lock(&sh.lock);
      ok = resolve_exact_shared(dec, meta, gptr(a.x1)[k], gptr(a.y1)[k], gptr(a.z1)[k],
                                gptr(a.x2)[k], gptr(a.y2)[k], gptr(a.z2)[k], in.z0, sh.arena);
      lds_unlock(&sh.lock);
    });
    fill_window(a, in.arc, w, sh);
    w.mesh = -1;
    src = lane << 2;
    D = fetch_dec(w.d, src);
    if (need) {
      o = decide_shared<true>(in.valid, D, in.z0, dec, S, xy);
      if (!ok) o.flags |= F_INTERNAL;
    }
  }
  // every lane runs the points (their terms come from other lanes, which must all be
  // active); only lanes with hits keep them
  PairOut q = o;
  points_eft_g(
      [&](int k) {
        switch (k) {
          case 0: return bperm_d(src, w.p.Fx);
          case 1: return bperm_d(src, w.p.eFx);
          case 2: return bperm_d(src, w.p.Fy);
          case 3: return bperm_d(src, w.p.eFy);
          case 4: return bperm_d(src, w.p.nx);
          case 5: return bperm_d(src, w.p.enx);
          case 6: return bperm_d(src, w.p.ny);
          default: return bperm_d(src, w.p.eny);
        }
      },
      D.S2, in.z0, S, q);
  if (o.count) o = q;
  // only valid lanes store here: the window fills already leave the compiler unsure how many
  // memory operations a row issues, so unconditional stores would gain nothing
  const int cnt = in.valid ? o.count : 0;
  o.count = cnt;
  if (in.valid) {
    gptr(a.ocount + c.base)[in.o] = (uint8_t)cnt;
    if (a.oflags) gptr(a.oflags + c.base)[in.o] = (uint8_t)o.flags;
  }
  const unsigned long long b1 = __ballot(cnt >= 1);
  const unsigned long long b2 = __ballot(cnt >= 2);
  const bool err = (o.flags & F_INTERNAL) != 0;
  r.err = j == 0 ? err : r.err || err;
  if (j == 0) r.agg = 0;
  r.woff[j] = r.agg + __popcll(b1 & lt) + __popcll(b2 & lt);
  r.agg += __popcll(b1) + __popcll(b2);
}

// Moves row j's hits from registers into the wavefront's staging buffer.
template <int WPPT>
__device__ __forceinline__ void stage_row(const TileRegs<WPPT>& r, int j, WaveStage<WPPT>& st) {
  const int lane = __lane_id();
  const PairOut& o = r.o[j];
  const int p = r.woff[j];
  const uint16_t off = (uint16_t)(j * 64 + lane);
  if (o.count >= 1) {
    st.x[p] = o.px0;
    st.y[p] = o.py0;
    st.pair[p] = (uint16_t)(off | (o.r0 << 15));
  }
  if (o.count >= 2) {
    st.x[p + 1] = o.px1;
    st.y[p + 1] = o.py1;
    st.pair[p + 1] = (uint16_t)(off | (o.r1 << 15));
  }
}

// Copies a staged tile's `count` hits to the output at offset `prefix` (coalesced).
template <int WPPT>
__device__ __forceinline__ void flush_tile(const KArgs& a, int64_t tile, int count, int64_t prefix,
                                           const WaveStage<WPPT>& st) {
  const int lane = __lane_id();
  const int64_t base = tile * (int64_t)(64 * WPPT);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // hits [prefix, prefix + count) clipped to the capacity, from uniform bases
  const int64_t room = a.cap - prefix;
  const int n = room <= 0 ? 0 : (room < count ? (int)room : count);
  double* ox = a.ox + prefix;
  double* oy = a.oy + prefix;
  int64_t* op = a.opair + prefix;
  uint8_t* orr = a.oroot + prefix;
  for (int k = lane; k < n; k += 64) {  // k < 2 * 64 * WPPT <= 2048
    const uint32_t kk = (uint32_t)k & 2047u;
    gptr(ox)[kk] = st.x[kk];
    gptr(oy)[kk] = st.y[kk];
    const uint32_t w = st.pair[kk];
    gptr(op)[kk] = base + (w & 1023u);
    gptr(orr)[kk] = (uint8_t)(w >> 15);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The exclusive prefix of a finished tile: published by the scanner (LB == false), or found
// by decoupled look-back (LB == true; the owner of a call's last tile then writes its total).
template <bool LB>
__device__ __forceinline__ int64_t tile_prefix(const KArgs& a, int64_t tile, int agg) {
  if (!LB) return wait_prefix(a.status, tile, a.ws, a.wait_ticks);
  const int64_t prefix = lookback_prefix(a.status, tile, agg, a.ws, a.wait_ticks);
  if (tile == a.ntiles - 1 && __lane_id() == 0) *a.ototal = prefix + agg;
  return prefix;
}

// One wavefront's share of the tiles: tiles come from `next` (the KArgs index and local
// tile, or false when done).  Loads run one row ahead of evaluation (the next tile's first
// row is fetched while the current tile's last row is evaluated); a CSR row's first-level
// loads run two rows ahead.  A tile's hit count is
// published when its last row is done; the previous tile's hits are written out after the
// first FLUSH_AT rows of the next tile, which gives the scanner that much time to publish
// its offset.  Rows evaluated after that point go straight to the staging buffer, so at most
// FLUSH_AT rows of results are held in registers.
template <int MODE, int WPPT, bool CSR, int FLUSH_AT, bool LB, bool SHARE = false, class Next>
__device__ __forceinline__ void wave_loop(const KArgs* args, WgShared<MODE, WPPT, CSR>& sh,
                                          Next&& next) {
  static_assert(!SHARE || (MODE == 1 && CSR), "arc records are shared in EFT mode over CSR lists");
  static_assert(FLUSH_AT >= 1 && FLUSH_AT <= WPPT, "flush point inside the tile");
  static_assert(WPPT <= 16, "pair and hit offsets within a tile are masked to 10 and 11 bits");
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  WaveStage<WPPT>& st = sh.stage[wave];
  bool pending = false;
  int pm = 0, pagg = 0;
  int64_t ptile = 0;
  int m = 0, m2 = 0;
  int64_t tile = 0, tile2 = 0;
  TileRegs<WPPT> r;
  bool have = next(m, tile);
  if (!have) return;
  m = __builtin_amdgcn_readfirstlane(m);  // wavefront-uniform: the arguments load as scalars
  TileCtx ctx = tile_ctx<WPPT, CSR>(args[m], tile), ctx2;
  RowIn cur = load_row<CSR, SHARE>(args[m], ctx, 0), nxt;
  // CSR rows with two or more rows per tile: the first-level loads of the row after the
  // next one (ix) are in flight while the next row's gathers are issued from the values
  // loaded a row earlier.  Not with shared arc records below four rows per tile: those
  // kernels sit at the register limit of four wavefronts per SIMD, where the extra row in
  // flight spills.
  constexpr bool PIPE = CSR && WPPT >= 2 && (!SHARE || WPPT >= 4);
  RowIdx ix = load_idx<PIPE>(args[m], ctx, 1);
  ArcWin win;
  win.base = 0;
  win.mesh = -1;
  // the next tile, fetched one row before the end of this one (PIPE) or at its last row;
  // past the last tile the fetches repeat this tile (unused)
  auto fetch_tile = [&]() {
    const bool h = next(m2, tile2);
    if (!h) {
      m2 = m;
      tile2 = tile;
    }
    m2 = __builtin_amdgcn_readfirstlane(m2);
    ctx2 = tile_ctx<WPPT, CSR>(args[m2], tile2);
    return h;
  };
  while (have) {
    const KArgs& a = args[m];
    bool have2 = false;
#pragma unroll
    for (int j = 0; j < WPPT; ++j) {
      if constexpr (PIPE) {
        if (j + 1 < WPPT)
          nxt = load_row<CSR, SHARE>(a, ctx, j + 1, ix);
        else
          nxt = load_row<CSR, SHARE>(args[m2], ctx2, 0, ix);
        if (j + 2 < WPPT) {
          ix = load_idx<CSR>(a, ctx, j + 2);
        } else if (j + 2 == WPPT) {
          have2 = fetch_tile();
          ix = load_idx<CSR>(args[m2], ctx2, 0);
        } else {
          ix = load_idx<CSR>(args[m2], ctx2, 1);
        }
      } else if (j + 1 < WPPT) {
        nxt = load_row<CSR, SHARE>(a, ctx, j + 1);
      } else {
        have2 = fetch_tile();
        nxt = load_row<CSR, SHARE>(args[m2], ctx2, 0);
      }
      if constexpr (SHARE)
        eval_row_shared<WPPT>(a, m, ctx, cur, j, r, sh, win);
      else
        eval_row<MODE, WPPT>(a, ctx, cur, j, r, sh);
      if (j + 1 == FLUSH_AT) {
        if (pending) {
          const KArgs& pa = args[pm];
          const int64_t prefix = tile_prefix<LB>(pa, ptile, pagg);
          flush_tile<WPPT>(pa, ptile, pagg, prefix, st);
        }
#pragma unroll
        for (int jj = 0; jj <= j; ++jj) stage_row<WPPT>(r, jj, st);
      } else if (j + 1 > FLUSH_AT) {
        stage_row<WPPT>(r, j, st);
      }
      cur = nxt;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (__lane_id() == 0)
      __hip_atomic_store(a.status + tile, ((uint64_t)r.agg << 2) | ST_AGG, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (MODE && __ballot(r.err) && __lane_id() == 0) atomicOr(a.ws + 1, ERR_EXACT);
    pending = true;
    pm = m;
    ptile = tile;
    pagg = r.agg;
    have = have2;
    m = m2;
    tile = tile2;
    ctx = ctx2;
  }
  if (pending) {
    const KArgs& pa = args[pm];
    const int64_t prefix = tile_prefix<LB>(pa, ptile, pagg);
    flush_tile<WPPT>(pa, ptile, pagg, prefix, st);
  }
}

// Rows evaluated before the previous tile is written out, i.e. held in registers while the
// scanner publishes that tile's offset: two (one with shared arc records, whose window
// already takes the registers, and in one-row tiles).
template <int MODE, int WPPT, bool SHARE = false>
constexpr int flush_at() {
  return (MODE && SHARE) || WPPT < 2 ? 1 : 2;
}

// Persistent wavefronts with a static order.  The grid never exceeds what the device holds
// at once, so every tile the scanner waits on belongs to a running wavefront; there is no
// atomic tile counter (a single contended address serialises at tens of millions of
// operations per second).  The last wavefront of the grid is the scanner; compute wavefront
// c of the other W takes tiles c, c + W, c + 2W, ...
template <int MODE, int WPPT, bool CSR, bool SHARE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_intersect_w(KArgs a) {
  __shared__ WgShared<MODE, WPPT, CSR> sh;
  if (threadIdx.x == 0) sh.lock = 0;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int64_t gw = (int64_t)blockIdx.x * NWAVE + wave;
  const int64_t W = (int64_t)gridDim.x * NWAVE - 1;
  if (gw == W) {
    // The scanner shares its SIMD with compute wavefronts; at the default priority it gets
    // a fraction of the issue slots and every tile's prefix waits on it.
    __builtin_amdgcn_s_setprio(3);
    scan_tiles<scan_k<WPPT>()>(a.status, a.ntiles, a.ototal, a.ws, a.wait_ticks,
                               reinterpret_cast<uint64_t*>(&sh.stage[wave]));
    return;
  }
  int64_t t = gw;
  wave_loop<MODE, WPPT, CSR, flush_at<MODE, WPPT, SHARE>(), false, SHARE>(&a, sh, [&](int& m, int64_t& tile) {
    if (t >= a.ntiles) return false;
    m = 0;
    tile = t;
    t += W;
    return true;
  });
}

}  // namespace sphint
