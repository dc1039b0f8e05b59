// Host-side helpers shared by the single-call and batched entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "sphint.h"
#include "sphint_kernels.hpp"

namespace sphint {

inline int64_t tiles_for(int64_t nnz, int ppt = 1) {
  const int64_t per = (int64_t)BLOCK * ppt;
  return nnz > 0 ? (nnz + per - 1) / per : 0;
}

inline int64_t wave_tiles_for(int64_t nnz, int wppt) {
  const int64_t per = (int64_t)64 * wppt;
  return nnz > 0 ? (nnz + per - 1) / per : 0;
}

inline bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// Events a caller asked to have recorded around the timed kernel of each call on this thread
// (sphint_set_profile_events): the main kernel of sphint_arc_constlat, pass 1 of
// sphint_arc_constlat_adaptive.
struct ProfileEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

inline ProfileEvents& profile_events() {
  static thread_local ProfileEvents ev;
  return ev;
}

// Compute units of the current device (queried once per device).
inline int device_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cached[dev].load(std::memory_order_relaxed);
  if (!c) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        c <= 0)
      c = 256;
    cached[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

// Workspace of one call over nnz pairs: header, one status word per tile of the finest
// schedule (64 pairs), then the CSR pair-to-arc table (4 bytes per pair).
inline size_t status_words_for(int64_t nnz) {
  const int64_t t = wave_tiles_for(nnz < 0 ? 0 : nnz, 1);
  return (size_t)(t > 0 ? t : 1);
}
inline size_t workspace_bytes_for(int64_t nnz) {
  return WS_HEADER + 8 * status_words_for(nnz) + 4 * (size_t)(nnz > 0 ? nnz : 0);
}

// Workgroup size of the init and pair-to-arc launches.
constexpr int INIT_BLOCK = 256;

// Workgroups for the pair-to-arc table of n_arcs arcs: one lane per FILL_G arcs, capped
// (the fill loops over the rest).
inline int64_t fill_blocks(int64_t n_arcs) {
  const int64_t lanes = (n_arcs + FILL_G - 1) / FILL_G;
  const int64_t b = (lanes + INIT_BLOCK - 1) / INIT_BLOCK;
  return b > 8192 ? 8192 : (b < 1 ? 1 : b);
}

// Argument checks shared by the single-call and batched paths.
inline sphint_status validate(int64_t n_arcs, const sphint_pts_soa& p1, const sphint_pts_soa& p2,
                              const double* lat_z, int64_t n_lat, const int64_t* off,
                              const int32_t* idx, int64_t nnz, const sphint_hits& out,
                              const uint8_t* out_count, const int64_t* out_total) {
  if (n_arcs < 0 || n_lat < 0 || nnz < 0 || out.capacity < 0) return SPHINT_E_INVAL;
  if (!out_total) return SPHINT_E_INVAL;
  const bool csr = off != nullptr || idx != nullptr;
  if (csr) {
    if (!off || (!idx && nnz > 0)) return SPHINT_E_INVAL;
    if (nnz > 0 && (n_arcs == 0 || n_lat == 0 || !lat_z)) return SPHINT_E_INVAL;
    if (n_arcs >= ((int64_t)1 << 32)) return SPHINT_E_INVAL;  // arc ids are 32-bit
  } else {
    if (n_lat != n_arcs || nnz != n_arcs) return SPHINT_E_INVAL;
  }
  if (nnz > 0) {
    if (!p1.x || !p1.y || !p1.z || !p2.x || !p2.y || !p2.z || !lat_z || !out_count)
      return SPHINT_E_INVAL;
  }
  if (out.capacity > 0 && (!out.x || !out.y || !out.pair || !out.root)) return SPHINT_E_INVAL;
  if (nnz > ((int64_t)1 << 40)) return SPHINT_E_INVAL;
  return SPHINT_OK;
}

// Limit of the kernels' bounded waits for launches enqueued from now on (real-time counter
// ticks, 100 MHz); sphint_set_wait_limit sets it.
inline std::atomic<uint64_t>& wait_ticks_setting() {
  static std::atomic<uint64_t> ticks{WAIT_TICKS};
  return ticks;
}

inline KArgs make_args(int64_t n_arcs, const sphint_pts_soa& p1, const sphint_pts_soa& p2,
                       const double* lat_z, int64_t n_lat, const int64_t* off,
                       const int32_t* idx, int64_t nnz, const sphint_hits& out,
                       uint8_t* out_count, uint8_t* out_flags, int64_t* out_total,
                       uint32_t* ws, uint64_t* status, int64_t ntiles, uint32_t* parc) {
  KArgs k;
  k.n_arcs = n_arcs;
  k.n_lat = n_lat;
  k.nnz = nnz;
  k.x1 = p1.x; k.y1 = p1.y; k.z1 = p1.z;
  k.x2 = p2.x; k.y2 = p2.y; k.z2 = p2.z;
  k.lat_z = lat_z;
  k.off = off;
  k.idx = off ? idx : nullptr;
  k.parc = off ? parc : nullptr;
  k.ox = out.x; k.oy = out.y; k.opair = out.pair; k.oroot = out.root; k.cap = out.capacity;
  k.ocount = out_count;
  k.oflags = out_flags;
  k.ototal = out_total;
  k.ws = ws;
  k.status = status;
  k.ntiles = ntiles;
  k.wait_ticks = wait_ticks_setting().load(std::memory_order_relaxed);
  return k;
}

// Cross-stream ordering of this library's launches on one device.  A persistent grid is
// sized to what the device holds at once and relies on all its workgroups being resident
// together (every wait inside a launch is on a tile of a running wavefront).  Two such
// launches running at once on different streams could each hold part of the device and
// wait for workgroups that the other keeps out, until the bounded waits give up.  So each
// launch waits for the previous launch of the device, on whatever stream that one ran (one
// event per device).  Launches being captured into a graph are not chained: a caller that
// replays graphs on several streams orders the replays itself.  The stream must belong to
// the current device.
struct ChainState {
  std::mutex m;
  hipEvent_t ev = nullptr;
  hipStream_t last = nullptr;
  bool armed = false;
};

inline ChainState& chain_state(int dev) {
  static ChainState s[64];
  return s[dev & 63];
}

class LaunchChain {
 public:
  LaunchChain() = default;
  LaunchChain(const LaunchChain&) = delete;
  LaunchChain& operator=(const LaunchChain&) = delete;
  ~LaunchChain() {
    if (c_) c_->m.unlock();
  }

  // Call before the launch: makes `st` wait for the device's previous launch.
  hipError_t begin(hipStream_t st) {
    st_ = st;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    ChainState& c = chain_state(dev);
    c.m.lock();
    c_ = &c;
    if (!c.ev) {
      e = hipEventCreateWithFlags(&c.ev, hipEventDisableTiming);
      if (e != hipSuccess) {
        c.ev = nullptr;
        return e;
      }
    }
    if (c.armed && c.last != st) return hipStreamWaitEvent(st, c.ev, 0);
    return hipSuccess;
  }

  // Call after the launch was enqueued: the next launch of the device waits for this one.
  hipError_t end() {
    if (!c_) return hipSuccess;
    hipError_t e = hipEventRecord(c_->ev, st_);
    if (e == hipSuccess) {
      c_->armed = true;
      c_->last = st_;
    }
    return e;
  }

 private:
  ChainState* c_ = nullptr;
  hipStream_t st_ = nullptr;
};

}  // namespace sphint
