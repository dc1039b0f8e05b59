// Host-side helpers shared by the single-call and batched entry points.
#pragma once

#include <hip/hip_runtime.h>

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

inline KArgs make_args(int64_t n_arcs, const sphint_pts_soa& p1, const sphint_pts_soa& p2,
                       const double* lat_z, int64_t n_lat, const int64_t* off,
                       const int32_t* idx, int64_t nnz, const sphint_hits& out,
                       uint8_t* out_count, uint8_t* out_flags, int64_t* out_total,
                       uint32_t* ws, uint64_t* status, int64_t ntiles) {
  KArgs k;
  k.n_arcs = n_arcs;
  k.n_lat = n_lat;
  k.nnz = nnz;
  k.x1 = p1.x; k.y1 = p1.y; k.z1 = p1.z;
  k.x2 = p2.x; k.y2 = p2.y; k.z2 = p2.z;
  k.lat_z = lat_z;
  k.off = off;
  k.idx = off ? idx : nullptr;
  k.ox = out.x; k.oy = out.y; k.opair = out.pair; k.oroot = out.root; k.cap = out.capacity;
  k.ocount = out_count;
  k.oflags = out_flags;
  k.ototal = out_total;
  k.ws = ws;
  k.status = status;
  k.ntiles = ntiles;
  return k;
}

}  // namespace sphint
