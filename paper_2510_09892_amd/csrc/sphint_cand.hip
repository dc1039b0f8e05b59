// C-ABI entry points for building CSR candidate lists on the GPU (include/sphint.h).
//
// Two calls on one stream and one workspace:
//   sphint_candidates_count: per arc, the first candidate latitude and the count (one lane
//     per arc; the latitude table is staged in LDS, sized to it, when it has at most
//     LDS_LAT entries; both ends found by one lockstep binary search), per-block sums, one
//     block scanning the block sums, then every block writing its exclusive prefixes into
//     lat_offsets and the last one the total;
//   sphint_candidates_fill: lat_idx, written by wavefronts that take 64 arcs at a time and
//     write their entries together (coalesced), each entry finding its arc by a binary
//     search over the 64 arcs' offsets held one per lane.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "sphint.h"
#include "sphint_cand.hpp"
#include "sphint_host.hpp"

using namespace sphint;

namespace {

constexpr int CB = 256;                 // threads per block
constexpr int CPER = 4;                 // arcs per thread
constexpr int CARCS = CB * CPER;        // arcs per block
constexpr int LDS_LAT = 4096;           // latitude tables up to this size are staged in LDS
constexpr size_t CWS_HEADER = 256;

struct CandWs {
  int32_t* first;
  int32_t* count;
  int64_t* bsum;  // [n_blocks]
};

int64_t cand_blocks(int64_t n_arcs) { return (n_arcs + CARCS - 1) / CARCS; }

CandWs cand_ws(void* ws, int64_t n_arcs) {
  char* p = (char*)ws + CWS_HEADER;
  CandWs w;
  w.first = (int32_t*)p;
  p += ((4 * (size_t)n_arcs + 255) / 256) * 256;
  w.count = (int32_t*)p;
  p += ((4 * (size_t)n_arcs + 255) / 256) * 256;
  w.bsum = (int64_t*)p;
  return w;
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* lds) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6;
  if (__lane_id() == 0) lds[wave] = v;
  __syncthreads();
  int64_t s = 0;
  for (int w = 0; w < CB / 64; ++w) s += lds[w];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(CB) void k_cand_count(const double* __restrict__ x1,
                                                   const double* __restrict__ y1,
                                                   const double* __restrict__ z1,
                                                   const double* __restrict__ x2,
                                                   const double* __restrict__ y2,
                                                   const double* __restrict__ z2,
                                                   int64_t n_arcs, const double* __restrict__ lat_z,
                                                   int32_t n_lat, double pad, CandWs w) {
  extern __shared__ double lz[];  // n_lat entries when staged (sized at launch)
  __shared__ int64_t red[CB / 64];
  const bool staged = n_lat <= LDS_LAT;
  if (staged)
    for (int k = threadIdx.x; k < n_lat; k += CB) lz[k] = lat_z[k];
  __syncthreads();
  const double* table = staged ? lz : lat_z;
  int64_t s = 0;
  for (int k = 0; k < CPER; ++k) {
    const int64_t a = (int64_t)blockIdx.x * CARCS + k * CB + threadIdx.x;
    if (a < n_arcs) {
      int32_t f, c;
      arc_candidates(x1[a], y1[a], z1[a], x2[a], y2[a], z2[a], table, n_lat, pad, f, c);
      w.first[a] = f;
      w.count[a] = c;
      s += c;
    }
  }
  const int64_t t = block_sum(s, red);
  if (threadIdx.x == 0) w.bsum[blockIdx.x] = t;
}

// One block: exclusive scan of the block sums in place; the total goes to *nnz and to
// offsets[n_arcs].
__global__ __launch_bounds__(1024) void k_cand_scan_blocks(int64_t* bsum, int64_t n_blocks,
                                                           int64_t* nnz, int64_t* offsets,
                                                           int64_t n_arcs) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_blocks + 1023) / 1024;
  const int64_t b0 = t * per, b1 = b0 + per < n_blocks ? b0 + per : n_blocks;
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += bsum[b];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan of the 1024 partial sums
    const int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = t ? part[t - 1] : 0;
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t v = bsum[b];
    bsum[b] = run;
    run += v;
  }
  if (t == 1023) {
    *nnz = part[1023];
    offsets[n_arcs] = part[1023];
  }
}

// Every block: exclusive prefixes of its arcs' counts, from its block's base.
__global__ __launch_bounds__(CB) void k_cand_offsets(CandWs w, int64_t n_arcs, int64_t* offsets) {
  __shared__ int64_t wsum[CB / 64];
  // thread t owns arcs base + t * CPER .. + CPER - 1 (consecutive, so one scan orders them)
  const int64_t a0 = (int64_t)blockIdx.x * CARCS + (int64_t)threadIdx.x * CPER;
  int32_t c[CPER];
  int64_t s = 0;
  for (int k = 0; k < CPER; ++k) {
    c[k] = a0 + k < n_arcs ? w.count[a0 + k] : 0;
    s += c[k];
  }
  int64_t inc = s;  // inclusive scan over the wavefront
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t v = __shfl_up(inc, o, 64);
    if (__lane_id() >= o) inc += v;
  }
  const int wave = threadIdx.x >> 6;
  if (__lane_id() == 63) wsum[wave] = inc;
  __syncthreads();
  int64_t base = w.bsum[blockIdx.x];
  for (int v = 0; v < wave; ++v) base += wsum[v];
  int64_t run = base + inc - s;
  for (int k = 0; k < CPER; ++k) {
    if (a0 + k < n_arcs) offsets[a0 + k] = run;
    run += c[k];
  }
}

// lat_idx[q] for every entry q < capacity; 64 arcs per wavefront at a time.
__global__ __launch_bounds__(CB) void k_cand_fill(CandWs w, int64_t n_arcs,
                                                  const int64_t* __restrict__ offsets,
                                                  int32_t* __restrict__ lat_idx,
                                                  int64_t capacity) {
  const int lane = __lane_id();
  const int64_t wv = (int64_t)blockIdx.x * (CB / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (CB / 64);
  for (int64_t a0 = wv * 64; a0 < n_arcs; a0 += nw * 64) {  // wavefront-uniform loop
    const int64_t a = a0 + lane;
    const bool ok = a < n_arcs;
    const int64_t b = ok ? offsets[a] : INT64_MAX;
    const int32_t c = ok ? w.count[a] : 0;
    const int32_t f = ok ? w.first[a] : 0;
    const int last = n_arcs - a0 < 64 ? (int)(n_arcs - a0) - 1 : 63;
    const int64_t lo = __shfl(b, 0, 64);
    int64_t hi = __shfl(b, last, 64) + __shfl(c, last, 64);
    hi = hi < capacity ? hi : capacity;
    for (int64_t q0 = lo; q0 < hi; q0 += 64) {
      const int64_t q = q0 + lane;
      int l = 0;  // largest lane with b <= q
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const int64_t bc = __shfl(b, l + step, 64);
        if (bc <= q) l += step;
      }
      const int64_t bl = __shfl(b, l, 64);
      const int32_t cl = __shfl(c, l, 64);
      const int32_t fl = __shfl(f, l, 64);
      if (q < hi && q - bl < cl) lat_idx[q] = fl + (int32_t)(q - bl);
    }
  }
}

}  // namespace

extern "C" size_t sphint_candidates_workspace_size(int64_t n_arcs) {
  if (n_arcs < 0) n_arcs = 0;
  const size_t per = ((4 * (size_t)n_arcs + 255) / 256) * 256;
  return CWS_HEADER + 2 * per + 8 * (size_t)(cand_blocks(n_arcs) + 1);
}

extern "C" sphint_status sphint_candidates_count(int64_t n_arcs, sphint_pts_soa p1,
                                                 sphint_pts_soa p2, const double* lat_z,
                                                 int64_t n_lat, double pad,
                                                 int64_t* lat_offsets, int64_t* out_nnz,
                                                 void* workspace, size_t workspace_bytes,
                                                 void* stream) {
  if (n_arcs < 0 || n_lat < 0 || n_lat > 0x7fffffffLL || !lat_offsets || !out_nnz ||
      !(pad >= 0.0) || !workspace || !aligned256(workspace) ||
      workspace_bytes < sphint_candidates_workspace_size(n_arcs))
    return SPHINT_E_INVAL;
  if (n_arcs > 0 && (!p1.x || !p1.y || !p1.z || !p2.x || !p2.y || !p2.z))
    return SPHINT_E_INVAL;
  if (n_arcs > 0 && n_lat > 0 && !lat_z) return SPHINT_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const CandWs w = cand_ws(workspace, n_arcs);
  const int64_t nb = cand_blocks(n_arcs);
  if (nb > 0x7fffffffLL) return SPHINT_E_INVAL;
  if (nb > 0) {
    // the latitude table in LDS only as large as it is: more workgroups fit on a CU
    const size_t lds = n_lat <= LDS_LAT ? 8 * (size_t)n_lat : 0;
    hipLaunchKernelGGL(k_cand_count, dim3((unsigned)nb), dim3(CB), lds, st, p1.x, p1.y, p1.z,
                       p2.x, p2.y, p2.z, n_arcs, lat_z, (int32_t)n_lat, pad, w);
    if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  }
  hipLaunchKernelGGL(k_cand_scan_blocks, dim3(1), dim3(1024), 0, st, w.bsum, nb, out_nnz,
                     lat_offsets, n_arcs);
  if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  if (nb > 0) {
    hipLaunchKernelGGL(k_cand_offsets, dim3((unsigned)nb), dim3(CB), 0, st, w, n_arcs,
                       lat_offsets);
    if (hipGetLastError() != hipSuccess) return SPHINT_E_HIP;
  }
  return SPHINT_OK;
}

extern "C" sphint_status sphint_candidates_fill(int64_t n_arcs, const int64_t* lat_offsets,
                                                int32_t* lat_idx, int64_t capacity,
                                                void* workspace, size_t workspace_bytes,
                                                void* stream) {
  if (n_arcs < 0 || capacity < 0 || !lat_offsets || (capacity > 0 && !lat_idx) || !workspace ||
      !aligned256(workspace) || workspace_bytes < sphint_candidates_workspace_size(n_arcs))
    return SPHINT_E_INVAL;
  if (n_arcs == 0 || capacity == 0) return SPHINT_OK;
  hipStream_t st = (hipStream_t)stream;
  const CandWs w = cand_ws(workspace, n_arcs);
  int64_t blocks = (n_arcs + CB - 1) / CB;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_cand_fill, dim3((unsigned)blocks), dim3(CB), 0, st, w, n_arcs,
                     lat_offsets, lat_idx, capacity);
  return hipGetLastError() == hipSuccess ? SPHINT_OK : SPHINT_E_HIP;
}
