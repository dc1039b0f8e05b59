/*
 * A plain C client of libsphint: the public header and the HIP runtime API, nothing else.
 *
 *   sphint_client IN OUT
 *
 * IN holds n (int64) and then seven arrays of n binary64 values: x1, y1, z1, x2, y2, z2, z0
 * (n dense arc-latitude pairs).  For each mode (naive, then EFT) the client copies them to
 * device memory, sizes and allocates the workspace with sphint_workspace_size, calls
 * sphint_arc_constlat on a stream of its own, reads the total back, asks sphint_check, and
 * then repeats the call with a hit capacity one short of the total, which sphint_check
 * must report as SPHINT_E_CAPACITY with the same total.  It also checks that a call with
 * a missing count array is refused with SPHINT_E_INVAL.
 *
 * OUT receives, per mode: int32 status of the call, int32 status of sphint_check, int32
 * status of the short-capacity check, int32 status of the refused call, int64 total, int64
 * total of the short-capacity call, n uint8 counts, n uint8 flags, and total binary64 x,
 * total binary64 y, total int64 pair indices and total uint8 roots.
 *
 * Exit status 0 when every HIP call succeeded (the library's statuses are reported, not
 * judged, here), 1 on bad usage or input, 2 on a HIP error.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "sphint.h"

#define HIP_OK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      fprintf(stderr, "%s:%d: %s: %s\n", __FILE__, __LINE__, #call,               \
              hipGetErrorString(e_));                                             \
      exit(2);                                                                    \
    }                                                                             \
  } while (0)

static void *dev_copy(const void *host, size_t bytes) {
  void *d = NULL;
  HIP_OK(hipMalloc(&d, bytes > 0 ? bytes : 1));
  if (bytes > 0) HIP_OK(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  return d;
}

static void put(FILE *f, const void *p, size_t bytes) {
  if (bytes > 0 && fwrite(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "write failed\n");
    exit(1);
  }
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
    return 1;
  }
  FILE *in = fopen(argv[1], "rb");
  if (!in) {
    perror(argv[1]);
    return 1;
  }
  int64_t n = 0;
  if (fread(&n, sizeof n, 1, in) != 1 || n <= 0 || n > ((int64_t)1 << 28)) {
    fprintf(stderr, "bad pair count\n");
    return 1;
  }
  double *host[7];
  for (int k = 0; k < 7; ++k) {
    host[k] = (double *)malloc((size_t)n * sizeof(double));
    if (!host[k] || fread(host[k], sizeof(double), (size_t)n, in) != (size_t)n) {
      fprintf(stderr, "short input\n");
      return 1;
    }
  }
  fclose(in);
  FILE *out = fopen(argv[2], "wb");
  if (!out) {
    perror(argv[2]);
    return 1;
  }

  double *dev[7];
  for (int k = 0; k < 7; ++k) dev[k] = (double *)dev_copy(host[k], (size_t)n * sizeof(double));
  const sphint_pts_soa p1 = {dev[0], dev[1], dev[2]};
  const sphint_pts_soa p2 = {dev[3], dev[4], dev[5]};
  const int64_t cap = 2 * n;  /* always enough */
  sphint_hits hits;
  HIP_OK(hipMalloc((void **)&hits.x, (size_t)cap * sizeof(double)));
  HIP_OK(hipMalloc((void **)&hits.y, (size_t)cap * sizeof(double)));
  HIP_OK(hipMalloc((void **)&hits.pair, (size_t)cap * sizeof(int64_t)));
  HIP_OK(hipMalloc((void **)&hits.root, (size_t)cap));
  hits.capacity = cap;
  uint8_t *count = NULL, *flags = NULL;
  int64_t *total = NULL;
  HIP_OK(hipMalloc((void **)&count, (size_t)n));
  HIP_OK(hipMalloc((void **)&flags, (size_t)n));
  HIP_OK(hipMalloc((void **)&total, sizeof(int64_t)));
  const size_t ws_bytes = sphint_workspace_size(n);
  void *ws = NULL;
  HIP_OK(hipMalloc(&ws, ws_bytes));  /* hipMalloc returns 256-byte aligned memory */
  hipStream_t stream;
  HIP_OK(hipStreamCreate(&stream));

  uint8_t *hc = (uint8_t *)malloc((size_t)n), *hf = (uint8_t *)malloc((size_t)n);
  double *hx = (double *)malloc((size_t)cap * sizeof(double));
  double *hy = (double *)malloc((size_t)cap * sizeof(double));
  int64_t *hp = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
  uint8_t *hr = (uint8_t *)malloc((size_t)cap);
  if (!hc || !hf || !hx || !hy || !hp || !hr) {
    fprintf(stderr, "host allocation failed\n");
    return 1;
  }

  const sphint_mode modes[2] = {SPHINT_NAIVE_FP64, SPHINT_EFT_FP64};
  for (int m = 0; m < 2; ++m) {
    int32_t st_call = (int32_t)sphint_arc_constlat(n, p1, p2, dev[6], n, NULL, NULL, n, hits,
                                                   count, flags, total, modes[m], ws, ws_bytes,
                                                   (void *)stream);
    HIP_OK(hipStreamSynchronize(stream));
    int64_t t = -1;
    HIP_OK(hipMemcpy(&t, total, sizeof t, hipMemcpyDeviceToHost));
    int32_t st_check = (int32_t)sphint_check(ws, t, cap);
    if (t < 0 || t > cap) {
      fprintf(stderr, "total %lld outside [0, %lld]\n", (long long)t, (long long)cap);
      return 1;
    }
    HIP_OK(hipMemcpy(hc, count, (size_t)n, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hf, flags, (size_t)n, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hx, hits.x, (size_t)t * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hy, hits.y, (size_t)t * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hp, hits.pair, (size_t)t * sizeof(int64_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hr, hits.root, (size_t)t, hipMemcpyDeviceToHost));

    /* one hit short: the call still runs, writes stop at the capacity, the total is exact */
    sphint_hits shorter = hits;
    shorter.capacity = t > 0 ? t - 1 : 0;
    int64_t t2 = -1;
    int32_t st_short = (int32_t)sphint_arc_constlat(n, p1, p2, dev[6], n, NULL, NULL, n,
                                                    shorter, count, flags, total, modes[m],
                                                    ws, ws_bytes, (void *)stream);
    HIP_OK(hipStreamSynchronize(stream));
    HIP_OK(hipMemcpy(&t2, total, sizeof t2, hipMemcpyDeviceToHost));
    if (st_short == SPHINT_OK) st_short = (int32_t)sphint_check(ws, t2, shorter.capacity);

    /* refused before any launch: the count array is required */
    int32_t st_inval = (int32_t)sphint_arc_constlat(n, p1, p2, dev[6], n, NULL, NULL, n, hits,
                                                    NULL, flags, total, modes[m], ws, ws_bytes,
                                                    (void *)stream);

    put(out, &st_call, sizeof st_call);
    put(out, &st_check, sizeof st_check);
    put(out, &st_short, sizeof st_short);
    put(out, &st_inval, sizeof st_inval);
    put(out, &t, sizeof t);
    put(out, &t2, sizeof t2);
    put(out, hc, (size_t)n);
    put(out, hf, (size_t)n);
    put(out, hx, (size_t)t * sizeof(double));
    put(out, hy, (size_t)t * sizeof(double));
    put(out, hp, (size_t)t * sizeof(int64_t));
    put(out, hr, (size_t)t);
  }
  if (fclose(out) != 0) {
    perror(argv[2]);
    return 1;
  }

  HIP_OK(hipStreamDestroy(stream));
  HIP_OK(hipFree(ws));
  HIP_OK(hipFree(total));
  HIP_OK(hipFree(flags));
  HIP_OK(hipFree(count));
  HIP_OK(hipFree(hits.root));
  HIP_OK(hipFree(hits.pair));
  HIP_OK(hipFree(hits.y));
  HIP_OK(hipFree(hits.x));
  for (int k = 0; k < 7; ++k) {
    HIP_OK(hipFree(dev[k]));
    free(host[k]);
  }
  free(hc);
  free(hf);
  free(hx);
  free(hy);
  free(hp);
  free(hr);
  return 0;
}
