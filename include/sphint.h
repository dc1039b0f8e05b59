/*
 * sphint: intersections of great-circle arcs with lines of constant latitude on MI355X.
 *
 * The operation (Chen, Ullrich & Panetta, "Fast and Accurate Intersections on a Sphere",
 * Sec. 1.2 problem definition and Sec. 2): given binary64 arc endpoints x1, x2 (any
 * nonzero length; the arc is the shorter great-circle path between x1/|x1| and x2/|x2|)
 * and a latitude z = z0, return the 0, 1 or 2 points P = (P_x, P_y, z0) of the unit
 * sphere where the arc meets the latitude circle.  Points follow Eq. (2.2):
 *
 *     P = -( z0 n_x n_z +- s n_y , z0 n_y n_z -+ s n_x ) / |n_xy|^2 ,
 *     n = x1 x x2,  s = sqrt(|n_xy|^2 - |n|^2 z0^2),
 *
 * root SPHINT_ROOT_PLUS taking the upper signs (the crossing where z increases along the
 * arc from x1 to x2) and SPHINT_ROOT_MINUS the lower signs.
 *
 * Modes:
 *   SPHINT_NAIVE_FP64  Eq. (2.2) operation by operation in binary64 (Sec. 4), with binary64
 *                      existence/containment tests that take the endpoint heights as the
 *                      raw z1, z2 (inputs assumed unit length).
 *   SPHINT_EFT_FP64    Alg. 8 (AccuX, Sec. 6) with error-free transformations (the normal's
 *                      compensated pairs renormalised before the sums of squares); hit
 *                      counts, roots and flags are exact (containment against the
 *                      normalised endpoints x_i/|x_i|; exact ties count, i.e. the arc is
 *                      closed); each point is within 4 * 2^-53 (max-norm) of the exact
 *                      intersection away from tangency (s well above 2^-53 |n|).
 *
 * Inputs must be finite for a result (non-finite inputs give 0 hits and
 * SPHINT_F_NONFINITE) and, for the exactness claims, nonzero magnitudes roughly within
 * [2^-150, 2^150] (no overflow or underflow in products of up to six inputs).
 *
 * Memory: every array argument is DEVICE memory owned by the caller; the library never
 * allocates on these calls.  Calls are asynchronous on `stream` (a hipStream_t; NULL is the
 * default stream): outputs are valid once the stream reaches the end of the call.  All
 * entry points are reentrant; concurrent calls must use distinct workspaces.
 *
 * Ordering across streams: each launch's grid is sized to what the device holds at once and
 * needs all of its workgroups resident together, so the library orders its launches on one
 * device across streams (every launch waits, on the device, for the previous launch of the
 * device, whatever stream that used).  Work of other libraries on other streams still
 * overlaps.  Launches recorded while a stream is being captured into a graph are not
 * ordered this way: replays of such graphs on different streams must not overlap.  The
 * stream must belong to the current device.
 */
#ifndef SPHINT_H
#define SPHINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SPHINT_NAIVE_FP64 = 0, SPHINT_EFT_FP64 = 1 } sphint_mode;

typedef enum {
  SPHINT_OK = 0,
  SPHINT_E_INVAL = 1,    /* invalid argument; nothing was launched */
  SPHINT_E_CAPACITY = 2, /* reported by sphint_check: *out_total exceeded out.capacity */
  SPHINT_E_HIP = 3,      /* a HIP runtime call failed */
  SPHINT_E_NOMEM = 4,    /* host allocation failed (plans only) */
  SPHINT_E_DEVICE = 5    /* the kernel reported an internal limit (see sphint_check) */
} sphint_status;

/* Per-pair flag bits (out_flags). */
#define SPHINT_F_EXISTS 1u    /* the great circle meets the latitude circle: s^2 >= 0 */
#define SPHINT_F_TANGENT 2u   /* s^2 == 0: the circles touch; a double root counted once */
#define SPHINT_F_DEGEN_N 4u   /* n == 0: zero, equal or antipodal endpoints */
#define SPHINT_F_HORIZ 8u     /* n_xy == 0, n != 0: the arc lies on the equator */
#define SPHINT_F_NONFINITE 16u/* an input is inf or nan */
/* Diagnostic bits (EFT mode only; not part of the result a pair is compared on): */
#define SPHINT_F_FALLBACK 32u /* a floating-point filter could not certify one of the pair's
                               * signs, which exact expansion arithmetic then decided */
#define SPHINT_F_INTERNAL 64u /* an exact evaluation outgrew its fixed buffer (inputs outside
                               * binary64's normal range); that sign was taken as 0, and
                               * sphint_check reports SPHINT_E_DEVICE for the call */

#define SPHINT_ROOT_PLUS 0
#define SPHINT_ROOT_MINUS 1

/* Structure-of-arrays endpoints: component k of point i is x[i], y[i], z[i]. */
typedef struct {
  const double *x, *y, *z;
} sphint_pts_soa;

/* Compacted hit output.  Hit j is (x[j], y[j], z0 of pair[j]); root[j] is SPHINT_ROOT_*.
 * Hits are ordered by pair index, and within a pair along the arc from x1 to x2.  Writes
 * stop at `capacity` hits (2 * number of pairs always suffices); *out_total still holds the
 * required count. */
typedef struct {
  double *x, *y;
  int64_t *pair;
  uint8_t *root;
  int64_t capacity;
} sphint_hits;

/*
 * Intersections for a batch of arc-latitude pairs.
 *
 * Pairs (Sec. 1.2 inputs x1, x2, z0):
 *   dense form  (lat_offsets == NULL, lat_idx == NULL): pair i is arc i with latitude
 *               lat_z[i]; n_lat must equal n_arcs and nnz must equal n_arcs.
 *   CSR form    pair k is (arc i, latitude lat_z[lat_idx[k]]) for k in
 *               [lat_offsets[i], lat_offsets[i+1]); lat_offsets has n_arcs + 1
 *               non-decreasing entries with lat_offsets[0] == 0 and lat_offsets[n_arcs] ==
 *               nnz; lat_idx has nnz entries in [0, n_lat); n_arcs < 2^32.  An
 *               out-of-range lat_idx entry yields a NONFINITE pair, not a memory access
 *               out of bounds; malformed offsets give unspecified pairs but never an
 *               access outside the arrays.
 * p1, p2      arc endpoints, n_arcs entries per component (device).
 * out         compacted hits (device); may have capacity 0 with NULL pointers.
 * out_count   [nnz] hit count per pair, 0..2 (device, required when nnz > 0).
 * out_flags   [nnz] SPHINT_F_* per pair (device, may be NULL).
 * out_total   one int64 (device): total hits of this call.
 * workspace   device memory of at least sphint_workspace_size(nnz) bytes, 256-byte
 *             aligned, used only by this call while it runs.
 * EFT calls in the CSR form with at least 2.5 candidates per arc on average
 * (2 * nnz >= 5 * n_arcs) evaluate each arc's z0-free part (Alg. 8's normal, norms and F
 * pairs, and the containment rule's slope signs) once per tile row window and share it
 * among the arc's candidates; the results are the same bytes either way.
 * Returns SPHINT_E_INVAL (no launch) for negative sizes, missing pointers, mismatched
 * dense sizes, n_arcs >= 2^32 in the CSR form, nnz > 2^40 or more than 2^31 - 1 tiles of
 * 192 (EFT) or 256 (naive) pairs, or a short workspace; SPHINT_E_HIP if a launch fails;
 * else SPHINT_OK.
 */
sphint_status sphint_arc_constlat(int64_t n_arcs, sphint_pts_soa p1, sphint_pts_soa p2,
                                  const double *lat_z, int64_t n_lat,
                                  const int64_t *lat_offsets, const int32_t *lat_idx,
                                  int64_t nnz, sphint_hits out, uint8_t *out_count,
                                  uint8_t *out_flags, int64_t *out_total, sphint_mode mode,
                                  void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes sphint_arc_constlat needs for `nnz` pairs (any mode or form):
 * 256 + 8 * max(1, ceil(nnz / 64)) + 4 * nnz (a header, one scan state per tile of the
 * finest schedule, and the CSR pair-to-arc table). */
size_t sphint_workspace_size(int64_t nnz);

/*
 * After the stream has completed a call that used `workspace`: SPHINT_E_DEVICE if a kernel
 * hit an internal limit (bounded wait or exact-arithmetic capacity), SPHINT_E_CAPACITY if
 * host_total (the value of *out_total copied back by the caller) exceeds capacity, else
 * SPHINT_OK.  Synchronous (reads 8 bytes of the workspace).
 */
sphint_status sphint_check(const void *workspace, int64_t host_total, int64_t capacity);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sphint_arc_constlat without a
 * workspace argument.  The same kernels run with the same results; their workspace (the
 * error word, the tile scan states and, for the CSR form, the pair-to-arc table) is a
 * static device array of SPHINT_NOALLOC_SCRATCH_BYTES inside the library, one per device,
 * held until the process ends.  Nothing is allocated on any call.
 *
 * Scratch a call takes: dense form 256 + 8 * max(1, ceil(nnz / 64)) bytes (up to about
 * 5.4e8 pairs), CSR form 256 + 8 * max(1, ceil(nnz / 64)) + 4 * nnz bytes (up to about
 * 1.6e7 pairs); a call that would need more returns SPHINT_E_INVAL before any launch.
 *
 * out_error  one int32 (device, may be NULL): after the call, 0, or the kernels' error bits
 *            (nonzero where sphint_check would report SPHINT_E_DEVICE).  Capacity overflow
 *            shows as *out_total > out.capacity, as for sphint_arc_constlat.
 * All calls on one device share that device's array, and each call starts by clearing what
 * it reads before writing it.  The library orders its own launches on a device across
 * streams, so calls made directly from one process do not overlap; calls recorded into
 * graphs (not ordered by the library) that run at the same time on one device race on the
 * array and give undefined results.  Other arguments and errors as sphint_arc_constlat.
 */
#define SPHINT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

sphint_status sphint_arc_constlat_noalloc(int64_t n_arcs, sphint_pts_soa p1, sphint_pts_soa p2,
                                          const double *lat_z, int64_t n_lat,
                                          const int64_t *lat_offsets, const int32_t *lat_idx,
                                          int64_t nnz, sphint_hits out, uint8_t *out_count,
                                          uint8_t *out_flags, int64_t *out_total,
                                          int32_t *out_error, sphint_mode mode, void *stream);

/*
 * Every wait inside a launch (a tile waiting for its output offset, the scanner waiting for
 * a tile's count) is bounded: past the limit it gives up, the launch finishes with its
 * outputs undefined, and sphint_check / sphint_batch_check report SPHINT_E_DEVICE.  This
 * sets the limit, in seconds (default 2; 0 makes every wait give up at its first check),
 * for calls enqueued afterwards from any thread (a batch plan takes the limit in force when
 * it is created or its schedule is set, and keeps it in its graph).  A launch whose grid does not become
 * resident in time (the device shared with other work) thus ends with an error instead of
 * waiting forever.  SPHINT_E_INVAL for a negative, non-finite or over-3600 value.
 */
sphint_status sphint_set_wait_limit(double seconds);

/*
 * Instrumentation.  While set (non-NULL), every sphint_arc_constlat call made from this host
 * thread records `start` (a hipEvent_t) on its stream immediately before its main kernel and
 * `stop` immediately after it, so the caller can time that kernel alone, and every
 * sphint_arc_constlat_adaptive call does the same around its pass 1; NULL, NULL stops it.
 * The events are owned by the caller.
 */
sphint_status sphint_set_profile_events(void *start, void *stop);

/* ------------------------------------------------------------------ batched meshes */

/* One independent mesh of a batch: the arguments of one CSR (or dense) call. */
typedef struct {
  int64_t n_arcs, n_lat, nnz;
  sphint_pts_soa p1, p2;
  const double *lat_z;
  const int64_t *lat_offsets; /* NULL for the dense form */
  const int32_t *lat_idx;
  sphint_hits out;
  uint8_t *out_count, *out_flags;
  int64_t *out_total;
} sphint_mesh_desc;

typedef struct sphint_plan sphint_plan;

/*
 * Plan for running many meshes in one persistent launch.  Copies the descriptors to the
 * device (the plan's own allocations: descriptor table, tile table, scan states) and
 * prepares the tile schedule.  All meshes of a plan must have the same form (all CSR or all
 * dense), else SPHINT_E_INVAL.  Each mesh's results equal a sphint_arc_constlat call on that
 * mesh alone.
 */
sphint_status sphint_batch_plan_create(const sphint_mesh_desc *meshes, int n_meshes,
                                       sphint_mode mode, sphint_plan **plan);
/* Times the plan's candidate schedules (pairs per thread 1-4 x persistent grid sizes x the
 * two ways of ordering tile offsets, see sphint_batch_set_scan; for an EFT plan over CSR
 * lists also with arc records shared, see sphint_batch_set_share) by running the whole batch
 * on `stream`, keeps the fastest, and synchronizes the stream;
 * reads/appends a text cache at cache_path (may be NULL) keyed by the plan's shape.  The
 * batch's outputs are overwritten (with the same values). */
sphint_status sphint_batch_autotune(sphint_plan *plan, const char *cache_path, void *stream);
/* Launches the plan on `stream`: the first launch captures the init and persistent kernels
 * into a HIP graph (on a stream of the plan's own), every launch replays it. */
sphint_status sphint_batch_launch(sphint_plan *plan, void *stream);
/* Schedule of the plan: pairs per lane (a wavefront tile is 64 * pairs_per_thread pairs) and
 * workgroups per compute unit of the persistent grid (0: as many as the CU holds; never more,
 * since the grid's wavefronts must all be resident). */
sphint_status sphint_batch_params(const sphint_plan *plan, int *pairs_per_thread,
                                  int *wg_per_cu);
/* Sets the schedule by hand (pairs_per_thread 1 to 4, or 5 on a plan with shared arc
 * records; wg_per_cu >= 0, capped at what a CU holds) instead of the autotuner's choice; the
 * next launch re-captures the graph. */
sphint_status sphint_batch_set_params(sphint_plan *plan, int pairs_per_thread, int wg_per_cu);
/* How tiles learn their offsets in the compacted outputs: 0 = one scanner wavefront turns the
 * tiles' hit counts into prefixes in tile order; 1 = decoupled look-back (each wavefront sums
 * its predecessors' counts back to the nearest published inclusive prefix and publishes its
 * own), which spares small tiles the wait on one scanner.  Results are identical.  Setting
 * it re-captures the graph at the next launch. */
sphint_status sphint_batch_scan(const sphint_plan *plan, int *lookback);
sphint_status sphint_batch_set_scan(sphint_plan *plan, int lookback);
/* Whether an EFT plan over CSR lists shares each arc's z0-free part among the arc's
 * candidates (Alg. 8's normal, norms and F pairs, and the slope signs of the containment
 * rule, Sec. 2, depend on the arc alone): 1 = a wavefront computes the records of 64
 * consecutive arcs once, one arc per lane, and every pair of a tile row fetches its arc's
 * record from the lane holding it; 0 = every pair computes its arc's part (the single-call
 * path).  Results are identical, bit for bit.  SPHINT_E_INVAL for share = 1 on a naive or
 * dense plan, and for share = 0 while the plan has 5 pairs per thread (a shared-only tile
 * size).  Setting it re-captures the graph at the next launch. */
sphint_status sphint_batch_share(const sphint_plan *plan, int *share);
sphint_status sphint_batch_set_share(sphint_plan *plan, int share);
/* After the stream has completed a launch of the plan: SPHINT_E_DEVICE if a kernel of that
 * launch reported an internal limit (as sphint_check), else SPHINT_E_CAPACITY if some mesh's
 * *out_total exceeds its out.capacity, else SPHINT_OK.  Synchronous (reads the plan's error
 * word and every mesh's total). */
sphint_status sphint_batch_check(const sphint_plan *plan);
void sphint_plan_destroy(sphint_plan *plan);

/*
 * One-shot batched launch, for continuous batching (a request loop whose set of meshes
 * changes on every launch): up to SPHINT_BATCH_RUN_MAX meshes of one form (all CSR or all
 * dense) in one persistent launch, without a plan.  The meshes' arguments travel to the
 * device with the launch (as kernel arguments), so the call allocates nothing and does not
 * synchronise: an init kernel writes them into `workspace`, clears the tile states and
 * fills the CSR pair-to-arc tables, and the plan's persistent batched kernel follows on
 * `stream` (pairs per lane as in sphint_arc_constlat; EFT launches over CSR lists holding
 * at least 2.5 candidates per arc in all share arc records, as single calls do).  Each
 * mesh's outputs equal a sphint_arc_constlat call on that mesh alone.
 *
 * workspace   device memory of at least sphint_batch_run_workspace_size(n_meshes, sum of
 *             the meshes' nnz) bytes, 256-byte aligned, used only by this launch while it
 *             runs (a later launch on the same stream may reuse it).  After the stream has
 *             completed the launch, sphint_check(workspace, total, capacity) reports the
 *             kernels' error word for every mesh of the launch.
 * SPHINT_E_INVAL (no launch) for n_meshes outside [1, SPHINT_BATCH_RUN_MAX], mixed forms, a
 * mesh that sphint_arc_constlat would reject, more than 2^40 pairs in all or a short or
 * misaligned workspace; SPHINT_E_HIP if a launch fails.
 */
#define SPHINT_BATCH_RUN_MAX 16

size_t sphint_batch_run_workspace_size(int n_meshes, int64_t total_nnz);
sphint_status sphint_batch_run(const sphint_mesh_desc *meshes, int n_meshes, sphint_mode mode,
                               void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ candidate lists (CSR) */

/*
 * The step before the intersection path: each arc's candidate latitudes, as the CSR lists
 * sphint_arc_constlat takes.  lat_z (n_lat < 2^31 entries, device) must be ascending.  Arc
 * i's candidates are the latitudes in [lo_i - pad - 2^-46, hi_i + pad + 2^-46], where
 * [lo_i, hi_i] is the height range the minor arc covers (Sec. 2's containment rule read as a
 * range query: the heights of the normalised endpoints, extended to the top or bottom of the
 * great circle when the slope signs at the endpoints put it inside the arc, an uncertified
 * sign counting as both), computed in binary64; the 2^-46 covers the rounding of those
 * bounds, so every latitude the arc meets is a candidate.  Arcs with a non-finite
 * coordinate get none.  pad >= 0.
 *
 * Two calls, in order on one stream with one workspace of at least
 * sphint_candidates_workspace_size(n_arcs) bytes (256-byte aligned):
 *   sphint_candidates_count writes lat_offsets[0..n_arcs] (device int64; lat_offsets[0] = 0,
 *     lat_offsets[n_arcs] = nnz) and *out_nnz (device int64), and keeps each arc's first
 *     candidate and count in the workspace;
 *   sphint_candidates_fill then writes lat_idx[0..min(nnz, capacity)) (device int32): the
 *     candidates of arc i, ascending, at [lat_offsets[i], lat_offsets[i+1]).  A caller that
 *     does not know nnz reads *out_nnz after the first call (or passes an upper bound).
 * SPHINT_E_INVAL (no launch) for negative sizes, missing pointers, a short or misaligned
 * workspace or a negative pad; SPHINT_E_HIP if a launch fails.
 */
size_t sphint_candidates_workspace_size(int64_t n_arcs);
sphint_status sphint_candidates_count(int64_t n_arcs, sphint_pts_soa p1, sphint_pts_soa p2,
                                      const double *lat_z, int64_t n_lat, double pad,
                                      int64_t *lat_offsets, int64_t *out_nnz, void *workspace,
                                      size_t workspace_bytes, void *stream);
sphint_status sphint_candidates_fill(int64_t n_arcs, const int64_t *lat_offsets,
                                     int32_t *lat_idx, int64_t capacity, void *workspace,
                                     size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ adaptive evaluation */

/*
 * Filtered switching between the direct binary64 evaluation and the EFT evaluation, which
 * the paper names as future work (Sec. 9), for dense pairs (pair i = arc i with latitude
 * z0[i]).  Pass 1 evaluates Eq. 2.2 in binary64, operation for operation as
 * SPHINT_NAIVE_FP64 does, and bounds its own rounding error as it goes; a pair is accepted
 * when the bound certifies every decision (the slope signs, the sign of s^2 and the height
 * comparisons against the normalised endpoints: the exact decisions of SPHINT_EFT_FP64) and
 * each point lies within tol * 2^-53 (max-norm) of the exact intersection.  Every other pair
 * (tangencies among them) goes to a queue that pass 2 evaluates with SPHINT_EFT_FP64's
 * arithmetic; those pairs carry SPHINT_F_RECOMPUTED.  So counts, roots and flags equal the
 * EFT mode's exactly, and every point is within max(tol, 4) * 2^-53 of the exact one.
 * tol = 0 sends every pair with an intersection to pass 2.
 *
 * out         dense per-pair output (device): slots 2i and 2i+1 hold pair i's hits in
 *             along-arc order, unused slots hold 0; out.root and out.flags may be NULL.
 * out_recomputed  one int64 (device, may be NULL): the number of pairs pass 2 evaluated.
 * workspace   device memory of at least sphint_adaptive_workspace_size(n) bytes, 256-byte
 *             aligned, used only by this call while it runs.
 * n < 2^32.  SPHINT_E_INVAL (no launch) for a negative or too large n, tol < 0 or NaN,
 * missing pointers or a short or misaligned workspace; SPHINT_E_HIP if a launch fails.
 */
#define SPHINT_F_RECOMPUTED 128u /* adaptive: evaluated by the EFT pass */

typedef struct {
  double *x, *y;  /* [2 n] */
  uint8_t *root;  /* [2 n] SPHINT_ROOT_*, may be NULL */
  uint8_t *count; /* [n] 0..2 */
  uint8_t *flags; /* [n] SPHINT_F_*, may be NULL */
} sphint_dense_out;

size_t sphint_adaptive_workspace_size(int64_t n);
sphint_status sphint_arc_constlat_adaptive(int64_t n, sphint_pts_soa p1, sphint_pts_soa p2,
                                           const double *z0, double tol, sphint_dense_out out,
                                           int64_t *out_recomputed, void *workspace,
                                           size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ alternative point formulas */

/*
 * For accuracy comparisons (Sec. 7's comparison of formulas, Sec. S2 on Kahan's
 * determinant): both points where the great circle of x1 -> x2 meets the latitude circle
 * z = z0, by one formula in binary64, with no containment test.  Formulas:
 *   SPHINT_FORMULA_EQ22   Eq. (2.2) on n = x1 x x2, directly (the naive mode's arithmetic);
 *   SPHINT_FORMULA_EQ21   Eq. (2.1) on the unit normal n / |n|;
 *   SPHINT_FORMULA_EQ71   Eq. (7.1): Eq. (2.1) with the denominator 1 - n^z^2;
 *   SPHINT_FORMULA_KAHAN  Eq. (2.2) with n by Kahan's DiffOfProd (Alg. 3);
 *   SPHINT_FORMULA_ACCUX  AccuX (Alg. 8), the EFT mode's arithmetic.
 * out_x, out_y  [2 n] (device): slot 2i the upper-sign point (SPHINT_ROOT_PLUS), slot 2i+1
 *               the lower one; 0 where the formula gives none.
 * out_ok        [n] (device): 1 where the formula's s^2 is non-negative and its
 *               denominator positive, else 0.
 * Dense pairs (arc i with z0[i]), one launch.  SPHINT_E_INVAL (no launch) for n < 0, an
 * unknown formula or missing pointers; SPHINT_E_HIP if the launch fails.
 */
#define SPHINT_FORMULA_EQ22 0
#define SPHINT_FORMULA_EQ21 1
#define SPHINT_FORMULA_EQ71 2
#define SPHINT_FORMULA_KAHAN 3
#define SPHINT_FORMULA_ACCUX 4

sphint_status sphint_circle_points(int64_t n, sphint_pts_soa p1, sphint_pts_soa p2,
                                   const double *z0, int formula, double *out_x, double *out_y,
                                   uint8_t *out_ok, void *stream);

/* ------------------------------------------------------------ arc x arc intersections */

/*
 * Intersection of two minor great-circle arcs A = a1 -> a2 and B = b1 -> b2 (the further
 * application the paper names for its accurate cross product, Sec. 1 and Sec. 9).  Their
 * great circles meet at +-p, p = (a1 x a2) x (b1 x b2) / |(a1 x a2) x (b1 x b2)|; the
 * result is the one of the two that lies on both closed arcs, if any.  With n_A = a1 x a2
 * and n_B = b1 x b2, +p is on both arcs iff n_B.a1 >= 0 >= n_B.a2 and n_A.b2 >= 0 >= n_A.b1,
 * -p iff all four inequalities are reversed (Binet-Cauchy on the containment tests);
 * endpoints need not be unit length (the arcs are those of x/|x|).
 *
 * Modes:
 *   SPHINT_NAIVE_FP64  every cross product, the four orientation signs, the norm and the
 *                      divisions in plain binary64.
 *   SPHINT_EFT_FP64    n_A and n_B by AccuDOP (Alg. 4) as compensated pairs; the four
 *                      orientation signs exact (two filter stages, then exact expansion
 *                      arithmetic); each component of n_A x n_B by AccuDOP (Alg. 4) on
 *                      the leading parts of the two pairs plus the four first-order
 *                      products of their trailing parts (the trailing x trailing products
 *                      lie below u^2 of the result), |.|^2 by SumOfSquares (Alg. 5), one
 *                      square root, three divisions.  Counts and flags are exact; the point is within a few
 *                      units of 2^-53 of the exact one (the same input range as above).
 *
 * Pairs: pair k takes arc ia[k] of A (arc k when ia == NULL, then n_a must equal n_pairs)
 * and arc ib[k] of B (likewise).  An index outside [0, n_a) / [0, n_b) yields a NONFINITE
 * pair, never an access out of bounds.  a1, a2 have n_a entries per component, b1, b2 n_b
 * (device).
 * out         [n_pairs] per component (device): the point, (0, 0, 0) when there is none.
 * out_count   [n_pairs] 0 or 1 (device, required).
 * out_flags   [n_pairs] SPHINT_AA_* bits (device, may be NULL).
 * No workspace; one kernel launch on `stream`.  SPHINT_E_INVAL (no launch) for negative
 * sizes, missing pointers, a bad mode or a direct side whose size is not n_pairs;
 * SPHINT_E_HIP if the launch fails.
 */
#define SPHINT_AA_HIT 1u       /* the arcs meet in one point */
#define SPHINT_AA_DEGEN 4u     /* an arc has a zero normal (equal or antipodal endpoints) */
#define SPHINT_AA_COPLANAR 8u  /* both arcs lie on one great circle: no isolated point */
#define SPHINT_AA_NONFINITE 16u/* an input is inf or nan, or an index is out of range */
#define SPHINT_AA_EXACT 32u    /* diagnostic (EFT): an orientation needed exact arithmetic */
#define SPHINT_AA_INTERNAL 64u /* exact arithmetic exceeded its buffer (not for valid input) */

typedef struct {
  double *x, *y, *z;
} sphint_pts_out;

sphint_status sphint_arc_arc(int64_t n_pairs, sphint_pts_soa a1, sphint_pts_soa a2, int64_t n_a,
                             sphint_pts_soa b1, sphint_pts_soa b2, int64_t n_b,
                             const int32_t *ia, const int32_t *ib, sphint_pts_out out,
                             uint8_t *out_count, uint8_t *out_flags, int mode, void *stream);

const char *sphint_status_string(sphint_status s);
/* "sphint <version> gfx950" */
const char *sphint_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPHINT_H */
