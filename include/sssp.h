/*
 * sssp.h -- C ABI of the MI355X (gfx950) delta-stepping single-source
 * shortest-path library.
 *
 * The method is the linear-algebra delta-stepping of Sridhar et al.,
 * "Delta-stepping SSSP: from Vertices and Edges to GraphBLAS Implementations"
 * (IPDPSW 2019): the adjacency matrix is split into light and heavy parts
 * (Sec. IV-A), buckets are selected by the mask i*delta <= t < (i+1)*delta
 * (Sec. IV-B), and each processing phase is a masked min-plus product
 * t_Req = A_L^T (t o t_Bi) or A_H^T (t o S) merged into t by an element-wise
 * min (Sec. IV-C, IV-D; Fig. 1 left).
 *
 * Conventions for every entry point
 *   - Return value: an sssp_status. Nothing throws across this boundary.
 *   - Pointers documented as "device" are HIP device pointers on the device
 *     that is current when sssp_create is called; "host" pointers are ordinary
 *     host memory. The caller owns every pointer it passes; the library never
 *     frees caller memory and keeps no caller pointer after a call returns,
 *     except the trace buffer that sssp_set_trace attaches (kept until
 *     detached or replaced).
 *   - stream: a hipStream_t passed as void* (NULL = the null stream). Work is
 *     enqueued on it; calls documented as synchronising wait for it.
 *   - On error, outputs are unspecified and a handle stays valid (except that
 *     sssp_create stores NULL into *out).
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef SSSP_MI355X_H
#define SSSP_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSSP_OK = 0,
  SSSP_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad sizes, malformed CSR, bad delta or source */
  SSSP_ERR_INVALID_WEIGHT = 2,   /* a weight that is zero, negative, NaN or infinite */
  SSSP_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed */
  SSSP_ERR_DEVICE = 4,           /* a HIP runtime error or an aborted device schedule (a barrier wait
                                    without progress past its limit, or an internal queue over capacity) */
  SSSP_ERR_OVERFLOW = 5,         /* a reachable vertex's distance is not representable */
  SSSP_ERR_NO_FORWARD = 6,       /* sssp_backward before any successful sssp_solve */
  SSSP_ERR_UNSUPPORTED = 7,      /* a size or type outside what the library handles */
} sssp_status;

typedef enum {
  SSSP_WEIGHT_U32 = 0, /* uint32 weights >= 1; distances uint32, UINT32_MAX = unreachable */
  SSSP_WEIGHT_F32 = 1, /* float weights, finite and > 0; distances float, +inf = unreachable */
  SSSP_WEIGHT_F64 = 2, /* double weights, finite and > 0; distances double, +inf = unreachable
                          (the paper's own precision, GrB_FP64 in Fig. 4) */
} sssp_weight_type;

/*
 * Directed weighted graph as the CSR of its adjacency matrix A: row u holds the
 * out-edges of vertex u, A(u, v) = weight of u -> v (Sec. II, graph as a matrix).
 * All arrays are DEVICE memory, caller-owned, read only, and only borrowed for
 * the duration of sssp_create (the handle keeps its own copy).
 *   n        number of vertices, 1 <= n < 2^31
 *   m        number of edges, 0 <= m < 2^32
 *   row_ptr  int64 [n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = m
 *   col_idx  int32 [m], 0 <= col_idx[e] < n; parallel edges and self-loops are
 *            accepted (parallel edges act as their minimum, self-loops never
 *            improve a distance because weights are positive)
 *   weights  [m] of wtype
 */
typedef struct {
  int64_t n;
  int64_t m;
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const void *weights;
  int32_t wtype; /* sssp_weight_type */
} sssp_graph;

/* Counters of the last sssp_solve, summed over its sources. */
typedef struct {
  uint64_t sources;      /* solves performed */
  uint64_t buckets;      /* bucket rounds (non-empty buckets processed) */
  uint64_t light_phases; /* light relaxation phases (inner-loop iterations) */
  uint64_t heavy_phases; /* heavy relaxation phases */
  uint64_t far_phases;   /* redistributions of far-future buckets */
  uint64_t light_edges;  /* light edges scanned */
  uint64_t heavy_edges;  /* heavy edges scanned */
  uint64_t improvements; /* relaxations that lowered a tentative distance */
  uint64_t attempts;     /* atomic min operations on tentative distances (requests that passed the
                            cached comparison; attempts - improvements lost to a lower value) */
  uint64_t barriers;     /* device-wide synchronisations */
  uint64_t trace_records; /* step records produced (see sssp_set_trace) */
} sssp_stats;

/* Schedule parameters (every field 0 = library default). */
typedef struct {
  int32_t workgroups_per_cu; /* workgroups per compute unit of a launch with one source (or one
                                multi-source row): 1 = one of 1024 threads; 0 (default) or 2 and
                                more = two of 512 threads. Concurrent sources always run two
                                512-thread workgroups per compute unit */
  int32_t ring_buckets;      /* buckets held in the near ring, power of two in [2, 64] (default: fit max weight) */
  int32_t inline_edges;      /* phases scanning at most this many edges (and at most inline_entries list
                                entries) run on one workgroup without a device-wide barrier (default 4096) */
  int32_t concurrent_sources; /* sources solved at the same time, each by its own group of workgroups
                                 (a power of two dividing the launch's workgroup counts, at most 256; default 1).
                                 Each extra group holds its own working set, about (14 + ring) * 4 * n bytes
                                 (fp64: 2 more) plus m / 13 bytes of hub queues */
  int32_t wait_limit_ms;     /* a device-wide barrier wait that sees neither the release nor progress of the
                                workgroup running steps alone inside the barrier for this long aborts the
                                solve with SSSP_ERR_DEVICE instead of hanging (default 30000) */
  int32_t hub_edges;         /* tile schedule: a vertex with at least this many edges in a phase is cut into
                                pieces that the whole group relaxes (a hub step); power of two in
                                [256, 65536] (default 1024) */
  int32_t chunk_entries;     /* tile schedule: most list entries a workgroup claims and expands at a time;
                                power of two in [32, 512] (default 512, 256 in groups of 128 or more
                                workgroups) */
  int32_t inline_entries;    /* tile schedule: most list entries of a phase that one workgroup runs alone
                                inside the barrier, in [1, 512] (default: the chunk size; 512 with
                                leader_chain 1) */
  int32_t leader_chain;      /* 1: the workgroup running a light phase alone keeps the vertices it
                                re-inserts in LDS and runs the bucket's next light phase from them at
                                once while it stays within the two limits above (no list round trip
                                and no barrier in between); 2: one phase at a time; 0 (default): 1 on
                                graphs with at most 6 edges per vertex on average, else 2 */
} sssp_tuning;

typedef struct sssp_handle sssp_handle;

/*
 * sssp_create -- prepare a graph and delta for repeated solves.
 *   Validates the CSR and the weights, then splits A into its light and heavy
 *   parts, A_L = A o (0 < A <= delta) and A_H = A o (A > delta) (Sec. IV-A;
 *   Fig. 1 left, first two lines; light(v) and heavy(v) of Sec. III-A), stored as
 *   one row-partitioned copy: each row holds its light edges, then its heavy ones.
 *   delta: for SSSP_WEIGHT_U32 an integer in [1, 2^32-1]; for SSSP_WEIGHT_F32 the
 *   threshold is (float)delta, which must be finite and > 0, and the total weight
 *   times exp((n-1) * 2^-24) (a bound on any rounded path sum) divided by delta
 *   must stay below 2^32 - 256 (bucket indices fit 32 bits); for SSSP_WEIGHT_F64
 *   delta itself, finite and > 0, with the same bound using 2^-53.
 *   stream: enqueue work here; the call synchronises it before returning.
 *   out: host pointer receiving the new handle (library-owned; free with
 *   sssp_destroy), NULL on error.
 *   Errors: INVALID_ARGUMENT (null pointers, n/m/CSR, delta), INVALID_WEIGHT,
 *   UNSUPPORTED (sizes), OUT_OF_MEMORY, DEVICE.
 */
sssp_status sssp_create(const sssp_graph *g, double delta, void *stream, sssp_handle **out);

/*
 * sssp_solve -- shortest-path distances from k sources, one after another.
 *   For source s = sources[r], row r of dist receives d_s(v) = the minimum over
 *   directed paths from s to v of the path weight (Sec. III, problem statement),
 *   computed by delta-stepping (Fig. 1): buckets B_i selected by
 *   i*delta <= t < (i+1)*delta, light phases t_Req = A_L^T (t o t_Bi) repeated
 *   while vertices re-enter B_i, then one heavy phase t_Req = A_H^T (t o S).
 *   Path weights add left to right in the weight type: exact integers for u32
 *   (a distance above 2^32-2 is SSSP_ERR_OVERFLOW), binary32 (binary64)
 *   round-to-nearest-even for f32 (f64) (a sum that rounds to +inf is
 *   SSSP_ERR_OVERFLOW). The result does not depend on the order of relaxations.
 *   sources: HOST int32 [k], each in [0, n).  k >= 1.
 *   dist: DEVICE, caller-owned, [k][n] of the weight type (uint32, float or
 *   double), row-major; fully overwritten. d(s) = 0; unreachable = UINT32_MAX / +inf.
 *   stream: the call synchronises it before returning (to report overflow).
 *   Errors: INVALID_ARGUMENT, OVERFLOW, DEVICE.
 */
sssp_status sssp_solve(sssp_handle *h, const int32_t *sources, int32_t k, void *dist, void *stream);

/*
 * sssp_solve_async -- the same solves as sssp_solve, enqueued only.
 *   The k independent single-source problems of one call are the columns of a
 *   distance matrix T (n x k); each step of Fig. 1 then applies to every column
 *   with its own bucket index, i.e. T_Req = A_L^T (T o T_B) column by column
 *   (Sec. IV-C with the vector t generalised to a matrix). With
 *   concurrent_sources = G, G columns are advanced at the same time.
 *   sources: DEVICE int32 [k], read when the work runs; an entry outside [0, n)
 *   leaves its row all-unreachable and is reported by sssp_solve_status.
 *   dist: DEVICE [k][n] as for sssp_solve. k >= 1.
 *   Nothing is synchronised and no memory is allocated or set by copy/memset
 *   calls, so the call may be recorded into a HIP graph by stream capture (its
 *   kernels: a control-block reset and one cooperative launch) and replayed;
 *   every replay recomputes dist from the sources it finds in memory.
 *   Errors (before anything is enqueued): INVALID_ARGUMENT, DEVICE.
 */
sssp_status sssp_solve_async(sssp_handle *h, const int32_t *sources, int32_t k, void *dist, void *stream);

/*
 * sssp_solve_multi -- distances from the nearest of k sources, in one solve.
 *   dist receives d(v) = min over r of d_{sources[r]}(v): delta-stepping with
 *   every source at distance 0 in the first bucket (Fig. 1 left, initialisation
 *   t(s) = 0 applied to each source). For a graph that is the disjoint union of
 *   several graphs (a block-diagonal adjacency matrix) with one source in each,
 *   this solves every graph of the batch at once: each block's rows of dist are
 *   its own single-source distances.
 *   sources: HOST int32 [k], each in [0, n), repeats allowed.  dist: DEVICE [n]
 *   of the weight type, overwritten.  Synchronises the stream.
 *   Errors: INVALID_ARGUMENT, OVERFLOW, DEVICE.
 */
sssp_status sssp_solve_multi(sssp_handle *h, const int32_t *sources, int32_t k, void *dist, void *stream);

/*
 * sssp_solve_multi_async -- sssp_solve_multi, enqueued only (sources in DEVICE
 *   memory, read when the work runs; capturable like sssp_solve_async; outcome
 *   from sssp_solve_status). Errors before enqueueing: INVALID_ARGUMENT, DEVICE.
 */
sssp_status sssp_solve_multi_async(sssp_handle *h, const int32_t *sources, int32_t k, void *dist, void *stream);

/*
 * sssp_solve_status -- wait for the last enqueued solve (sssp_solve_async, or
 *   the last replay of a graph that recorded it) on `stream` and report its
 *   outcome; on success its counters become those of sssp_last_stats and
 *   sssp_backward may use its distances. Synchronises the stream.
 *   Errors: NO_FORWARD (nothing enqueued on this handle), INVALID_ARGUMENT (a
 *   source outside [0, n)), OVERFLOW, DEVICE.
 */
sssp_status sssp_solve_status(sssp_handle *h, void *stream);

/*
 * sssp_backward -- gradient of a loss of the distances with respect to the
 *   edge weights (fp32 handles). For each source s = sources[r] with distances
 *   dist[r] (as returned by sssp_solve on this handle with its current weights)
 *   and dL/dd = grad_dist[r], d_s(v) is the sum of the weights along v's path in
 *   the shortest-path tree (Sec. III: the minimum-weight path; the relaxations
 *   of Sec. III-C define which in-edge is tight), so
 *     dL/dw_e = sum over sources of the sum of grad_dist over the tree's
 *               subtree below e        (0 for edges in no tree).
 *   The tree is recomputed from dist: the parent of v is its tight in-edge
 *   (dist(u) (+) w == dist(v)) from a strictly closer vertex (dist(u) <
 *   dist(v)) with the smallest caller edge index, which makes the result well
 *   defined under ties. Under fp32 rounding a weight can be absorbed (d (+) w
 *   == d), so a vertex may be tight only through in-edges from vertices at its
 *   own distance; such vertices are resolved in rounds, each taking the
 *   smallest-index tight in-edge from a vertex resolved in the round before
 *   (round 0: the source and the vertices with a strictly closer parent).
 *   dist is checked on the device to be the shortest-path vector: dist(s) =
 *   +0, no edge out of a reached vertex can lower its target (dist(v) <=
 *   dist(u) (+) w), and every reached vertex hangs below s in the tree.
 *   grad_dist at unreachable vertices and at the source is ignored. Sums run
 *   in fp64; grad_w is written in fp32.
 *   sources: HOST int32 [k].  dist: DEVICE [k][n] float.  grad_dist: DEVICE
 *   [k][n] float.  grad_w: DEVICE [m] float, caller edge order, overwritten.
 *   With concurrent_sources = G (sssp_set_tuning), G sources are processed at
 *   the same time, as in the forward solve. The call synchronises the stream.
 *   Errors: INVALID_ARGUMENT (pointers, sources, or dist not a shortest-path
 *   vector of this graph), UNSUPPORTED (uint32 and double handles), NO_FORWARD (no
 *   successful sssp_solve since the handle's weights were set), DEVICE.
 */
sssp_status sssp_backward(sssp_handle *h, const int32_t *sources, int32_t k, const void *dist,
                          const float *grad_dist, float *grad_w, void *stream);

/*
 * sssp_backward_noalloc -- sssp_backward for callers that cannot allocate device
 *   memory during the call (tight serving or training loops, harnesses that
 *   forbid hipMalloc): the adjoint's working set (distances and parents in
 *   solver order, child counts, levels, fp64 accumulators of grad_dist and of
 *   dL/dw) lives in a static device array of the library, 64 MiB per GPU, held
 *   by every GPU the library runs on until the process ends; nothing is
 *   allocated, freed or staged through host buffers by the call.
 *   The result is that of sssp_backward (same kernels and tie rule), with
 *   these differences:
 *     sources: DEVICE int32 [k] (read when the work runs; an entry outside
 *       [0, n) leaves its row out and returns INVALID_ARGUMENT);
 *     the working set takes 8 m bytes plus 28 n bytes per concurrent group
 *       (each part rounded up to 256 bytes) and 34 KiB of launch parameters; the call
 *       runs as many of the handle's concurrent groups as fit (at least one);
 *       a graph for which one group does not fit returns UNSUPPORTED (about
 *       n = 2^18 with m = 2^22, or m up to about 8.3 million edges with few
 *       vertices).
 *   Every call on one GPU (any handle, any stream) uses the same array and
 *   leaves its contents behind; the call clears what must start at zero.
 *   Calls that overlap in time on one GPU race and must be serialised by the
 *   caller. Synchronises the stream.
 *   Errors: INVALID_ARGUMENT, UNSUPPORTED (weight type, or the graph does not
 *   fit the array), NO_FORWARD, DEVICE.
 */
sssp_status sssp_backward_noalloc(sssp_handle *h, const int32_t *sources, int32_t k, const void *dist,
                                  const float *grad_dist, float *grad_w, void *stream);

/*
 * sssp_set_weights -- replace the weights of the handle's graph (same CSR
 *   structure, caller edge order) and redo the light/heavy split for the
 *   handle's delta (Sec. IV-A). weights: DEVICE [m] of the handle's weight
 *   type, validated as in sssp_create. Synchronises the stream.
 *   Errors: INVALID_WEIGHT, UNSUPPORTED (fp32 bucket range as for sssp_create),
 *   OUT_OF_MEMORY, DEVICE, INVALID_ARGUMENT.
 */
sssp_status sssp_set_weights(sssp_handle *h, const void *weights, void *stream);

/* Counters of the last successful sssp_solve (host struct, caller-owned). */
sssp_status sssp_last_stats(const sssp_handle *h, sssp_stats *out);

/*
 * Replace the schedule parameters of a handle (host struct; copied). Allocates
 * the working sets of new concurrent groups (and synchronises the device).
 * Errors: INVALID_ARGUMENT (negative fields, a ring size other than the
 * handle's), UNSUPPORTED (concurrent_sources above 256 or not dividing the
 * workgroup counts), OUT_OF_MEMORY.
 */
sssp_status sssp_set_tuning(sssp_handle *h, const sssp_tuning *t);

/*
 * sssp_get_tuning -- the handle's schedule parameters with every default
 *   resolved for a launch of its current concurrent-source count (out: HOST
 *   struct, caller-owned). Errors: INVALID_ARGUMENT.
 */
sssp_status sssp_get_tuning(const sssp_handle *h, sssp_tuning *out);

/*
 * sssp_set_trace -- attach a step trace (profiling aid; NULL/0 detaches).
 *   device_buffer: DEVICE uint64 [4 * capacity], caller-owned, must stay valid
 *   while attached. Every later sssp_solve writes one record per step when the
 *   step begins: word 0 = device wall clock (hipDeviceAttributeWallClockRate
 *   ticks); word 1 = (input entries << 32) | (bucket & 0xFFFFFF) << 8 | action
 *   (1 light phase, 2 heavy phase, 3 far redistribution, 4 done, 5 overflow
 *   check, 6 high-degree pieces of the previous phase; bit 0x80 set when one
 *   workgroup ran the phase alone); words 2 and 3 = edges scanned and distances
 *   lowered by the previous step. Records past capacity are counted in
 *   trace_records but not written. Tracing adds one atomic per workgroup per step.
 */
sssp_status sssp_set_trace(sssp_handle *h, uint64_t *device_buffer, int64_t capacity);

/* Outcome of sssp_autotune. */
typedef struct {
  double delta;               /* the chosen delta */
  int32_t concurrent_sources; /* the chosen number of concurrent groups */
  int32_t trials;             /* configurations timed */
  float ms;                   /* device time of one solve of the sample with the chosen configuration */
  sssp_tuning tuning;         /* the chosen schedule, every field resolved (as sssp_get_tuning) */
} sssp_autotune_result;

/*
 * sssp_autotune -- create a handle whose delta, concurrent-source count and
 *   tile schedule are the fastest found for a sample of sources. delta is the
 *   method's only parameter (bucket width and light/heavy threshold, Sec. III-A
 *   and IV-A): a small delta means many buckets with small phases, a large one
 *   means light edges relaxed more than once. For each candidate delta the
 *   graph is split (as sssp_create) and the sample solved with 1, 8, 16, ...
 *   concurrent groups (up to k; the search over group counts stops when the
 *   time rises), one warm-up and one timed solve per pair. Then, on the fastest
 *   pair, the tile schedule is searched one field at a time (workgroups_per_cu
 *   for one group, hub_edges, chunk_entries, inline_edges, inline_entries; a
 *   value is kept when the faster of two timed solves beats the current choice
 *   by 2 %).
 *   g: as for sssp_create.  sources: HOST int32 [k], each in [0, n).
 *   mode: 0 = one row per source (sssp_solve), 1 = nearest-source distances
 *   (sssp_solve_multi; one group).  deltas: HOST [n_deltas] candidates, or NULL
 *   and 0 for powers of two around the mean weight (integers >= 1 for uint32
 *   weights).  dist: DEVICE scratch of the solves ([k][n] for mode 0, [n] for
 *   mode 1), overwritten.  out: receives the handle (tuned; free with
 *   sssp_destroy).  result: HOST, may be NULL.  Synchronises the stream.
 *   Errors: INVALID_ARGUMENT, INVALID_WEIGHT, OUT_OF_MEMORY, DEVICE, and the
 *   last error of a candidate when no candidate could be timed.
 */
sssp_status sssp_autotune(const sssp_graph *g, const int32_t *sources, int32_t k, int32_t mode,
                          const double *deltas, int32_t n_deltas, void *dist, void *stream, sssp_handle **out,
                          sssp_autotune_result *result);

/* Vertex and edge counts and the weight type of a handle (host out-pointers, any may be NULL). */
sssp_status sssp_graph_info(const sssp_handle *h, int64_t *n, int64_t *m, int32_t *wtype);

/* Release a handle and all device memory it owns. NULL is a no-op. */
void sssp_destroy(sssp_handle *h);

/* Static, human-readable name of a status. */
const char *sssp_status_string(sssp_status s);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_MI355X_H */
