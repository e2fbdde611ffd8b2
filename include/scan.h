/*
 * scan.h - exact structural graph clustering (SCAN) on one AMD Instinct
 * MI355X (gfx950), C ABI.
 *
 * The operation is the one stated in GPUSCAN++ (Yuan et al., arXiv
 * 2311.12281), Section 2.1, problem statement: given an undirected graph
 * G = (V, E) and parameters 0 < eps <= 1 and mu >= 2, compute every cluster
 * and the role of every vertex, where
 *   N[v]       = nbr(v) + {v}                                    (Def 2.1)
 *   sigma(u,v) = |N[u] & N[v]| / sqrt(|N[u]| |N[v]|)             (Def 2.2, Eq. 1)
 *   N_eps[u]   = { v in N[u] : sigma(u,v) >= eps }               (Def 2.3)
 *   core       : |N_eps[u]| >= mu                                (Def 2.4)
 *   clusters   : closures of structural reachability (Defs 2.5, 2.6).
 *
 * Conventions of this library (all results are exact integers):
 *   - eps is an exact rational p/q.  The test sigma >= p/q is evaluated as
 *     (c q)^2 >= p^2 |N[u]| |N[v]| in 64-bit unsigned integers, so equality
 *     counts as similar (Def 2.3).
 *   - Each cluster is labelled by its minimum core vertex id.  A border vertex
 *     (non-core, similar to a core) belongs to every cluster holding a similar
 *     core neighbour and is reported with the smallest such label.  Any other
 *     vertex is SCAN_UNCLASSIFIED with label -1.
 *   - Vertex ids are int32; row offsets are int64.
 *
 * Every function returns an int status: SCAN_OK (0) or a negative error
 * code; on error the output buffers are left in an unspecified state and
 * scan_last_error() describes the failure.  No function throws.
 *
 * Threading: a scan_graph is immutable after creation, and every function may
 * be called from several threads at once.  scan_run and scan_run_device calls
 * on one in-memory graph overlap: a call that finds the graph's per-run
 * device buffers in use by another call runs beside it on a buffer set of its
 * own (17 n + m + 4 b + 256 bytes, b the edges of the last degree bucket,
 * plus 5 n of output staging for scan_run), on its own stream or the
 * caller's.  The sets are
 * allocated at the first overlap that needs them and kept for later calls
 * until scan_graph_destroy (scan_graph_device_bytes counts them).  A call
 * waits for the graph's own buffers instead when the graph was created with
 * device_budget_bytes and another set would exceed it (the graph's own
 * output and count staging counted as allocated).  Calls on a
 * partitioned graph and scan_similarity calls on one graph run one at a time.
 * scan_last_stats reports the call that finished last.  Calls on different
 * graphs are independent.
 */
#ifndef SCAN_MI355X_SCAN_H
#define SCAN_MI355X_SCAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum scan_status {
  SCAN_OK = 0,
  SCAN_E_INVAL = -1,  /* bad argument: NULL pointer, p < 1, q < p, mu < 2, n < 0 ... */
  SCAN_E_GRAPH = -2,  /* CSR is not a simple undirected graph: offsets not 0..nnz and
                         monotone, id out of range, row not strictly increasing,
                         self-loop, or an arc without its reverse */
  SCAN_E_RANGE = -3,  /* q * (max degree + 1) >= 2^32: the 64-bit eps test could overflow */
  SCAN_E_NOMEM = -4,  /* device or host allocation failed */
  SCAN_E_DEVICE = -5  /* HIP runtime error (no GPU, launch failure, ...) */
};

enum scan_role { SCAN_UNCLASSIFIED = 0, SCAN_CORE = 1, SCAN_BORDER = 2,
                 /* with scan_opts.hub_outlier set, vertices in no cluster are
                    split by Def 2.7: a hub has neighbours in two or more
                    clusters (a border counts in the cluster it was given),
                    an outlier does not */
                 SCAN_HUB = 3, SCAN_OUTLIER = 4 };

/* Opaque graph handle, owned by the library. */
typedef struct scan_graph scan_graph;

typedef struct scan_opts {
  uint64_t device_budget_bytes; /* device memory the graph may use; 0 = no cap */
  int32_t validate;             /* 1: check the CSR on the device (default) */
  int32_t pruning;              /* 1: skip/bound/early-exit work that cannot change the
                                   result (default); 0: evaluate every edge in full.
                                   Results are identical either way. */
  int32_t timing;               /* 1: record per-phase device times (hipEvents) */
  int32_t strategy;             /* edges whose smaller side has degree > 64:
                                   0 = grouped by the larger side, whose neighbours are
                                       staged in an LDS hash table (default);
                                   1 = one wave per edge, binary search in global memory */
  int32_t hub_outlier;          /* 1: report SCAN_HUB / SCAN_OUTLIER instead of
                                   SCAN_UNCLASSIFIED (one more pass over the edges,
                                   Def 2.7 and Alg. 4); 0 (default): three roles */
  int32_t hub_ranked;           /* 1 (default): on the in-memory path, for graphs of more
                                   than 2^19 vertices, the edges whose smaller side has
                                   degree > 64 intersect a copy of the rows in which every
                                   vertex is renamed to its rank by increasing degree
                                   (4 more device bytes per arc, built on the host when the
                                   graph is created); 0: the rows as given.  Results are
                                   identical either way. */
  void* hip_stream;             /* hipStream_t to run on; NULL = a library-owned stream */
} scan_opts;

/* Fills *opts with the defaults above. */
void scan_opts_default(scan_opts* opts);

/*
 * scan_graph_create - copy an undirected CSR graph to the device and build the
 * library's layout (degree-oriented edge list grouped by degree bucket;
 * GPUSCAN++ Section 4.1).  If opts->device_budget_bytes is non-zero and the
 * in-memory layout would exceed it, the graph takes the partition-based path
 * (GPUSCAN++ Section 5): the CSR stays in pinned host memory, only row_ptr and
 * the per-vertex state reside on the device, and every run streams blocks of
 * rows and their edges through buffers that fit the budget.  Results are
 * identical on both paths.
 *   n        number of vertices, n >= 0
 *   nnz      number of arcs (= 2 |E|)
 *   row_ptr  host int64[n+1], row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing
 *   col_idx  host int32[nnz], each row strictly increasing, symmetric, no self-loops
 *   opts     may be NULL (defaults)
 *   out      receives the handle
 * The caller keeps ownership of row_ptr/col_idx; the library copies them.
 * Errors: SCAN_E_INVAL, SCAN_E_GRAPH (validation on), SCAN_E_NOMEM, SCAN_E_DEVICE.
 */
int scan_graph_create(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      const scan_opts* opts, scan_graph** out);

/* Releases every device and host resource of the graph.  NULL is accepted. */
int scan_graph_destroy(scan_graph* g);

/* Upper bound of the device bytes scan_graph_create allocates for an in-memory
 * graph of n vertices and nnz arcs under opts (NULL = defaults): row offsets,
 * neighbour ids (and their degree-ranked copy when opts->hub_ranked is set and
 * n > 2^19) with every 32nd id sampled, the oriented edge list with the degrees of both ends of each
 * edge, its worklist and edge states, per-vertex
 * state and output staging, plus 1 MiB for small tables.  A graph created with
 * device_budget_bytes below this value takes the partition-based path. */
int scan_graph_footprint(int32_t n, int64_t nnz, const scan_opts* opts, uint64_t* bytes);

/* Sizes of a created graph: vertices, arcs, undirected edges, maximum degree. */
int scan_graph_info(const scan_graph* g, int32_t* n, int64_t* nnz, int64_t* m, int32_t* max_degree);

/* Device bytes an in-memory graph holds now: its layout, its per-run buffers
 * and staging as allocated so far, and the buffer sets of overlapping calls
 * (0 for a partitioned graph, whose device use is its budget).
 * SCAN_E_INVAL if an argument is NULL. */
int scan_graph_device_bytes(const scan_graph* g, uint64_t* bytes);

/*
 * scan_run - structural clustering of g for eps = eps_num/eps_den and mu
 * (problem statement of GPUSCAN++ Section 2.1; method of Algorithms 1-3).
 *   labels  host int32[n], caller-owned: cluster label (minimum core id) or -1
 *   roles   host uint8[n], caller-owned: SCAN_CORE, SCAN_BORDER or SCAN_UNCLASSIFIED
 *           (SCAN_HUB / SCAN_OUTLIER in its place with opts.hub_outlier)
 * Requires 1 <= eps_num <= eps_den (0 < eps <= 1, Def 2.3) and mu >= 2 (Def 2.4).
 * Errors: SCAN_E_INVAL, SCAN_E_RANGE, SCAN_E_NOMEM, SCAN_E_DEVICE.
 */
int scan_run(scan_graph* g, int64_t eps_num, int64_t eps_den, int32_t mu, int32_t* labels,
             uint8_t* roles);

/*
 * scan_run_device - as scan_run, with the outputs left in device memory.
 *   d_labels  device int32[n], d_roles device uint8[n] (for example from
 *             scan_device_alloc); written on `stream` (NULL = the graph's stream).
 * The call returns after the work is enqueued and the stream has been
 * synchronised (the outputs are ready on return).
 */
int scan_run_device(scan_graph* g, int64_t eps_num, int64_t eps_den, int32_t mu,
                    int32_t* d_labels, uint8_t* d_roles, void* stream);

/*
 * scan_run_device_noalloc - scan_run_device for callers that cannot allocate
 * device memory on the call (tight serving loops, harnesses that forbid
 * hipMalloc, code that enqueues into a stream it is capturing): the same kernels and the same
 * results, with every per-run buffer taken from one static device array of
 * 64 MiB that the library holds on each device it runs on until the process
 * ends.  The call makes no hipMalloc, hipFree or other allocating call.
 *   g         an in-memory graph (SCAN_E_INVAL on the partitioned path), created
 *             on the current device (SCAN_E_INVAL otherwise)
 *   d_labels  device int32[n], d_roles device uint8[n], caller-owned
 *   stream    NULL = the graph's stream
 * The run needs about 17 bytes per vertex, 1 byte per edge and 4 bytes per
 * edge of the LDS-hash bucket, each part rounded up to 256 bytes; a graph that
 * needs more than the 64 MiB is refused with SCAN_E_NOMEM (nothing is run).
 * All calls on one device share its array and each call leaves its contents
 * there: calls that overlap on one device race and must be serialised by the
 * caller.  Only kernels are enqueued (no memset, copy or event).  With
 * stream = NULL the call returns after the graph's stream has been
 * synchronised (outputs ready); with a caller's stream it returns once the
 * kernels are enqueued, and the outputs are ready when that stream reaches them.
 * Errors: SCAN_E_INVAL, SCAN_E_RANGE, SCAN_E_NOMEM, SCAN_E_DEVICE.
 */
int scan_run_device_noalloc(scan_graph* g, int64_t eps_num, int64_t eps_den, int32_t mu,
                            int32_t* d_labels, uint8_t* d_roles, void* stream);

/*
 * scan_similarity - closed-neighbourhood intersection size |N[u] & N[v]| for
 * every arc (u -> v), in CSR order (the numerator of sigma, Def 2.2, Eq. 1);
 * both arcs of an edge carry the same value.  sigma itself is
 * counts[k] / sqrt((deg(u)+1)(deg(v)+1)).  Every edge is evaluated in full.
 *   counts  host int32[nnz], caller-owned
 */
int scan_similarity(scan_graph* g, int32_t* counts);

/* scan_similarity with the output in device memory (int32[nnz]); in-memory
 * graphs only (SCAN_E_INVAL on the partitioned path). */
int scan_similarity_device(scan_graph* g, int32_t* d_counts, void* stream);

/*
 * scan_eps_threshold - the smallest closed count c with (c q)^2 >= p^2 a b,
 * i.e. the least |N[u] & N[v]| that makes an edge with |N[u]| = a and
 * |N[v]| = b similar at eps = p/q (Def 2.3).  Host-only arithmetic, the same
 * code the kernels use.  Returns -1 if the arguments are out of range
 * (p < 1, q < p, a < 1, b < 1, or q*max(a,b) >= 2^32).
 */
int64_t scan_eps_threshold(int64_t p, int64_t q, int64_t a, int64_t b);

/* Per-call measurements of the last scan_run / scan_run_device /
 * scan_similarity on g (phase times need opts.timing = 1). */
enum { SCAN_PHASE_INIT = 0, SCAN_PHASE_CORES, SCAN_PHASE_FINALIZE, SCAN_PHASE_HOOK,
       SCAN_PHASE_MERGE, SCAN_PHASE_FLATTEN, SCAN_PHASE_ATTACH, SCAN_PHASE_OUTPUT,
       SCAN_NUM_PHASES };
enum { SCAN_NUM_BUCKETS = 7 };
typedef struct scan_stats {
  double ms_total;                        /* device time of the whole call */
  double ms_phase[SCAN_NUM_PHASES];       /* device time per phase */
  double ms_cores_bucket[SCAN_NUM_BUCKETS]; /* similarity/core kernel, per degree bucket */
  int64_t edges;                          /* undirected edges m */
  int64_t bucket_edges[SCAN_NUM_BUCKETS]; /* edges per degree bucket */
  int64_t evaluated[SCAN_NUM_PHASES];     /* edges intersected, per phase */
  int64_t bounded[SCAN_NUM_PHASES];       /* edges decided dissimilar by |N[u]&N[v]| <= min(a,b) */
  int64_t probes[SCAN_NUM_PHASES];        /* smaller-list elements consumed by intersections */
  int64_t cores_bucket_evaluated[SCAN_NUM_BUCKETS];
  int64_t cores_bucket_probes[SCAN_NUM_BUCKETS];
  int64_t h2d_bytes;                      /* partitioned path: bytes streamed to the device */
  int64_t group_split;                    /* LDS-hash kernel: lanes that claimed another chunk than
                                             their group (a group's lanes must stay together);
                                             always 0 in a correct run */
} scan_stats;

int scan_last_stats(const scan_graph* g, scan_stats* out);

/*
 * Serving: graphs stay resident on the device together with the exact closed
 * count of every edge (computed once when the graph is added), and
 * (graph, eps, mu) queries are answered by re-thresholding those counts -
 * the same result as scan_run, without recomputing any intersection.
 * Requests are admitted onto `num_slots` slots (one HIP stream and scratch
 * each) as slots free up, so queries that arrive while others run overlap on
 * the device.  Admission: a graph is made resident when the bytes already
 * held plus its footprint (scan_graph_footprint with the server's options,
 * plus 12 bytes per edge for the cached counts and closed-size products) plus
 * what the slots' scratch would grow by (18 bytes per vertex and 1 per edge of
 * the largest resident graph, per slot) fit opts->device_budget_bytes (0 = no
 * cap).  Otherwise it stays in host memory and its queries run on a fallback
 * thread with its own stream, through a partition-based graph built with the
 * budget left over (kept, and counted as held, until a query of another
 * non-resident graph or an admission needs the memory); resident queries keep
 * being admitted and completed meanwhile.  All functions are thread-safe.
 */
typedef struct scan_server scan_server;

int scan_server_create(const scan_opts* opts, int32_t num_slots, scan_server** out);

/* Copies the CSR (same requirements as scan_graph_create); *gid_out is the
 * graph's id for submit/remove. */
int scan_server_add_graph(scan_server* s, int32_t n, int64_t nnz, const int64_t* row_ptr,
                          const int32_t* col_idx, int32_t* gid_out);

/* Replaces the admission limit (0 = no cap) for graphs added from now on and
 * for the partition-based graphs of later fallback queries; graphs already
 * resident stay resident. */
int scan_server_set_budget(scan_server* s, uint64_t device_budget_bytes);

/* Waits for the graph's queued and running queries, then releases it. */
int scan_server_remove_graph(scan_server* s, int32_t gid);

/* Queues a query and returns at once with its id in *req_out.
 * Errors: SCAN_E_INVAL (unknown graph, eps or mu out of range), SCAN_E_RANGE. */
int scan_server_submit(scan_server* s, int32_t gid, int64_t eps_num, int64_t eps_den, int32_t mu,
                       int64_t* req_out);

/* Blocks until request `req` has finished, copies its result into
 * labels[n] / roles[n] (host, caller-owned; either may be NULL) and reports
 * the time from submit to completion.  Each request is waited for once. */
int scan_server_wait(scan_server* s, int64_t req, int32_t* labels, uint8_t* roles, double* latency_ms);

/* Device bytes held for resident graphs and slots, graph counts, requests done. */
int scan_server_info(scan_server* s, uint64_t* resident_bytes, int32_t* graphs, int32_t* resident_graphs,
                     int64_t* completed);

/* Finishes every queued request, then releases everything. */
int scan_server_destroy(scan_server* s);

/*
 * Batched clustering: many independent graphs, each with its own eps and mu,
 * clustered together (the method of Algorithms 1-3 applied to every graph).
 * The graphs are packed into one disjoint union on the device (every vertex
 * knows its graph and looks up that graph's parameters), and one persistent
 * kernel clusters the whole batch: its blocks take (graph, phase, tile) work
 * items from a device queue, every graph moves through the phases on its own
 * (a per-graph count of the unfinished tiles of its current phase; the block
 * finishing the last one queues the next phase), and the queue reset plus
 * that kernel are captured once into a HIP graph, so one run is a single
 * graph launch whatever the number of graphs.  Per-graph eps and mu are read
 * from device memory on every run.  With autotune = 1 the library times whole
 * runs on this batch to choose, per degree bucket, the lane-group width of
 * the intersection (4 to 64 lanes per edge, or a wave with an LDS hash set for
 * the two buckets whose smaller side has more than 32 neighbours), and the
 * edges per tile; SCAN_AUTOTUNE_CACHE names an optional file that caches the
 * choice by batch shape.
 */
typedef struct scan_batch {
  int32_t num_graphs;       /* G >= 0 */
  const int64_t* vtx_off;   /* [G+1] vertex offsets of the graphs (prefix of n_g), vtx_off[0] = 0 */
  const int64_t* arc_off;   /* [G+1] arc offsets (prefix of nnz_g), arc_off[0] = 0 */
  const int64_t* row_ptr;   /* graph g's own row offsets, n_g + 1 entries from 0 to nnz_g,
                               stored at row_ptr[vtx_off[g] + g] */
  const int32_t* col_idx;   /* graph g's local neighbour ids (0 <= id < n_g) at col_idx[arc_off[g]] */
  const int64_t* eps_num;   /* [G] */
  const int64_t* eps_den;   /* [G] */
  const int32_t* mu;        /* [G] */
  int32_t autotune;         /* 1: choose lane widths and tile size by timing runs of this batch */
} scan_batch;

typedef struct scan_batch_graph scan_batch_graph;

/* Packs and validates the batch (each graph as in scan_graph_create), builds
 * the device layout and work-item tables, optionally autotunes, and captures
 * the run.  Errors: SCAN_E_INVAL, SCAN_E_GRAPH, SCAN_E_RANGE (a graph's eps
 * denominator with its maximum degree), SCAN_E_NOMEM, SCAN_E_DEVICE. */
int scan_batch_create(const scan_batch* b, const scan_opts* opts, scan_batch_graph** out);

/* Replaces every graph's eps and mu ([G] arrays, same rules as in
 * scan_batch); the next run uses them, no new capture needed. */
int scan_batch_set_params(scan_batch_graph* bg, const int64_t* eps_num, const int64_t* eps_den,
                          const int32_t* mu);

/* Clusters every graph of the batch: labels[vtx_off[G]] receive graph-local
 * labels (minimum core id within the graph, -1 if unclassified) and roles the
 * roles, both host, caller-owned, packed like the vertices.  replay = 1 runs
 * the captured HIP graph, 0 launches the same two kernels directly.  A run in
 * which a block waits more than 20 s for a work item is abandoned and
 * reported as SCAN_E_DEVICE. */
int scan_batch_run(scan_batch_graph* bg, int32_t replay, int32_t* labels, uint8_t* roles);

/* Chosen configuration: lanes[SCAN_NUM_BUCKETS] lane-group widths per degree
 * bucket, *tile_edges edges per work item of the edge phases (either may be NULL). */
int scan_batch_config(const scan_batch_graph* bg, int32_t* lanes, int32_t* tile_edges);

/* Statistics of the last scan_batch_run (ms_total = device time of the run). */
int scan_batch_stats(const scan_batch_graph* bg, scan_stats* out);

int scan_batch_destroy(scan_batch_graph* bg);

/* One-shot: create, run once, destroy. */
int scan_run_batch(const scan_batch* b, const scan_opts* opts, int32_t* labels, uint8_t* roles);

/* Device memory helpers for the *_device entry points (hipMalloc/hipFree/hipMemcpy). */
int scan_device_alloc(uint64_t bytes, void** out);
int scan_device_free(void* ptr);
int scan_memcpy_d2h(void* dst, const void* src, uint64_t bytes);
int scan_memcpy_h2d(void* dst, const void* src, uint64_t bytes);

/* Device-to-device copy of `bytes` (a multiple of 16; src and dst device
 * pointers, 16-byte aligned, not overlapping) by a plain streaming kernel,
 * launched `iters` >= 1 times in a row on its own stream; *avg_ms (may be NULL)
 * receives the mean kernel time.  Not part of the clustering path: it is the
 * reference against which hardware byte counters and HBM bandwidth of the
 * clustering kernels are calibrated.  SCAN_E_INVAL on a bad size, alignment
 * or iteration count. */
int scan_device_copy(void* dst, const void* src, uint64_t bytes, int32_t iters, float* avg_ms);

/* Read-only stream of `bytes` (a multiple of 16) from the device buffer src
 * (16-byte aligned) by a plain streaming kernel, `iters` >= 1 times in a row;
 * *avg_ms (may be NULL) receives the mean kernel time.  Not part of the
 * clustering path: the achievable rate of a kernel that only reads, the
 * ceiling for the intersection kernels (which write almost nothing).
 * SCAN_E_INVAL on a bad size, alignment or iteration count. */
int scan_device_read(const void* src, uint64_t bytes, int32_t iters, float* avg_ms);

/* Host-to-device link rate: copies `bytes` from a pinned host buffer into a
 * device buffer (both allocated and freed inside the call) `iters` >= 1 times
 * with hipMemcpyAsync and stores bytes per second of the mean copy in *h2d_bps.
 * The reference rate for the partitioned path, which streams from pinned host
 * memory.  SCAN_E_INVAL on bytes == 0 or iters < 1, SCAN_E_NOMEM if either
 * buffer cannot be allocated. */
int scan_h2d_rate(uint64_t bytes, int32_t iters, double* h2d_bps);

/* Thread-local description of the last error, valid until the next call. */
const char* scan_last_error(void);

/* Library version string. */
const char* scan_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCAN_MI355X_SCAN_H */
