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
 * Threading: a scan_graph is immutable after creation.  Calls on one graph
 * are serialised internally (they share the graph's per-run device buffers);
 * calls on different graphs may run concurrently.
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

enum scan_role { SCAN_UNCLASSIFIED = 0, SCAN_CORE = 1, SCAN_BORDER = 2 };

/* Opaque graph handle, owned by the library. */
typedef struct scan_graph scan_graph;

typedef struct scan_opts {
  uint64_t device_budget_bytes; /* device memory the graph may use; 0 = no cap */
  int32_t validate;             /* 1: check the CSR on the device (default) */
  int32_t pruning;              /* 1: skip/bound/early-exit work that cannot change the
                                   result (default); 0: evaluate every edge in full.
                                   Results are identical either way. */
  int32_t timing;               /* 1: record per-phase device times (hipEvents) */
  int32_t reserved;
  void* hip_stream;             /* hipStream_t to run on; NULL = a library-owned stream */
} scan_opts;

/* Fills *opts with the defaults above. */
void scan_opts_default(scan_opts* opts);

/*
 * scan_graph_create - copy an undirected CSR graph to the device and build the
 * library's layout (degree-oriented edge list grouped by degree bucket;
 * GPUSCAN++ Section 4.1).
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

/* Sizes of a created graph: vertices, arcs, undirected edges, maximum degree. */
int scan_graph_info(const scan_graph* g, int32_t* n, int64_t* nnz, int64_t* m, int32_t* max_degree);

/*
 * scan_run - structural clustering of g for eps = eps_num/eps_den and mu
 * (problem statement of GPUSCAN++ Section 2.1; method of Algorithms 1-3).
 *   labels  host int32[n], caller-owned: cluster label (minimum core id) or -1
 *   roles   host uint8[n], caller-owned: SCAN_CORE, SCAN_BORDER or SCAN_UNCLASSIFIED
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
 * scan_similarity - closed-neighbourhood intersection size |N[u] & N[v]| for
 * every arc (u -> v), in CSR order (the numerator of sigma, Def 2.2, Eq. 1);
 * both arcs of an edge carry the same value.  sigma itself is
 * counts[k] / sqrt((deg(u)+1)(deg(v)+1)).  Every edge is evaluated in full.
 *   counts  host int32[nnz], caller-owned
 */
int scan_similarity(scan_graph* g, int32_t* counts);

/* scan_similarity with the output in device memory (int32[nnz]). */
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
enum { SCAN_NUM_BUCKETS = 6 };
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
} scan_stats;

int scan_last_stats(const scan_graph* g, scan_stats* out);

/* Device memory helpers for the *_device entry points (hipMalloc/hipFree/hipMemcpy). */
int scan_device_alloc(uint64_t bytes, void** out);
int scan_device_free(void* ptr);
int scan_memcpy_d2h(void* dst, const void* src, uint64_t bytes);
int scan_memcpy_h2d(void* dst, const void* src, uint64_t bytes);

/* Thread-local description of the last error, valid until the next call. */
const char* scan_last_error(void);

/* Library version string. */
const char* scan_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCAN_MI355X_SCAN_H */
