// C-ABI of the library (declared in include/scan.h): graph creation, the
// in-memory clustering run (GPUSCAN++ Algorithm 1 with Algorithms 2-3), the
// exact per-arc closed counts, statistics and small device-memory helpers.
#include "graph.h"

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>

namespace {
thread_local std::string g_error;

int64_t gcd64(int64_t a, int64_t b) {
  while (b) { int64_t t = a % b; a = b; b = t; }
  return a;
}
}  // namespace

namespace scan {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(SCAN_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(SCAN_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace scan



namespace {

void release_extra(ExtraRun& x) {
  void* ptrs[] = {x.R.lower, x.R.upper, x.R.role, x.R.parent, x.R.label, x.R.state, x.R.stats,
                  x.R.counters, x.R.worklist, x.d_out_labels, x.d_out_roles};
  for (void* p : ptrs)
    if (p) hipFree(p);
  for (auto& e : x.ev)
    if (e) hipEventDestroy(e);
  if (x.stream) hipStreamDestroy(x.stream);
  x = ExtraRun();
}

void release(scan_graph* g) {
  part_release(g);
  for (auto& x : g->extra) {
    if (x->stream) hipStreamSynchronize(x->stream);
    release_extra(*x);
  }
  g->extra.clear();
  g->extra_bytes = 0;
  void* ptrs[] = {g->d_rp, g->d_ci, g->d_hci, g->d_hsamp, g->d_edges, g->d_edeg, g->d_jobs, g->d_wtab, g->d_worklist, g->d_counters, g->d_lower, g->d_upper, g->d_role, g->d_parent,
                  g->d_label, g->d_state, g->d_stats, g->d_out_labels, g->d_out_roles, g->d_counts};
  for (void* p : ptrs)
    if (p) hipFree(p);
  for (auto& e : g->ev)
    if (e) hipEventDestroy(e);
  if (g->own_stream && g->stream) hipStreamDestroy(g->stream);
}

template <typename T>
hipError_t dalloc(T** p, int64_t count) {
  return hipMalloc((void**)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

}  // namespace

RunState scan::graph_state(scan_graph* g) {
  return RunState{g->d_lower, g->d_upper, g->d_role, g->d_parent, g->d_label,
                  g->d_state, g->d_stats, g->d_counters, g->d_worklist};
}

// One pass of `mode` over bucket k of the oriented edges.
void scan::launch_bucket(scan_graph* g, hipStream_t s, int mode, int k, EdgeArgs& A, const RunState& R,
                         const RunConfig* cfg) {
  A.e_begin = g->bucket_off[k];
  A.e_end = g->bucket_off[k + 1];
  A.bucket = k;
  const bool hub = cfg ? cfg->hub : g->opts.strategy == 0;
  if (k == kNumBuckets - 1 && hub && g->hub_jobs > 0)
    launch_hub(s, mode, A, g->d_jobs, g->hub_jobs, R.counters + mode, R.worklist);
  else if (cfg && cfg->lanes[k] > 0)
    launch_edges_lanes(s, mode, cfg->lanes[k], A);
  else
    launch_edges(s, mode, k, A);
}

// Enqueues Algorithm 1 (with Algorithms 2 and 3) on g: kernel launches only
// (no memset, copy or synchronisation), so that it can be captured in a HIP
// graph.  Per-graph parameters come from A.gid/gp/gq/gmu when set.
void scan::enqueue_clustering(scan_graph* g, EdgeArgs& A, int32_t* d_labels, uint8_t* d_roles,
                              const int32_t* gbase, hipStream_t s, bool timing, const RunConfig* cfg,
                              const RunState* state, hipEvent_t* events) {
  const int n = g->n;
  const int64_t m = g->m;
  const RunState R = state ? *state : graph_state(g);
  hipEvent_t* ev = events ? events : g->ev;
  auto mark = [&](int k) {
    if (timing) (void)hipEventRecord(ev[k], s);
  };
  A.rp = g->d_rp;
  A.ci = g->d_ci;
  A.hci = g->d_hci ? g->d_hci : g->d_ci;
  A.edges = g->d_edges;
  A.wtab = g->d_wtab;
  A.edeg = g->d_edeg;
  A.hsamp = g->d_hsamp;
  A.state = R.state;
  A.lower = R.lower;
  A.upper = R.upper;
  A.role = R.role;
  A.parent = R.parent;
  A.label = R.label;
  A.counts = nullptr;
  A.edge_counts = nullptr;
  A.stats = R.stats;
  // Events: 0 start, then the end of each phase; the cores phase also marks
  // the end of each bucket (slots SCAN_NUM_PHASES + 1 + k).
  mark(0);
  launch_zero_u64(s, R.stats, ST_COUNT);
  launch_init(s, n, g->d_rp, A.mu, R.lower, R.upper, R.role, R.parent, A.gid, A.gmu);
  launch_fill_u8(s, R.state, m, SIM_UNK);
  launch_zero_u64(s, R.counters, kCounters);
  mark(1);
  for (int k = 0; k < kNumBuckets; ++k) {
    launch_bucket(g, s, MODE_CORES, k, A, R, cfg);
    mark(SCAN_NUM_PHASES + 1 + k);
  }
  mark(2);
  launch_finalize_roles(s, n, A.mu, R.lower, R.role, A.gid, A.gmu, R.counters + 4);
  A.ncores = R.counters + 4;
  mark(3);
  launch_hook(s, m, g->d_edges, R.state, R.role, R.parent);
  mark(4);
  for (int k = 0; k < kNumBuckets; ++k) launch_bucket(g, s, MODE_MERGE, k, A, R, cfg);
  mark(5);
  launch_flatten(s, n, R.role, R.parent, R.label);
  mark(6);
  for (int k = 0; k < kNumBuckets; ++k) launch_bucket(g, s, MODE_ATTACH, k, A, R, cfg);
  mark(7);
  const int32_t split = g->opts.hub_outlier ? 1 : 0;
  if (split) {  // Def 2.7; the cores pass's upper bounds are no longer needed
    launch_fill_i32(s, R.upper, n, -1);
    launch_hub_outlier_edges(s, m, g->d_edges, R.label, R.upper, R.role);
  }
  launch_output(s, n, R.role, R.label, d_labels, d_roles, split, A.gid, gbase);
  mark(8);
}

// Reads the statistics counters and event times of the last enqueued run.
void scan::set_last(scan_graph* g, const scan_stats& L) {
  std::lock_guard<std::mutex> lk(g->stats_lock);
  g->last = L;
}

int scan::collect_stats(scan_graph* g, hipStream_t s, bool timing) {
  return collect_stats(g, s, timing, graph_state(g), g->ev);
}

int scan::collect_stats(scan_graph* g, hipStream_t s, bool timing, const RunState& R, hipEvent_t* ev) {
  const int64_t m = g->m;
  HIP_TRY(hipGetLastError(), "kernel launch");
  unsigned long long st[ST_COUNT];
  HIP_TRY(hipMemcpyAsync(st, R.stats, sizeof(st), hipMemcpyDeviceToHost, s), "stats copy");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  scan_stats L;
  memset(&L, 0, sizeof(L));
  L.edges = m;
  for (int k = 0; k < kNumBuckets; ++k) {
    L.bucket_edges[k] = g->bucket_off[k + 1] - g->bucket_off[k];
    L.cores_bucket_evaluated[k] = (int64_t)st[ST_BUCKET_EVAL + k];
    L.cores_bucket_probes[k] = (int64_t)st[ST_BUCKET_PROBES + k];
  }
  L.group_split = (int64_t)st[ST_GROUP_SPLIT];
  const int phase_of_mode[4] = {SCAN_PHASE_CORES, SCAN_PHASE_MERGE, SCAN_PHASE_ATTACH, SCAN_PHASE_CORES};
  for (int md = 0; md < 3; ++md) {
    L.evaluated[phase_of_mode[md]] = (int64_t)st[ST_EVAL + md];
    L.bounded[phase_of_mode[md]] = (int64_t)st[ST_BOUND + md];
    L.probes[phase_of_mode[md]] = (int64_t)st[ST_PROBES + md];
  }
  if (timing) {
    float ms = 0;
    for (int ph = 0; ph < SCAN_NUM_PHASES; ++ph) {
      hipEventElapsedTime(&ms, ev[ph], ev[ph + 1]);
      L.ms_phase[ph] = ms;
    }
    hipEventElapsedTime(&ms, ev[0], ev[SCAN_NUM_PHASES]);
    L.ms_total = ms;
    for (int k = 0; k < kNumBuckets; ++k) {
      hipEventElapsedTime(&ms, ev[k == 0 ? 1 : SCAN_NUM_PHASES + k], ev[SCAN_NUM_PHASES + 1 + k]);
      L.ms_cores_bucket[k] = ms;
    }
  }
  set_last(g, L);
  return SCAN_OK;
}

uint64_t scan::graph_device_bytes(const scan_graph* g) {
  if (g->partitioned) return 0;
  const uint64_t n = (uint64_t)g->n, nnz = (uint64_t)g->nnz;
  uint64_t b = graph_layout_bytes(g);
  if (g->d_out_labels) b += 5 * n;
  if (g->d_counts) b += 4 * nnz;
  return b + g->extra_bytes.load();
}

uint64_t scan::graph_layout_bytes(const scan_graph* g) {
  const uint64_t n = (uint64_t)g->n, nnz = (uint64_t)g->nnz, m = (uint64_t)g->m;
  const uint64_t b6 = (uint64_t)(g->bucket_off[kNumBuckets] - g->bucket_off[kNumBuckets - 1]);
  uint64_t b = 8 * (n + 1) + 4 * (nnz + kColPad) + 8 * m + (g->d_edeg ? 8 * m : 0) + sizeof(HubJob) * (uint64_t)g->hub_jobs + 4 * b6 +
               4 * (uint64_t)g->wtab_entries;
  if (g->d_hci) b += 4 * (nnz + kColPad);
  if (g->d_hsamp) b += 4 * (uint64_t)sample_lines((int64_t)nnz);
  b += 17 * n + m + 8ull * ST_COUNT + 8ull * kCounters;  // per-run state
  return b;
}

int scan::check_params(const scan_graph* g, int64_t& p, int64_t& q, int32_t mu) {
  if (p < 1 || q < p) return fail(SCAN_E_INVAL, "eps must satisfy 1 <= eps_num <= eps_den (got %lld/%lld)",
                                  (long long)p, (long long)q);
  if (mu < 2) return fail(SCAN_E_INVAL, "mu must be >= 2 (got %d)", mu);
  if (g->opts.strategy < 0 || g->opts.strategy > 1) return fail(SCAN_E_INVAL, "unknown strategy %d", g->opts.strategy);
  const int64_t gd = gcd64(p, q);
  p /= gd;
  q /= gd;
  if ((unsigned __int128)q * (unsigned __int128)((uint64_t)g->max_degree + 1) >= ((unsigned __int128)1 << 32))
    return fail(SCAN_E_RANGE, "eps denominator %lld with max degree %d exceeds the 64-bit test range",
                (long long)q, g->max_degree);
  return SCAN_OK;
}

namespace {

// Validates eps and mu and runs the in-memory or partitioned clustering.
int run_clustering(scan_graph* g, int64_t p, int64_t q, int32_t mu, int32_t* d_labels,
                   uint8_t* d_roles, hipStream_t s) {
  const int rc = check_params(g, p, q, mu);
  if (rc != SCAN_OK) return rc;
  if (g->partitioned) return part_run(g, (uint64_t)p, (uint64_t)q, mu, d_labels, d_roles, s);
  EdgeArgs A{};
  A.p = (uint64_t)p;
  A.q = (uint64_t)q;
  A.mu = mu;
  A.pruning = g->opts.pruning;
  const bool timing = g->opts.timing != 0;
  enqueue_clustering(g, A, d_labels, d_roles, nullptr, s, timing, nullptr);
  return collect_stats(g, s, timing);
}

// Device bytes of one extra buffer set (per-run state, and staging for host
// outputs).
uint64_t extra_run_bytes(const scan_graph* g, bool host) {
  const uint64_t n = (uint64_t)g->n, m = (uint64_t)g->m;
  const uint64_t b6 = (uint64_t)(g->bucket_off[kNumBuckets] - g->bucket_off[kNumBuckets - 1]);
  return 17 * n + m + 8ull * ST_COUNT + 8ull * kCounters + 4 * b6 + (host ? 5 * n : 0);
}

// Allocates what x lacks; the bytes were reserved when x was taken.
hipError_t alloc_extra(scan_graph* g, ExtraRun& x, bool host) {
  hipError_t e = hipSuccess;
  auto get = [&](auto** p, int64_t count) {
    if (e == hipSuccess && !*p) e = hipMalloc((void**)p, sizeof(**p) * (size_t)(count > 0 ? count : 1));
  };
  const int64_t n = g->n, m = g->m;
  get(&x.R.lower, n);
  get(&x.R.upper, n);
  get(&x.R.role, n);
  get(&x.R.parent, n);
  get(&x.R.label, n);
  get(&x.R.state, m);
  get(&x.R.stats, ST_COUNT);
  get(&x.R.counters, kCounters);
  get(&x.R.worklist, g->bucket_off[kNumBuckets] - g->bucket_off[kNumBuckets - 1]);
  if (host) {
    get(&x.d_out_labels, n);
    get(&x.d_out_roles, n);
  }
  if (e == hipSuccess && !x.stream) e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking);
  for (auto& ev : x.ev)
    if (e == hipSuccess && !ev) e = hipEventCreate(&ev);
  return e;
}

// For a call that found the graph's own per-run buffers in use: a free buffer
// set of the graph's pool (one with staging when the outputs go to host
// memory), or a new one, its device bytes reserved at once.  Null when the
// call should wait for the graph's own buffers instead: on a partitioned
// graph (its streaming buffers are single), or when a graph created under a
// device budget has no room for another set, or when the calling thread's
// current device is not the graph's (the set would be allocated there).
ExtraRun* take_extra(scan_graph* g, bool host) {
  if (g->partitioned) return nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device) return nullptr;
  std::lock_guard<std::mutex> lk(g->pool_lock);
  ExtraRun* x = nullptr;
  for (auto& c : g->extra)
    if (!c->busy && (!x || (host && c->d_out_labels && !x->d_out_labels))) x = c.get();
  const uint64_t want = extra_run_bytes(g, host || (x && x->d_out_labels));
  const uint64_t more = x ? want - std::min(want, x->bytes) : want;
  const uint64_t budget = g->opts.device_budget_bytes;
  // the graph's own staging (host outputs, counts) is counted as if allocated:
  // the call holding the graph's buffers may be allocating it right now
  const uint64_t held = graph_layout_bytes(g) + 5 * (uint64_t)g->n + 4 * (uint64_t)g->nnz + g->extra_bytes.load();
  if (budget && more && held + more > budget) return nullptr;
  if (!x) {
    g->extra.push_back(std::make_unique<ExtraRun>());
    x = g->extra.back().get();
  }
  g->extra_bytes += more;
  x->bytes += more;
  x->busy = true;
  return x;
}

// A clustering call on buffer set x of the graph's pool, on x's own stream
// (or the caller's), beside the call that holds the graph's own buffers.
// Host outputs go through x's staging.
int run_extra(scan_graph* g, ExtraRun* x, int64_t p, int64_t q, int32_t mu, int32_t* d_labels,
              uint8_t* d_roles, int32_t* h_labels, uint8_t* h_roles, hipStream_t caller) {
  auto give_back = [&]() {
    std::lock_guard<std::mutex> lk(g->pool_lock);
    x->busy = false;
  };
  int rc = check_params(g, p, q, mu);
  if (rc != SCAN_OK) {
    give_back();
    return rc;
  }
  const bool host = h_labels != nullptr;
  const hipError_t e = alloc_extra(g, *x, host);
  if (e != hipSuccess) {
    give_back();
    return fail_hip(e, "buffers for an overlapping call");
  }
  hipStream_t s = caller ? caller : x->stream;
  EdgeArgs A{};
  A.p = (uint64_t)p;
  A.q = (uint64_t)q;
  A.mu = mu;
  A.pruning = g->opts.pruning;
  const bool timing = g->opts.timing != 0;
  enqueue_clustering(g, A, host ? x->d_out_labels : d_labels, host ? x->d_out_roles : d_roles, nullptr, s, timing,
                     nullptr, &x->R, x->ev);
  rc = collect_stats(g, s, timing, x->R, x->ev);
  if (rc == SCAN_OK && host && g->n > 0) {
    hipError_t c = hipMemcpyAsync(h_labels, x->d_out_labels, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToHost, s);
    if (c == hipSuccess) c = hipMemcpyAsync(h_roles, x->d_out_roles, (size_t)g->n, hipMemcpyDeviceToHost, s);
    if (c == hipSuccess) c = hipStreamSynchronize(s);
    if (c != hipSuccess) rc = fail_hip(c, "copy outputs");
  }
  give_back();
  return rc;
}

}  // namespace

int scan::run_counts(scan_graph* g, int32_t* d_counts_arc, int32_t* d_counts_edge, hipStream_t s) {
  const bool timing = g->opts.timing != 0;
  HIP_TRY(hipMemsetAsync(g->d_stats, 0, sizeof(unsigned long long) * ST_COUNT, s), "hipMemsetAsync");
  launch_zero_u64(s, g->d_counters, kCounters);
  if (timing) hipEventRecord(g->ev[0], s);
  EdgeArgs A{};
  A.rp = g->d_rp;
  A.ci = g->d_ci;
  A.hci = g->d_hci ? g->d_hci : g->d_ci;
  A.edges = g->d_edges;
  A.wtab = g->d_wtab;
  A.hsamp = g->d_hsamp;
  A.counts = d_counts_arc;
  A.edge_counts = d_counts_edge;
  A.stats = g->d_stats;
  A.p = 1;
  A.q = 1;
  A.mu = 2;
  A.pruning = 0;
  const RunState R = graph_state(g);
  for (int k = 0; k < kNumBuckets; ++k) launch_bucket(g, s, MODE_COUNTS, k, A, R);
  if (timing) hipEventRecord(g->ev[1], s);
  HIP_TRY(hipGetLastError(), "kernel launch");
  unsigned long long st[ST_COUNT];
  HIP_TRY(hipMemcpyAsync(st, g->d_stats, sizeof(st), hipMemcpyDeviceToHost, s), "stats copy");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  scan_stats L;
  memset(&L, 0, sizeof(L));
  L.edges = g->m;
  L.evaluated[SCAN_PHASE_CORES] = (int64_t)st[ST_EVAL + MODE_COUNTS];
  L.group_split = (int64_t)st[ST_GROUP_SPLIT];
  L.probes[SCAN_PHASE_CORES] = (int64_t)st[ST_PROBES + MODE_COUNTS];
  for (int k = 0; k < kNumBuckets; ++k) L.bucket_edges[k] = g->bucket_off[k + 1] - g->bucket_off[k];
  if (timing) {
    float ms = 0;
    hipEventElapsedTime(&ms, g->ev[0], g->ev[1]);
    L.ms_total = ms;
    L.ms_phase[SCAN_PHASE_CORES] = ms;
  }
  set_last(g, L);
  return SCAN_OK;
}

extern "C" {

void scan_opts_default(scan_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->validate = 1;
  o->pruning = 1;
  o->hub_ranked = 1;
}

const char* scan_last_error(void) { return g_error.c_str(); }

const char* scan_version(void) { return "scan-mi355x 0.1 (gfx950)"; }

int64_t scan_eps_threshold(int64_t p, int64_t q, int64_t a, int64_t b) {
  if (p < 1 || q < p || a < 1 || b < 1) return -1;
  const int64_t mx = a > b ? a : b;
  if ((unsigned __int128)q * (unsigned __int128)mx >= ((unsigned __int128)1 << 32)) return -1;
  return (int64_t)closed_needed((uint64_t)p, (uint64_t)q, (uint64_t)a, (uint64_t)b);
}

int scan_graph_create(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      const scan_opts* opts, scan_graph** out) {
  g_error.clear();
  if (!out) return fail(SCAN_E_INVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || nnz < 0) return fail(SCAN_E_INVAL, "n and nnz must be non-negative");
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(SCAN_E_INVAL, "row_ptr/col_idx is NULL");
  if (row_ptr[0] != 0 || row_ptr[n] != nnz)
    return fail(SCAN_E_GRAPH, "row_ptr must start at 0 and end at nnz");
  if (nnz % 2 != 0) return fail(SCAN_E_GRAPH, "an undirected CSR has an even number of arcs");
  scan_graph* g = new (std::nothrow) scan_graph();
  if (!g) return fail(SCAN_E_NOMEM, "host allocation failed");
  if (opts) g->opts = *opts;
  else scan_opts_default(&g->opts);
  g->n = n;
  g->nnz = nnz;
  int rc = SCAN_OK;
  hipError_t e;
  LayoutResult lay{};
  std::vector<HubJob> jobs;
  std::vector<uint32_t> wtab;
  std::vector<int32_t> ranked;
#define CTRY(call, what)                         \
  do {                                           \
    e = (call);                                  \
    if (e != hipSuccess) { rc = fail_hip(e, what); goto error; } \
  } while (0)
  CTRY(hipGetDevice(&g->device), "hipGetDevice");
  (void)hub_grid_blocks();
  if (g->opts.hip_stream) {
    g->stream = (hipStream_t)g->opts.hip_stream;
  } else {
    CTRY(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking), "hipStreamCreate");
    g->own_stream = true;
  }
  if (g->opts.device_budget_bytes && inmemory_footprint(n, nnz, g->opts.hub_ranked != 0) > g->opts.device_budget_bytes) {
    // Partition-based path: the CSR stays in pinned host memory.
    rc = part_validate(n, nnz, row_ptr, col_idx, g->opts.validate != 0);
    if (rc != SCAN_OK) goto error;
    for (int32_t v = 0; v < n; ++v)
      g->max_degree = (int32_t)std::max<int64_t>(g->max_degree, row_ptr[v + 1] - row_ptr[v]);
    rc = part_create(g, row_ptr, col_idx, g->opts.device_budget_bytes);
    if (rc != SCAN_OK) goto error;
    CTRY(dalloc(&g->d_rp, (int64_t)n + 1), "hipMalloc row_ptr");
    CTRY(hipMemcpyAsync(g->d_rp, row_ptr, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, g->stream),
         "copy row_ptr");
    CTRY(dalloc(&g->d_lower, n), "hipMalloc");
    CTRY(dalloc(&g->d_upper, n), "hipMalloc");
    CTRY(dalloc(&g->d_role, n), "hipMalloc");
    CTRY(dalloc(&g->d_parent, n), "hipMalloc");
    CTRY(dalloc(&g->d_label, n), "hipMalloc");
    CTRY(dalloc(&g->d_stats, ST_COUNT), "hipMalloc");
    CTRY(dalloc(&g->d_counters, kCounters), "hipMalloc");
    for (auto& ev : g->ev) CTRY(hipEventCreate(&ev), "hipEventCreate");
    CTRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    *out = g;
    return SCAN_OK;
  }
  CTRY(dalloc(&g->d_rp, (int64_t)n + 1), "hipMalloc row_ptr");
  CTRY(dalloc(&g->d_ci, nnz + kColPad), "hipMalloc col_idx");
  CTRY(hipMemcpyAsync(g->d_rp, row_ptr, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice, g->stream),
       "copy row_ptr");
  if (nnz > 0)
    CTRY(hipMemcpyAsync(g->d_ci, col_idx, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, g->stream),
         "copy col_idx");
  CTRY(build_layout(g->stream, n, nnz, row_ptr, col_idx, g->d_rp, g->d_ci, g->opts.validate, &g->d_edges,
                    &jobs, &lay), "layout");
  if (lay.error) {
    rc = fail(SCAN_E_GRAPH, "CSR rejected (flags 0x%x: 1 offsets, 2 id range, 4 self-loop, "
              "8 row order/duplicate, 16 missing reverse arc, 32 inconsistent layout)", lay.error);
    goto error;
  }
  g->max_degree = lay.max_degree;
  g->hub_jobs = lay.hub_jobs;
  if (g->opts.hub_ranked && n > kHubBitmapBits && lay.hub_jobs > 0) {
    CTRY(dalloc(&g->d_hci, nnz + kColPad), "hipMalloc ranked rows");
    CTRY(build_ranked_rows(g->stream, n, nnz, row_ptr, col_idx, g->d_hci, &ranked), "ranked rows");
  }
  if (!jobs.empty()) {
    // LDS-hash windows of every hub row, from the rows the kernel reads
    assign_hub_windows(jobs, row_ptr, g->d_hci ? ranked.data() : col_idx, wtab);
    std::vector<int32_t>().swap(ranked);
    CTRY(dalloc(&g->d_jobs, (int64_t)jobs.size()), "hipMalloc jobs");
    CTRY(dalloc(&g->d_wtab, (int64_t)wtab.size()), "hipMalloc windows");
    CTRY(hipMemcpyAsync(g->d_jobs, jobs.data(), sizeof(HubJob) * jobs.size(), hipMemcpyHostToDevice, g->stream),
         "copy jobs");
    CTRY(hipMemcpyAsync(g->d_wtab, wtab.data(), sizeof(uint32_t) * wtab.size(), hipMemcpyHostToDevice, g->stream),
         "copy windows");
    CTRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    g->wtab_entries = (int64_t)wtab.size();
    // the first id of every 128-byte line of those rows
    CTRY(dalloc(&g->d_hsamp, sample_lines(nnz)), "hipMalloc line samples");
    launch_line_samples(g->stream, sample_lines(nnz), g->d_hci ? g->d_hci : g->d_ci, g->d_hsamp);
    CTRY(hipGetLastError(), "line samples");
  }
  for (int k = 0; k <= kNumBuckets; ++k) g->bucket_off[k] = lay.bucket_off[k];
  g->m = lay.bucket_off[kNumBuckets];
  if (g->opts.validate && g->m * 2 != nnz) {
    rc = fail(SCAN_E_GRAPH, "edge count %lld does not match nnz/2", (long long)g->m);
    goto error;
  }
  CTRY(dalloc(&g->d_edeg, g->m), "hipMalloc edge degrees");
  launch_edge_degrees(g->stream, g->m, g->d_rp, g->d_edges, g->d_edeg);
  CTRY(hipGetLastError(), "edge degrees");
  CTRY(dalloc(&g->d_lower, n), "hipMalloc");
  CTRY(dalloc(&g->d_upper, n), "hipMalloc");
  CTRY(dalloc(&g->d_role, n), "hipMalloc");
  CTRY(dalloc(&g->d_parent, n), "hipMalloc");
  CTRY(dalloc(&g->d_label, n), "hipMalloc");
  CTRY(dalloc(&g->d_state, g->m), "hipMalloc");
  CTRY(dalloc(&g->d_stats, ST_COUNT), "hipMalloc");
  CTRY(dalloc(&g->d_counters, kCounters), "hipMalloc");
  CTRY(dalloc(&g->d_worklist, g->bucket_off[kNumBuckets] - g->bucket_off[kNumBuckets - 1]), "hipMalloc");
  for (auto& ev : g->ev) CTRY(hipEventCreate(&ev), "hipEventCreate");
  CTRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
  *out = g;
  return SCAN_OK;
error:
  release(g);
  delete g;
#undef CTRY
  return rc;
}

int scan_graph_destroy(scan_graph* g) {
  if (!g) return SCAN_OK;
  {
    std::lock_guard<std::mutex> lk(g->lock);
    hipStreamSynchronize(g->stream);
    release(g);
  }
  delete g;
  return SCAN_OK;
}

int scan_graph_footprint(int32_t n, int64_t nnz, const scan_opts* opts, uint64_t* bytes) {
  if (n < 0 || nnz < 0 || !bytes) return fail(SCAN_E_INVAL, "n, nnz must be >= 0 and bytes non-NULL");
  scan_opts o;
  if (opts) o = *opts;
  else scan_opts_default(&o);
  *bytes = inmemory_footprint(n, nnz, o.hub_ranked != 0);
  return SCAN_OK;
}

int scan_graph_info(const scan_graph* g, int32_t* n, int64_t* nnz, int64_t* m, int32_t* max_degree) {
  if (!g) return fail(SCAN_E_INVAL, "graph is NULL");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (m) *m = g->m;
  if (max_degree) *max_degree = g->max_degree;
  return SCAN_OK;
}

int scan_run_device(scan_graph* g, int64_t eps_num, int64_t eps_den, int32_t mu, int32_t* d_labels,
                    uint8_t* d_roles, void* stream) {
  g_error.clear();
  if (!g) return fail(SCAN_E_INVAL, "graph is NULL");
  if (g->n > 0 && (!d_labels || !d_roles)) return fail(SCAN_E_INVAL, "output pointer is NULL");
  std::unique_lock<std::mutex> lk(g->lock, std::try_to_lock);
  if (!lk.owns_lock()) {
    if (ExtraRun* x = take_extra(g, false))
      return run_extra(g, x, eps_num, eps_den, mu, d_labels, d_roles, nullptr, nullptr, (hipStream_t)stream);
    lk.lock();
  }
  hipStream_t s = stream ? (hipStream_t)stream : g->stream;
  return run_clustering(g, eps_num, eps_den, mu, d_labels, d_roles, s);
}

int scan_run(scan_graph* g, int64_t eps_num, int64_t eps_den, int32_t mu, int32_t* labels,
             uint8_t* roles) {
  g_error.clear();
  if (!g) return fail(SCAN_E_INVAL, "graph is NULL");
  if (g->n > 0 && (!labels || !roles)) return fail(SCAN_E_INVAL, "output pointer is NULL");
  std::unique_lock<std::mutex> lk(g->lock, std::try_to_lock);
  if (!lk.owns_lock()) {
    if (ExtraRun* x = take_extra(g, true))
      return run_extra(g, x, eps_num, eps_den, mu, nullptr, nullptr, labels, roles, nullptr);
    lk.lock();
  }
  if (!g->d_out_labels) {
    HIP_TRY(dalloc(&g->d_out_labels, g->n), "hipMalloc");
    HIP_TRY(dalloc(&g->d_out_roles, g->n), "hipMalloc");
  }
  int rc = run_clustering(g, eps_num, eps_den, mu, g->d_out_labels, g->d_out_roles, g->stream);
  if (rc != SCAN_OK) return rc;
  if (g->n > 0) {
    HIP_TRY(hipMemcpyAsync(labels, g->d_out_labels, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToHost,
                           g->stream), "copy labels");
    HIP_TRY(hipMemcpyAsync(roles, g->d_out_roles, (size_t)g->n, hipMemcpyDeviceToHost, g->stream),
            "copy roles");
    HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
  }
  return SCAN_OK;
}

int scan_similarity_device(scan_graph* g, int32_t* d_counts, void* stream) {
  g_error.clear();
  if (!g) return fail(SCAN_E_INVAL, "graph is NULL");
  if (g->nnz > 0 && !d_counts) return fail(SCAN_E_INVAL, "counts is NULL");
  std::lock_guard<std::mutex> lk(g->lock);
  if (g->partitioned) return fail(SCAN_E_INVAL, "device output is not available on the partitioned path");
  hipStream_t s = stream ? (hipStream_t)stream : g->stream;
  return run_counts(g, d_counts, nullptr, s);
}

int scan_similarity(scan_graph* g, int32_t* counts) {
  g_error.clear();
  if (!g) return fail(SCAN_E_INVAL, "graph is NULL");
  if (g->nnz > 0 && !counts) return fail(SCAN_E_INVAL, "counts is NULL");
  std::lock_guard<std::mutex> lk(g->lock);
  if (g->nnz == 0) return SCAN_OK;
  if (g->partitioned) return part_counts(g, counts, g->stream);
  if (!g->d_counts) HIP_TRY(dalloc(&g->d_counts, g->nnz), "hipMalloc counts");
  int rc = run_counts(g, g->d_counts, nullptr, g->stream);
  if (rc != SCAN_OK) return rc;
  HIP_TRY(hipMemcpyAsync(counts, g->d_counts, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToHost,
                         g->stream), "copy counts");
  HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
  return SCAN_OK;
}

int scan_last_stats(const scan_graph* g, scan_stats* out) {
  if (!g || !out) return fail(SCAN_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g->stats_lock);
  *out = g->last;
  return SCAN_OK;
}

int scan_graph_device_bytes(const scan_graph* g, uint64_t* bytes) {
  if (!g || !bytes) return fail(SCAN_E_INVAL, "NULL argument");
  *bytes = graph_device_bytes(g);
  return SCAN_OK;
}

int scan_device_alloc(uint64_t bytes, void** out) {
  if (!out) return fail(SCAN_E_INVAL, "out is NULL");
  HIP_TRY(hipMalloc(out, bytes ? bytes : 1), "hipMalloc");
  return SCAN_OK;
}

int scan_device_free(void* ptr) {
  if (ptr) HIP_TRY(hipFree(ptr), "hipFree");
  return SCAN_OK;
}

int scan_memcpy_d2h(void* dst, const void* src, uint64_t bytes) {
  if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "hipMemcpy D2H");
  return SCAN_OK;
}

int scan_memcpy_h2d(void* dst, const void* src, uint64_t bytes) {
  if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy H2D");
  return SCAN_OK;
}

int scan_device_copy(void* dst, const void* src, uint64_t bytes, int32_t iters, float* avg_ms) {
  if (!dst || !src || (bytes & 15) || iters < 1 || (((uintptr_t)dst | (uintptr_t)src) & 15))
    return fail(SCAN_E_INVAL, "scan_device_copy: bytes must be a multiple of 16, pointers 16-byte aligned, iters >= 1");
  const uintptr_t d = (uintptr_t)dst, sp = (uintptr_t)src;
  if (bytes && d < sp + bytes && sp < d + bytes) return fail(SCAN_E_INVAL, "scan_device_copy: buffers overlap");
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  int rc = SCAN_OK;
  float ms = 0.f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = fail(SCAN_E_DEVICE, "hipEventCreate failed");
  } else {
    (void)hipEventRecord(e0, s);
    for (int32_t i = 0; i < iters; ++i) launch_copy16(s, src, dst, (int64_t)(bytes / 16));
    (void)hipEventRecord(e1, s);
    hipError_t err = hipStreamSynchronize(s);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) rc = fail_hip(err, "scan_device_copy");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (rc == SCAN_OK && avg_ms) *avg_ms = ms / (float)iters;
  return rc;
}

int scan_device_read(const void* src, uint64_t bytes, int32_t iters, float* avg_ms) {
  if (!src || (bytes & 15) || iters < 1 || ((uintptr_t)src & 15))
    return fail(SCAN_E_INVAL, "scan_device_read: bytes must be a multiple of 16, src 16-byte aligned, iters >= 1");
  uint32_t* sink = nullptr;
  HIP_TRY(hipMalloc((void**)&sink, sizeof(uint32_t) * (size_t)read16_sink_words()), "hipMalloc");
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SCAN_OK;
  float ms = 0.f;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    rc = fail(SCAN_E_DEVICE, "scan_device_read: stream or event creation failed");
  } else {
    (void)hipEventRecord(e0, s);
    for (int32_t i = 0; i < iters; ++i) launch_read16(s, src, (int64_t)(bytes / 16), sink);
    (void)hipEventRecord(e1, s);
    hipError_t err = hipStreamSynchronize(s);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) rc = fail_hip(err, "scan_device_read");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(sink);
  if (rc == SCAN_OK && avg_ms) *avg_ms = ms / (float)iters;
  return rc;
}

int scan_h2d_rate(uint64_t bytes, int32_t iters, double* h2d_bps) {
  if (!bytes || iters < 1 || !h2d_bps) return fail(SCAN_E_INVAL, "scan_h2d_rate: bytes > 0, iters >= 1, h2d_bps required");
  void* h = nullptr;
  void* d = nullptr;
  if (hipHostMalloc(&h, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SCAN_E_NOMEM, "scan_h2d_rate: hipHostMalloc of %llu bytes failed", (unsigned long long)bytes);
  }
  if (hipMalloc(&d, bytes) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(h);
    return fail(SCAN_E_NOMEM, "scan_h2d_rate: hipMalloc of %llu bytes failed", (unsigned long long)bytes);
  }
  memset(h, 1, bytes);
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SCAN_OK;
  float ms = 0.f;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    rc = fail(SCAN_E_DEVICE, "scan_h2d_rate: stream or event creation failed");
  } else {
    hipError_t err = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);  // warm-up
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int32_t i = 0; i < iters && err == hipSuccess; ++i) err = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) rc = fail_hip(err, "scan_h2d_rate");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(d);
  (void)hipHostFree(h);
  if (rc == SCAN_OK) *h2d_bps = ms > 0 ? (double)bytes * iters / (ms * 1e-3) : 0.0;
  return rc;
}

}  // extern "C"
