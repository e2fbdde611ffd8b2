// Batched clustering of many independent graphs in one go.
//
// The graphs are packed into one disjoint union (global id = vertex offset of
// the graph + local id).  SCAN on a disjoint union is SCAN on each graph, so
// one layout and one pipeline serve the whole batch; each vertex carries its
// graph id, through which every kernel looks up that graph's eps = p/q and mu.
// Labels (minimum core ids) are turned back into graph-local ids on output.
//
// The pipeline for the whole batch is captured once into a HIP graph and
// replayed (hipGraphLaunch), so a batch run is a single launch from the host
// regardless of the number of graphs.  An autotuner chooses, per degree
// bucket, the lane-group width of the group kernel and whether the last
// bucket uses the LDS-hash kernel, by timing the candidates on the batch
// itself; choices can be cached in a file named by SCAN_AUTOTUNE_CACHE.
#include "graph.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

struct scan_batch_graph {
  scan_graph* g = nullptr;
  int32_t G = 0;
  int32_t N = 0;
  int32_t* d_gid = nullptr;
  uint64_t* d_gp = nullptr;
  uint64_t* d_gq = nullptr;
  int32_t* d_gmu = nullptr;
  int32_t* d_gbase = nullptr;
  int32_t* d_labels = nullptr;
  uint8_t* d_roles = nullptr;
  RunConfig cfg{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::mutex lock;
};

namespace {

void batch_release(scan_batch_graph* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  void* d[] = {B->d_gid, B->d_gp, B->d_gq, B->d_gmu, B->d_gbase, B->d_labels, B->d_roles};
  for (void* p : d)
    if (p) (void)hipFree(p);
  if (B->g) scan_graph_destroy(B->g);
}

EdgeArgs batch_args(scan_batch_graph* B) {
  EdgeArgs A{};
  A.p = 1;
  A.q = 1;
  A.mu = 2;
  A.pruning = B->g->opts.pruning;
  A.gid = B->d_gid;
  A.gp = B->d_gp;
  A.gq = B->d_gq;
  A.gmu = B->d_gmu;
  return A;
}

int default_lanes(int k) {
  static const int d[kNumBuckets] = {4, 8, 16, 32, 64, 64, 64};
  return d[k];
}

std::string tune_key(const scan_graph* g) {
  std::string k = std::to_string(g->n) + ":" + std::to_string(g->m);
  for (int b = 0; b < kNumBuckets; ++b) k += ":" + std::to_string(g->bucket_off[b + 1] - g->bucket_off[b]);
  return k;
}

bool tune_cache_read(const std::string& key, RunConfig& cfg) {
  const char* path = getenv("SCAN_AUTOTUNE_CACHE");
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char kbuf[512];
  int l[kNumBuckets], hub;
  bool found = false;
  while (fscanf(f, "%511s %d %d %d %d %d %d %d %d", kbuf, &l[0], &l[1], &l[2], &l[3], &l[4], &l[5], &l[6], &hub) ==
         9) {
    if (key == kbuf) {
      for (int b = 0; b < kNumBuckets; ++b) cfg.lanes[b] = l[b];
      cfg.hub = hub != 0;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void tune_cache_write(const std::string& key, const RunConfig& cfg) {
  const char* path = getenv("SCAN_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s", key.c_str());
  for (int b = 0; b < kNumBuckets; ++b) fprintf(f, " %d", cfg.lanes[b]);
  fprintf(f, " %d\n", cfg.hub ? 1 : 0);
  fclose(f);
}

// Device time of bucket k's cores-pass kernel under cfg (median of 3 runs).
double time_bucket(scan_batch_graph* B, const RunConfig& cfg, int k) {
  scan_graph* g = B->g;
  double t[3];
  for (int r = 0; r < 4; ++r) {
    EdgeArgs A = batch_args(B);
    enqueue_clustering(g, A, B->d_labels, B->d_roles, B->d_gbase, g->stream, true, &cfg);
    if (collect_stats(g, g->stream, true) != SCAN_OK) return 1e30;
    if (r > 0) t[r - 1] = g->last.ms_cores_bucket[k];
  }
  std::sort(t, t + 3);
  return t[1];
}

// Greedy per bucket: lane widths around the default for the group-kernel
// buckets, and LDS-hash versus group kernel for the last bucket.
void autotune(scan_batch_graph* B) {
  scan_graph* g = B->g;
  const std::string key = tune_key(g);
  if (tune_cache_read(key, B->cfg)) return;
  for (int k = 0; k < kNumBuckets; ++k) {
    if (g->bucket_off[k + 1] == g->bucket_off[k]) continue;
    if (k == kNumBuckets - 1) {
      if (g->hub_jobs == 0) continue;
      RunConfig a = B->cfg, b = B->cfg;
      a.hub = true;
      b.hub = false;
      b.lanes[k] = 64;
      B->cfg = time_bucket(B, a, k) <= time_bucket(B, b, k) ? a : b;
      continue;
    }
    const int d = default_lanes(k);
    int cand[3] = {d / 2, d, d * 2};
    double best = 1e30;
    int best_l = d;
    for (int c : cand) {
      if (c < 4 || c > 64) continue;
      RunConfig x = B->cfg;
      x.lanes[k] = c;
      const double ms = time_bucket(B, x, k);
      if (ms < best) {
        best = ms;
        best_l = c;
      }
    }
    B->cfg.lanes[k] = best_l;
  }
  tune_cache_write(key, B->cfg);
}

int capture(scan_batch_graph* B) {
  scan_graph* g = B->g;
  hipStream_t s = g->stream;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  EdgeArgs A = batch_args(B);
  enqueue_clustering(g, A, B->d_labels, B->d_roles, B->d_gbase, s, false, &B->cfg);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
  B->graph = graph;
  HIP_TRY(hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  return SCAN_OK;
}

}  // namespace

extern "C" {

int scan_batch_create(const scan_batch* b, const scan_opts* opts, scan_batch_graph** out) {
  if (!b || !out) return fail(SCAN_E_INVAL, "NULL argument");
  *out = nullptr;
  const int32_t G = b->num_graphs;
  if (G < 0 || !b->vtx_off || !b->arc_off || (G > 0 && (!b->row_ptr || !b->eps_num || !b->eps_den || !b->mu)))
    return fail(SCAN_E_INVAL, "bad batch description");
  if (b->vtx_off[0] != 0 || b->arc_off[0] != 0) return fail(SCAN_E_INVAL, "offsets must start at 0");
  for (int32_t k = 0; k < G; ++k) {
    if (b->vtx_off[k + 1] < b->vtx_off[k] || b->arc_off[k + 1] < b->arc_off[k])
      return fail(SCAN_E_INVAL, "offsets must be non-decreasing");
    if (b->eps_num[k] < 1 || b->eps_den[k] < b->eps_num[k])
      return fail(SCAN_E_INVAL, "graph %d: eps must satisfy 1 <= eps_num <= eps_den", k);
    if (b->mu[k] < 2) return fail(SCAN_E_INVAL, "graph %d: mu must be >= 2", k);
  }
  const int64_t N64 = b->vtx_off[G], nnz = b->arc_off[G];
  if (N64 > 0x7fffffff) return fail(SCAN_E_INVAL, "batch has more than 2^31 - 1 vertices");
  if (nnz > 0 && !b->col_idx) return fail(SCAN_E_INVAL, "col_idx is NULL");
  const int32_t N = (int32_t)N64;
  // disjoint union, host side
  std::vector<int64_t> rp((size_t)N + 1);
  std::vector<int32_t> ci((size_t)(nnz > 0 ? nnz : 1));
  std::vector<int32_t> gid((size_t)(N > 0 ? N : 1));
  std::vector<int32_t> gdmax((size_t)(G > 0 ? G : 1), 0);
  std::vector<int> bad((size_t)(G > 0 ? G : 1), 0);
  {
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        for (int32_t k = t; k < G; k += nth) {
          const int64_t v0 = b->vtx_off[k], nk = b->vtx_off[k + 1] - v0, a0 = b->arc_off[k];
          const int64_t* lrp = b->row_ptr + v0 + k;
          if (lrp[0] != 0 || lrp[nk] != b->arc_off[k + 1] - a0) { bad[(size_t)k] = 1; continue; }
          for (int64_t v = 0; v < nk; ++v) {
            rp[(size_t)(v0 + v)] = a0 + lrp[v];
            gid[(size_t)(v0 + v)] = k;
            if (lrp[v + 1] < lrp[v]) bad[(size_t)k] = 1;
            gdmax[(size_t)k] = (int32_t)std::max<int64_t>(gdmax[(size_t)k], lrp[v + 1] - lrp[v]);
          }
          for (int64_t a = a0; a < b->arc_off[k + 1]; ++a) {
            const int32_t x = b->col_idx[a];
            if (x < 0 || x >= nk) bad[(size_t)k] = 1;
            ci[(size_t)a] = (int32_t)(v0 + x);
          }
        }
      });
    for (auto& x : th) x.join();
  }
  rp[(size_t)N] = nnz;
  for (int32_t k = 0; k < G; ++k)
    if (bad[(size_t)k]) return fail(SCAN_E_GRAPH, "graph %d: row offsets or neighbour ids out of range", k);
  // per-graph parameters (eps reduced by gcd; the 64-bit test's range per graph)
  std::vector<uint64_t> gp((size_t)(G > 0 ? G : 1)), gq((size_t)(G > 0 ? G : 1));
  std::vector<int32_t> gbase((size_t)(G > 0 ? G : 1));
  for (int32_t k = 0; k < G; ++k) {
    int64_t p = b->eps_num[k], q = b->eps_den[k], x = p, y = q;
    while (y) { int64_t t = x % y; x = y; y = t; }
    p /= x;
    q /= x;
    if ((unsigned __int128)q * (unsigned __int128)((uint64_t)gdmax[(size_t)k] + 1) >= ((unsigned __int128)1 << 32))
      return fail(SCAN_E_RANGE, "graph %d: eps denominator too large for its maximum degree", k);
    gp[(size_t)k] = (uint64_t)p;
    gq[(size_t)k] = (uint64_t)q;
    gbase[(size_t)k] = (int32_t)b->vtx_off[k];
  }
  auto* B = new (std::nothrow) scan_batch_graph();
  if (!B) return fail(SCAN_E_NOMEM, "host allocation failed");
  B->G = G;
  B->N = N;
  scan_opts o;
  if (opts) o = *opts;
  else scan_opts_default(&o);
  o.device_budget_bytes = 0;
  int rc = scan_graph_create(N, nnz, rp.data(), ci.data(), &o, &B->g);
  if (rc != SCAN_OK) {
    delete B;
    return rc;
  }
  const size_t NN = (size_t)(N > 0 ? N : 1), GG = (size_t)(G > 0 ? G : 1);
  hipError_t e;
#define BTRY(x, what) do { e = (x); if (e != hipSuccess) { rc = fail_hip(e, what); goto error; } } while (0)
  BTRY(hipMalloc((void**)&B->d_gid, 4 * NN), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_gp, 8 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_gq, 8 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_gmu, 4 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_gbase, 4 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_labels, 4 * NN), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_roles, NN), "hipMalloc");
  BTRY(hipMemcpy(B->d_gid, gid.data(), 4 * NN, hipMemcpyHostToDevice), "copy");
  BTRY(hipMemcpy(B->d_gp, gp.data(), 8 * GG, hipMemcpyHostToDevice), "copy");
  BTRY(hipMemcpy(B->d_gq, gq.data(), 8 * GG, hipMemcpyHostToDevice), "copy");
  if (G > 0) BTRY(hipMemcpy(B->d_gmu, b->mu, 4 * GG, hipMemcpyHostToDevice), "copy");
  BTRY(hipMemcpy(B->d_gbase, gbase.data(), 4 * GG, hipMemcpyHostToDevice), "copy");
  for (int k = 0; k < kNumBuckets; ++k) B->cfg.lanes[k] = default_lanes(k);
  B->cfg.hub = o.strategy == 0;
  if (b->autotune) autotune(B);
  rc = capture(B);
  if (rc != SCAN_OK) goto error;
  *out = B;
  return SCAN_OK;
error:
#undef BTRY
  batch_release(B);
  delete B;
  return rc;
}

int scan_batch_run(scan_batch_graph* B, int32_t replay, int32_t* labels, uint8_t* roles) {
  if (!B) return fail(SCAN_E_INVAL, "batch is NULL");
  if (B->N > 0 && (!labels || !roles)) return fail(SCAN_E_INVAL, "output pointer is NULL");
  std::lock_guard<std::mutex> lk(B->lock);
  scan_graph* g = B->g;
  hipStream_t s = g->stream;
  if (replay) {
    HIP_TRY(hipGraphLaunch(B->exec, s), "hipGraphLaunch");
  } else {
    EdgeArgs A = batch_args(B);
    enqueue_clustering(g, A, B->d_labels, B->d_roles, B->d_gbase, s, false, &B->cfg);
  }
  int rc = collect_stats(g, s, false);
  if (rc != SCAN_OK) return rc;
  if (B->N > 0) {
    HIP_TRY(hipMemcpyAsync(labels, B->d_labels, 4 * (size_t)B->N, hipMemcpyDeviceToHost, s), "copy labels");
    HIP_TRY(hipMemcpyAsync(roles, B->d_roles, (size_t)B->N, hipMemcpyDeviceToHost, s), "copy roles");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  }
  return SCAN_OK;
}

int scan_batch_config(const scan_batch_graph* B, int32_t* lanes, int32_t* hub) {
  if (!B) return fail(SCAN_E_INVAL, "batch is NULL");
  if (lanes)
    for (int k = 0; k < kNumBuckets; ++k) lanes[k] = B->cfg.lanes[k];
  if (hub) *hub = B->cfg.hub ? 1 : 0;
  return SCAN_OK;
}

int scan_batch_stats(const scan_batch_graph* B, scan_stats* out) {
  if (!B || !out) return fail(SCAN_E_INVAL, "NULL argument");
  *out = B->g->last;
  return SCAN_OK;
}

int scan_batch_destroy(scan_batch_graph* B) {
  if (!B) return SCAN_OK;
  batch_release(B);
  delete B;
  return SCAN_OK;
}

int scan_run_batch(const scan_batch* b, const scan_opts* opts, int32_t* labels, uint8_t* roles) {
  scan_batch_graph* B = nullptr;
  int rc = scan_batch_create(b, opts, &B);
  if (rc != SCAN_OK) return rc;
  rc = scan_batch_run(B, 1, labels, roles);
  scan_batch_destroy(B);
  return rc;
}

}  // extern "C"
