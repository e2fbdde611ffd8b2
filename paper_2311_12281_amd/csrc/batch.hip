// Batched clustering of many independent graphs in one go.
//
// The graphs are packed into one disjoint union (global id = vertex offset of
// the graph + local id).  SCAN on a disjoint union is SCAN on each graph, so
// one layout serves the whole batch; each vertex carries its graph id, through
// which every kernel looks up that graph's eps = p/q and mu (read from device
// memory on every run, so scan_batch_set_params changes them without a new
// capture).  Labels (minimum core ids) are turned back into graph-local ids on
// output.
//
// One persistent kernel clusters the whole batch: its blocks take (graph,
// phase, tile) items from a device queue, and every graph moves through the
// phases of Algorithm 1 (with Algorithms 2 and 3) on its own, with a per-graph
// count of the tiles its current phase still has; the block finishing the
// last of them queues the graph's next phase (kernels.hip, k_batch).  The
// queue reset and that kernel are captured once into a HIP graph and
// replayed.  An autotuner chooses the lane-group width of each degree bucket
// and the edges per tile by timing whole runs on the batch itself; choices can
// be cached in a file named by SCAN_AUTOTUNE_CACHE.
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
  int64_t* d_vtx_off = nullptr;
  int64_t* d_eoff = nullptr;
  int64_t* d_init_prefix = nullptr;
  int32_t* d_remaining = nullptr;
  unsigned long long* d_ncores = nullptr;
  unsigned long long* d_ctl = nullptr;
  unsigned long long* d_queue = nullptr;
  int64_t queue_alloc = 0;              // queue slots allocated
  std::vector<int64_t> vtx_off;         // host copies
  std::vector<int64_t> eoff;            // [kNumBuckets * (G + 1)]
  std::vector<int32_t> gdmax;           // maximum degree per graph
  int32_t* d_labels = nullptr;
  uint8_t* d_roles = nullptr;
  int32_t lanes[kNumBuckets] = {4, 8, 16, 32, 64, 64, 64};
  int32_t tile_edges = 4096;
  int grid = 0;
  BatchArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float last_ms = 0.f;
  std::mutex lock;
};

namespace {

constexpr int32_t kTileVertices = 4096;
constexpr int32_t kTileEdgeChoices[] = {1024, 2048, 4096, 8192, 16384};
constexpr int32_t kMinTileEdges = 1024;

void batch_release(scan_batch_graph* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->ev0) (void)hipEventDestroy(B->ev0);
  if (B->ev1) (void)hipEventDestroy(B->ev1);
  void* d[] = {B->d_gid, B->d_gp, B->d_gq, B->d_gmu, B->d_vtx_off, B->d_eoff, B->d_init_prefix,
               B->d_remaining, B->d_ncores, B->d_ctl, B->d_queue, B->d_labels, B->d_roles};
  for (void* p : d)
    if (p) (void)hipFree(p);
  if (B->g) scan_graph_destroy(B->g);
}

// Items of a whole run for the current tile size (no phase skipped), and the
// BP_INIT prefix over the graphs.
int64_t batch_items(const scan_batch_graph* B, int32_t tile_edges, std::vector<int64_t>* init_prefix) {
  const int32_t G = B->G;
  const int split = B->g->opts.hub_outlier ? 1 : 0;
  int64_t total = 0;
  if (init_prefix) init_prefix->assign((size_t)G + 1, 0);
  for (int32_t g = 0; g < G; ++g) {
    int64_t ek[kNumBuckets];
    for (int k = 0; k < kNumBuckets; ++k)
      ek[k] = B->eoff[(size_t)k * (G + 1) + g + 1] - B->eoff[(size_t)k * (G + 1) + g];
    const int64_t n = B->vtx_off[(size_t)g + 1] - B->vtx_off[(size_t)g];
    for (int ph = 0; ph < BP_DONE; ++ph) total += batch_phase_tiles(ph, n, ek, tile_edges, kTileVertices, split);
    if (init_prefix)
      (*init_prefix)[(size_t)g + 1] =
          (*init_prefix)[(size_t)g] + batch_phase_tiles(BP_INIT, n, ek, tile_edges, kTileVertices, split);
  }
  return total;
}

// Fills B->args for the current lanes and tile size (uploads the BP_INIT prefix).
int batch_prepare(scan_batch_graph* B) {
  scan_graph* g = B->g;
  std::vector<int64_t> init_prefix;
  const int64_t total = batch_items(B, B->tile_edges, &init_prefix);
  const int64_t init_items = init_prefix.back();
  if (total - init_items > B->queue_alloc) return fail(SCAN_E_INVAL, "batch queue smaller than the run's items");
  HIP_TRY(hipMemcpy(B->d_init_prefix, init_prefix.data(), sizeof(int64_t) * init_prefix.size(),
                    hipMemcpyHostToDevice), "copy tile prefix");
  BatchArgs& P = B->args;
  P = BatchArgs{};
  EdgeArgs& A = P.A;
  A.rp = g->d_rp;
  A.ci = g->d_ci;
  A.hci = g->d_ci;
  A.edges = g->d_edges;
  A.state = g->d_state;
  A.lower = g->d_lower;
  A.upper = g->d_upper;
  A.role = g->d_role;
  A.parent = g->d_parent;
  A.label = g->d_label;
  A.stats = g->d_stats;
  A.pruning = g->opts.pruning;
  A.gid = B->d_gid;
  A.gp = B->d_gp;
  A.gq = B->d_gq;
  A.gmu = B->d_gmu;
  P.G = B->G;
  P.vtx_off = B->d_vtx_off;
  P.eoff = B->d_eoff;
  P.lanes_code = 0;
  for (int k = 0; k < kNumBuckets; ++k) {
    uint32_t c = 0;
    while ((4 << c) < B->lanes[k]) ++c;
    P.lanes_code |= c << (3 * k);
  }
  P.tile_edges = B->tile_edges;
  P.tile_vertices = kTileVertices;
  P.split = g->opts.hub_outlier ? 1 : 0;
  P.out_labels = B->d_labels;
  P.out_roles = B->d_roles;
  P.queue = B->d_queue;
  P.init_prefix = B->d_init_prefix;
  P.remaining = B->d_remaining;
  P.ncores = B->d_ncores;
  P.ctl = B->d_ctl;
  P.total = total;
  P.init_items = init_items;
  P.queue_cap = total - init_items;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device) != hipSuccess || khz <= 0)
    khz = 100000;
  P.watchdog_ticks = (uint64_t)khz * 1000ull * 20ull;  // 20 s without an item to take
  // SCAN_BATCH_WATCHDOG_US shortens the wait (tests of the abandoned-run report)
  if (const char* w = getenv("SCAN_BATCH_WATCHDOG_US")) P.watchdog_ticks = (uint64_t)khz * strtoull(w, nullptr, 10) / 1000ull;
  return SCAN_OK;
}

// Runs the batch once on the graph's stream (eagerly); device time in ms.
int batch_run_eager(scan_batch_graph* B, float* ms) {
  hipStream_t s = B->g->stream;
  HIP_TRY(hipEventRecord(B->ev0, s), "hipEventRecord");
  launch_batch(s, B->args, B->grid);
  HIP_TRY(hipEventRecord(B->ev1, s), "hipEventRecord");
  HIP_TRY(hipGetLastError(), "batch launch");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (ms) HIP_TRY(hipEventElapsedTime(ms, B->ev0, B->ev1), "hipEventElapsedTime");
  return SCAN_OK;
}

// Reads the run's statistics and the queue's error flag.
int batch_collect(scan_batch_graph* B) {
  scan_graph* g = B->g;
  unsigned long long ctl[4];
  HIP_TRY(hipMemcpy(ctl, B->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost), "copy queue counters");
  if (ctl[2]) return fail(SCAN_E_DEVICE, "batched run abandoned: a block waited too long for its work item");
  const int rc = collect_stats(g, g->stream, false);
  g->last.ms_total = B->last_ms;
  return rc;
}

std::string tune_key(const scan_batch_graph* B) {
  const scan_graph* g = B->g;
  std::string k = "persistent:" + std::to_string(B->G) + ":" + std::to_string(g->n) + ":" + std::to_string(g->m);
  for (int b = 0; b < kNumBuckets; ++b) k += ":" + std::to_string(g->bucket_off[b + 1] - g->bucket_off[b]);
  return k;
}

bool tune_cache_read(const std::string& key, scan_batch_graph* B) {
  const char* path = getenv("SCAN_AUTOTUNE_CACHE");
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char kbuf[512];
  int l[kNumBuckets], te;
  bool found = false;
  while (fscanf(f, "%511s %d %d %d %d %d %d %d %d", kbuf, &l[0], &l[1], &l[2], &l[3], &l[4], &l[5], &l[6], &te) ==
         9) {
    if (key == kbuf) {
      bool ok = te >= kMinTileEdges && te % 64 == 0;
      for (int b = 0; b < kNumBuckets; ++b) ok = ok && (l[b] == 4 || l[b] == 8 || l[b] == 16 || l[b] == 32 || l[b] == 64);
      if (!ok) continue;
      for (int b = 0; b < kNumBuckets; ++b) B->lanes[b] = l[b];
      B->tile_edges = te;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void tune_cache_write(const std::string& key, const scan_batch_graph* B) {
  const char* path = getenv("SCAN_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s", key.c_str());
  for (int b = 0; b < kNumBuckets; ++b) fprintf(f, " %d", B->lanes[b]);
  fprintf(f, " %d\n", B->tile_edges);
  fclose(f);
}

// Median device time of 3 runs of the whole batch under the current choice.
int time_config(scan_batch_graph* B, double* ms) {
  int rc = batch_prepare(B);
  if (rc != SCAN_OK) return rc;
  float t[4];
  for (int r = 0; r < 4; ++r) {
    rc = batch_run_eager(B, &t[r]);
    if (rc != SCAN_OK) return rc;
    rc = batch_collect(B);
    if (rc != SCAN_OK) return rc;
  }
  std::sort(t + 1, t + 4);
  *ms = t[2];
  return SCAN_OK;
}

// Coordinate descent: for each degree bucket with edges, lane widths around
// the current one (half, same, double); then the edges per tile.
int autotune(scan_batch_graph* B) {
  scan_graph* g = B->g;
  const std::string key = tune_key(B);
  if (tune_cache_read(key, B)) return SCAN_OK;
  double best = 0;
  int rc = time_config(B, &best);
  if (rc != SCAN_OK) return rc;
  for (int k = 0; k < kNumBuckets; ++k) {
    if (g->bucket_off[k + 1] == g->bucket_off[k]) continue;
    const int d = B->lanes[k];
    for (int c : {d / 2, d * 2}) {
      if (c < 4 || c > 64) continue;
      B->lanes[k] = c;
      double ms = 0;
      rc = time_config(B, &ms);
      if (rc != SCAN_OK) return rc;
      if (ms < best) best = ms;
      else B->lanes[k] = d;
    }
  }
  const int32_t t0 = B->tile_edges;
  for (int32_t te : kTileEdgeChoices) {
    if (te == t0) continue;
    const int32_t keep = B->tile_edges;
    B->tile_edges = te;
    double ms = 0;
    rc = time_config(B, &ms);
    if (rc != SCAN_OK) return rc;
    if (ms < best) best = ms;
    else B->tile_edges = keep;
  }
  tune_cache_write(key, B);
  return SCAN_OK;
}

int capture(scan_batch_graph* B) {
  int rc = batch_prepare(B);
  if (rc != SCAN_OK) return rc;
  if (B->exec) {
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  if (B->graph) {
    (void)hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  hipStream_t s = B->g->stream;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  launch_batch(s, B->args, B->grid);
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
  B->graph = graph;
  HIP_TRY(hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  return SCAN_OK;
}

// Per-graph eps (reduced) and mu, checked against each graph's degree range.
int upload_params(scan_batch_graph* B, const int64_t* eps_num, const int64_t* eps_den, const int32_t* mu) {
  const int32_t G = B->G;
  const size_t GG = (size_t)(G > 0 ? G : 1);
  std::vector<uint64_t> gp(GG), gq(GG);
  std::vector<int32_t> gmu(GG, 2);
  for (int32_t k = 0; k < G; ++k) {
    if (eps_num[k] < 1 || eps_den[k] < eps_num[k])
      return fail(SCAN_E_INVAL, "graph %d: eps must satisfy 1 <= eps_num <= eps_den", k);
    if (mu[k] < 2) return fail(SCAN_E_INVAL, "graph %d: mu must be >= 2", k);
    int64_t p = eps_num[k], q = eps_den[k], x = p, y = q;
    while (y) { int64_t t = x % y; x = y; y = t; }
    p /= x;
    q /= x;
    if ((unsigned __int128)q * (unsigned __int128)((uint64_t)B->gdmax[(size_t)k] + 1) >= ((unsigned __int128)1 << 32))
      return fail(SCAN_E_RANGE, "graph %d: eps denominator too large for its maximum degree", k);
    gp[(size_t)k] = (uint64_t)p;
    gq[(size_t)k] = (uint64_t)q;
    gmu[(size_t)k] = mu[k];
  }
  HIP_TRY(hipMemcpy(B->d_gp, gp.data(), 8 * GG, hipMemcpyHostToDevice), "copy eps");
  HIP_TRY(hipMemcpy(B->d_gq, gq.data(), 8 * GG, hipMemcpyHostToDevice), "copy eps");
  HIP_TRY(hipMemcpy(B->d_gmu, gmu.data(), 4 * GG, hipMemcpyHostToDevice), "copy mu");
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
  auto* B = new (std::nothrow) scan_batch_graph();
  if (!B) return fail(SCAN_E_NOMEM, "host allocation failed");
  B->G = G;
  B->N = N;
  B->vtx_off.assign(b->vtx_off, b->vtx_off + G + 1);
  B->gdmax.assign((size_t)(G > 0 ? G : 1), 0);
  int rc = SCAN_OK;
  {
    // disjoint union, host side
    std::vector<int64_t> rp((size_t)N + 1);
    std::vector<int32_t> ci((size_t)(nnz > 0 ? nnz : 1));
    std::vector<int32_t> gid((size_t)(N > 0 ? N : 1));
    std::vector<int> bad((size_t)(G > 0 ? G : 1), 0);
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
            B->gdmax[(size_t)k] = (int32_t)std::max<int64_t>(B->gdmax[(size_t)k], lrp[v + 1] - lrp[v]);
          }
          for (int64_t a = a0; a < b->arc_off[k + 1]; ++a) {
            const int32_t x = b->col_idx[a];
            if (x < 0 || x >= nk) bad[(size_t)k] = 1;
            ci[(size_t)a] = (int32_t)(v0 + x);
          }
        }
      });
    for (auto& x : th) x.join();
    rp[(size_t)N] = nnz;
    for (int32_t k = 0; k < G; ++k)
      if (bad[(size_t)k]) {
        delete B;
        return fail(SCAN_E_GRAPH, "graph %d: row offsets or neighbour ids out of range", k);
      }
    scan_opts o;
    if (opts) o = *opts;
    else scan_opts_default(&o);
    o.device_budget_bytes = 0;
    o.hub_ranked = 0;  // the batch kernel reads the rows as given
    rc = scan_graph_create(N, nnz, rp.data(), ci.data(), &o, &B->g);
    if (rc != SCAN_OK) {
      delete B;
      return rc;
    }
    const size_t NN = (size_t)(N > 0 ? N : 1);
    hipError_t e = hipMalloc((void**)&B->d_gid, 4 * NN);
    if (e == hipSuccess) e = hipMemcpy(B->d_gid, gid.data(), 4 * NN, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      rc = fail_hip(e, "graph ids");
      batch_release(B);
      delete B;
      return rc;
    }
  }
  scan_graph* g = B->g;
  const size_t GG = (size_t)(G > 0 ? G : 1), G1 = (size_t)G + 1;
  hipError_t e;
  int64_t queue_need = 0;
#define BTRY(x, what) do { e = (x); if (e != hipSuccess) { rc = fail_hip(e, what); goto error; } } while (0)
  BTRY(hipMalloc((void**)&B->d_gp, 8 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_gq, 8 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_gmu, 4 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_vtx_off, 8 * G1), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_eoff, 8 * G1 * kNumBuckets), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_init_prefix, 8 * G1), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_remaining, 4 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_ncores, 8 * GG), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_ctl, 8 * 4), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_labels, 4 * (size_t)(N > 0 ? N : 1)), "hipMalloc");
  BTRY(hipMalloc((void**)&B->d_roles, (size_t)(N > 0 ? N : 1)), "hipMalloc");
  BTRY(hipEventCreate(&B->ev0), "hipEventCreate");
  BTRY(hipEventCreate(&B->ev1), "hipEventCreate");
  BTRY(hipMemcpy(B->d_vtx_off, b->vtx_off, 8 * G1, hipMemcpyHostToDevice), "copy");
  rc = upload_params(B, b->eps_num, b->eps_den, b->mu);
  if (rc != SCAN_OK) goto error;
  // each graph's edge range in every bucket
  launch_batch_edge_offsets(g->stream, G, B->d_vtx_off, g->d_edges, g->bucket_off, B->d_eoff);
  BTRY(hipGetLastError(), "edge offsets");
  BTRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
  B->eoff.resize(G1 * kNumBuckets);
  BTRY(hipMemcpy(B->eoff.data(), B->d_eoff, 8 * G1 * kNumBuckets, hipMemcpyDeviceToHost), "copy");
  {
    // tile indices are 28-bit fields of a work item
    std::vector<int64_t> ip;
    const int64_t total = batch_items(B, kMinTileEdges, &ip);
    queue_need = total - ip.back();
    for (int32_t k = 0; k < G; ++k) {
      int64_t ek[kNumBuckets];
      for (int b2 = 0; b2 < kNumBuckets; ++b2) ek[b2] = B->eoff[(size_t)b2 * G1 + k + 1] - B->eoff[(size_t)b2 * G1 + k];
      const int64_t nk = B->vtx_off[(size_t)k + 1] - B->vtx_off[(size_t)k];
      for (int ph = 0; ph < BP_DONE; ++ph)
        if (batch_phase_tiles(ph, nk, ek, kMinTileEdges, kTileVertices, 1) >= (1 << 28)) {
          rc = fail(SCAN_E_INVAL, "graph %d is too large for one batch", k);
          goto error;
        }
    }
  }
  B->queue_alloc = queue_need;
  BTRY(hipMalloc((void**)&B->d_queue, 8 * (size_t)(queue_need > 0 ? queue_need : 1)), "hipMalloc queue");
  B->grid = batch_grid_blocks();
  if (b->autotune) {
    rc = autotune(B);
    if (rc != SCAN_OK) goto error;
  }
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

int scan_batch_set_params(scan_batch_graph* B, const int64_t* eps_num, const int64_t* eps_den, const int32_t* mu) {
  if (!B) return fail(SCAN_E_INVAL, "batch is NULL");
  if (B->G > 0 && (!eps_num || !eps_den || !mu)) return fail(SCAN_E_INVAL, "NULL parameter array");
  std::lock_guard<std::mutex> lk(B->lock);
  return upload_params(B, eps_num, eps_den, mu);
}

int scan_batch_run(scan_batch_graph* B, int32_t replay, int32_t* labels, uint8_t* roles) {
  if (!B) return fail(SCAN_E_INVAL, "batch is NULL");
  if (B->N > 0 && (!labels || !roles)) return fail(SCAN_E_INVAL, "output pointer is NULL");
  std::lock_guard<std::mutex> lk(B->lock);
  scan_graph* g = B->g;
  hipStream_t s = g->stream;
  if (replay) {
    HIP_TRY(hipEventRecord(B->ev0, s), "hipEventRecord");
    HIP_TRY(hipGraphLaunch(B->exec, s), "hipGraphLaunch");
    HIP_TRY(hipEventRecord(B->ev1, s), "hipEventRecord");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    HIP_TRY(hipEventElapsedTime(&B->last_ms, B->ev0, B->ev1), "hipEventElapsedTime");
  } else {
    int rc = batch_run_eager(B, &B->last_ms);
    if (rc != SCAN_OK) return rc;
  }
  int rc = batch_collect(B);
  if (rc != SCAN_OK) return rc;
  if (B->N > 0) {
    HIP_TRY(hipMemcpyAsync(labels, B->d_labels, 4 * (size_t)B->N, hipMemcpyDeviceToHost, s), "copy labels");
    HIP_TRY(hipMemcpyAsync(roles, B->d_roles, (size_t)B->N, hipMemcpyDeviceToHost, s), "copy roles");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  }
  return SCAN_OK;
}

int scan_batch_config(const scan_batch_graph* B, int32_t* lanes, int32_t* tile_edges) {
  if (!B) return fail(SCAN_E_INVAL, "batch is NULL");
  if (lanes)
    for (int k = 0; k < kNumBuckets; ++k) lanes[k] = B->lanes[k];
  if (tile_edges) *tile_edges = B->tile_edges;
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
