// Partition-based path for graphs larger than the device budget (GPUSCAN++
// Section 5: edge-extended subgraphs, Def. 5.1; exactness of sigma on them,
// Lemma 5.1; the three streamed passes of Alg. 5).
//
// Redesign for one MI355X: instead of packing edges greedily into subgraphs
// (Alg. 5, host loop), vertices are cut into contiguous ranges ("units") whose
// rows fit a quarter of the device row buffer, and consecutive pairs of units
// form "blocks".  The edges between a block and a unit of a later block (or
// inside a block) are processed with the complete rows of both on the device,
// so every intersection sees both full neighbourhoods - the edge-extended
// subgraph of those edges - and sigma is exact (Lemma 5.1).  The block sits
// in the first half of the row buffer, units in two slots of the second half:
// the next unit's rows are uploaded on a stream of their own while the current
// one is read.  Per-vertex state (bounds,
// roles, parents, labels) and row_ptr stay resident for the whole run; edge
// states travel with their edges (uploaded before, read back after each chunk,
// like the store step of Alg. 5).  One run streams the pairs three times: the
// cores pass, the merge pass (known-similar hooks, then progressive merging,
// chunk by chunk) and the attach pass; union-find roots and labels are global,
// so unions made in one chunk are seen by all later ones (no per-subgraph
// re-initialisation of the forest).
#include "graph.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

namespace scan {

uint64_t inmemory_footprint(int32_t n, int64_t nnz, bool ranked) {
  const uint64_t m = (uint64_t)nnz / 2;
  // row_ptr, col_idx (and its ranked copy) with a sample per 32 ids, oriented
  // edges and their degree pairs, hub worklist, edge state, per-vertex state +
  // outputs
  const uint64_t cols = (ranked && n > kHubBitmapBits) ? 8ull : 4ull;
  return 8ull * ((uint64_t)n + 1) + cols * nnz + 4ull * (uint64_t)sample_lines(nnz) + 16ull * m + 4ull * m +
         1ull * m + 22ull * n + (1ull << 20);
}

namespace {

// device bytes per chunk edge: two buffers of (endpoints, state), one count,
// one worklist slot
constexpr uint64_t kEdgeBytes = 2 * (8 + 1) + 4 + 4;

// the in-memory layout's buckets: by the smaller degree, and the LDS-hash
// bucket for edges whose larger side has more than kHubMinDegree neighbours
int part_bucket(int64_t ds, int64_t dl) {
  const int b = bucket_of(ds);
  return (b == kNumBuckets - 2 && dl > kHubMinDegree) ? kNumBuckets - 1 : b;
}

}  // namespace

void part_release(scan_graph* g) {
  PartPlan& P = g->part;
  if (P.h_ci) (void)hipHostFree(P.h_ci);
  if (P.h_edges) (void)hipHostFree(P.h_edges);
  if (P.h_state) (void)hipHostFree(P.h_state);
  if (P.h_ecount) (void)hipHostFree(P.h_ecount);
  void* d[] = {P.d_rows, P.d_edges, P.d_state, P.d_edges2, P.d_state2, P.d_ecount, P.d_jobs, P.d_wtab,
               P.d_worklist, P.d_jobctr};
  for (void* p : d)
    if (p) (void)hipFree(p);
  for (int b = 0; b < 2; ++b) {
    if (P.up[b]) (void)hipEventDestroy(P.up[b]);
    if (P.done[b]) (void)hipEventDestroy(P.done[b]);
    if (P.rready[b]) (void)hipEventDestroy(P.rready[b]);
    if (P.rfree[b]) (void)hipEventDestroy(P.rfree[b]);
  }
  if (P.copy) (void)hipStreamDestroy(P.copy);
  if (P.rowcopy) (void)hipStreamDestroy(P.rowcopy);
  P = PartPlan();
}

// Host-side CSR checks (the graph never resides on the device whole):
// same conditions as the device validation of the in-memory path.
int part_validate(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci, bool full) {
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v] || rp[v] < 0 || rp[v + 1] > nnz) return fail(SCAN_E_GRAPH, "row offsets not monotone");
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<int> bad((size_t)nth, 0);
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      for (int32_t u = t; u < n && !bad[(size_t)t]; u += nth)
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
          const int32_t v = ci[k];
          if (v < 0 || v >= n) { bad[(size_t)t] = 2; break; }
          if (!full) continue;
          if (v == u) { bad[(size_t)t] = 4; break; }
          if (k > rp[u] && ci[k - 1] >= v) { bad[(size_t)t] = 8; break; }
          if (!std::binary_search(ci + rp[v], ci + rp[v + 1], u)) { bad[(size_t)t] = 16; break; }
        }
    });
  for (auto& x : th) x.join();
  for (int b : bad)
    if (b) return fail(SCAN_E_GRAPH, "CSR rejected (flag 0x%x: 2 id range, 4 self-loop, 8 row order/duplicate, "
                                     "16 missing reverse arc)", b);
  return SCAN_OK;
}

int part_create(scan_graph* g, const int64_t* rp, const int32_t* ci, uint64_t budget) {
  PartPlan& P = g->part;
  const int32_t n = g->n;
  const int64_t nnz = g->nnz;
  const int64_t m = nnz / 2;
  const uint64_t resident = 8ull * ((uint64_t)n + 1) + 22ull * (uint64_t)n + (1ull << 20);
  if (budget <= resident + (1ull << 16))
    return fail(SCAN_E_NOMEM, "budget %llu bytes cannot hold the per-vertex state (%llu bytes)",
                (unsigned long long)budget, (unsigned long long)resident);
  const uint64_t rest = budget - resident;
  int64_t chunk_cap = (int64_t)((rest / 4) / kEdgeBytes);
  if (chunk_cap > m) chunk_cap = m;
  if (chunk_cap < 1) chunk_cap = 1;
  // The row buffer holds a block (its first half) and units of later blocks
  // (the second half).  A block is two units of at most a quarter of the
  // buffer, so the second half has two unit slots and the next unit's rows
  // are uploaded while the current one is read; when the longest row does not
  // fit a quarter, a block is one unit and the second half a single slot.
  const int64_t row_cap = (int64_t)((rest - (uint64_t)chunk_cap * kEdgeBytes) / 4);
  int64_t maxdeg = 0;
  for (int32_t v = 0; v < n; ++v) maxdeg = std::max(maxdeg, rp[v + 1] - rp[v]);
  const bool two = row_cap / 4 >= 1 && maxdeg <= row_cap / 4;
  P.upb = two ? 2 : 1;
  P.nslots = two ? 2 : 1;
  P.jcap = row_cap / 2 / P.nslots;
  const int64_t ucap = P.jcap;
  if (maxdeg > ucap || ucap < 1)
    return fail(SCAN_E_NOMEM, "budget too small: a row of %lld neighbours does not fit a block of %lld",
                (long long)maxdeg, (long long)(row_cap / 2));
  // units: contiguous vertex ranges with at most ucap arcs; blocks: runs of upb units
  P.unit_lo.clear();
  P.unit_lo.push_back(0);
  for (int32_t v = 0; v < n; ++v) {
    const int64_t start = rp[P.unit_lo.back()];
    if (rp[v + 1] - start > ucap) P.unit_lo.push_back(v);
  }
  P.unit_lo.push_back(n);
  const int32_t U = (int32_t)P.unit_lo.size() - 1;
  const int32_t K = (U + P.upb - 1) / P.upb;
  P.block_lo.clear();
  for (int32_t b = 0; b < K; ++b) P.block_lo.push_back(P.unit_lo[(size_t)b * P.upb]);
  P.block_lo.push_back(n);
  P.h_rp.assign(rp, rp + n + 1);
  auto block_of = [&](int32_t x) {
    return (int32_t)(std::upper_bound(P.block_lo.begin(), P.block_lo.end(), x) - P.block_lo.begin()) - 1;
  };
  auto unit_of = [&](int32_t x) {
    return (int32_t)(std::upper_bound(P.unit_lo.begin(), P.unit_lo.end(), x) - P.unit_lo.begin()) - 1;
  };
  // pairs of block i: its own edges, then one per unit of a later block
  const int32_t upb = P.upb;
  std::vector<int64_t> pair_base((size_t)K + 1, 0);
  for (int32_t i = 0; i < K; ++i) pair_base[(size_t)i + 1] = pair_base[(size_t)i] + 1 + std::max(0, U - upb * (i + 1));
  auto pair_local = [&](int32_t i, int32_t j) { return j < 0 ? 0 : 1 + (j - upb * (i + 1)); };
  auto pair_index = [&](int32_t i, int32_t j) { return pair_base[(size_t)i] + pair_local(i, j); };
  const int64_t npairs = pair_base[(size_t)K];
  const int NB = kNumBuckets;
  std::vector<int64_t> cnt((size_t)(npairs * NB), 0);
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // an edge {u, v} is listed from the row of its endpoint in the lower block
  // (the smaller id inside one block), in the pair of that block with the
  // other endpoint's unit (or the block's own pair); it is stored as
  // (smaller, larger) by (degree, id) and bucketed by the smaller degree
  auto for_edges_of_block = [&](int32_t i, auto&& fn) {
    for (int32_t u = P.block_lo[i]; u < P.block_lo[i + 1]; ++u) {
      for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
        const int32_t v = ci[k];
        const int32_t bv = block_of(v);
        if (bv < i || (bv == i && v < u)) continue;
        const int32_t j = bv == i ? -1 : unit_of(v);
        const int64_t du = rp[u + 1] - rp[u], dv = rp[v + 1] - rp[v];
        const bool u_small = du < dv || (du == dv && u < v);
        fn(j, u_small ? u : v, u_small ? v : u, u_small ? part_bucket(du, dv) : part_bucket(dv, du));
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        for (int32_t i = t; i < K; i += nth)
          for_edges_of_block(i, [&](int32_t j, int32_t, int32_t, int b) { cnt[(size_t)(pair_index(i, j) * NB + b)]++; });
      });
    for (auto& x : th) x.join();
  }
  std::vector<int64_t> off((size_t)(npairs * NB + 1), 0);
  for (int64_t k = 0; k < npairs * NB; ++k) off[(size_t)k + 1] = off[(size_t)k] + cnt[(size_t)k];
  if (off.back() != m) return fail(SCAN_E_GRAPH, "edge count %lld does not match nnz/2", (long long)off.back());
  hipError_t e;
  if ((e = hipHostMalloc((void**)&P.h_edges, sizeof(int2) * (size_t)std::max<int64_t>(m, 1), hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&P.h_state, (size_t)std::max<int64_t>(m, 1), hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&P.h_ecount, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1), hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void**)&P.h_ci, sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1), hipHostMallocDefault)) != hipSuccess)
    return fail_hip(e, "pinned host memory");
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        std::vector<int64_t> cur((size_t)NB);
        for (int32_t i = t; i < K; i += nth) {
          // cursors of the pairs of block i: written only by this thread
          const int64_t np = pair_base[(size_t)i + 1] - pair_base[(size_t)i];
          std::vector<int64_t> pc((size_t)(np * NB));
          for (int64_t q = 0; q < np; ++q)
            for (int b = 0; b < NB; ++b) pc[(size_t)(q * NB + b)] = off[(size_t)((pair_base[(size_t)i] + q) * NB + b)];
          for_edges_of_block(i, [&](int32_t j, int32_t su, int32_t lv, int b) {
            P.h_edges[pc[(size_t)(pair_local(i, j) * NB + b)]++] = make_int2(su, lv);
          });
        }
      });
    for (auto& x : th) x.join();
  }
  if (nnz > 0) memcpy(P.h_ci, ci, sizeof(int32_t) * (size_t)nnz);
  {
    // the last bucket of every pair grouped by the larger side, as the LDS-hash jobs need
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        for (int64_t pi = t; pi < npairs; pi += nth) {
          int2* b = P.h_edges + off[(size_t)(pi * NB + NB - 1)];
          int2* e = P.h_edges + off[(size_t)(pi * NB + NB)];
          std::sort(b, e, [](const int2& x, const int2& y) { return x.y != y.y ? x.y < y.y : x.x < y.x; });
        }
      });
    for (auto& x : th) x.join();
  }
  // chunks: runs of one pair of at most chunk_cap edges; a block's own pair
  // first, then its pairs with later units from the last unit down, so that
  // the last units read are the next block's (their rows are copied on the
  // device when that block comes up)
  for (int32_t i = 0; i < K; ++i)
    for (int32_t j = -1; j == -1 || j >= upb * (i + 1); j = (j < 0 ? U - 1 : j - 1)) {
      if (j >= U) continue;
      const int64_t pi = pair_index(i, j);
      const int64_t b0 = off[(size_t)(pi * NB)], b1 = off[(size_t)(pi * NB + NB)];
      for (int64_t c0 = b0; c0 < b1; c0 += chunk_cap) {
        PartChunk C;
        C.bi = i;
        C.bj = j;
        C.begin = c0;
        C.end = std::min(b1, c0 + chunk_cap);
        for (int b = 0; b <= kNumBuckets; ++b) {
          const int64_t x = b < NB ? off[(size_t)(pi * NB + b)] : b1;
          C.bucket_off[b] = std::min(std::max(x, C.begin), C.end);
        }
        P.chunks.push_back(C);
      }
    }
  // LDS-hash jobs of each chunk's last bucket: runs of one larger side, cut like
  // the in-memory job table, heaviest larger side first; edges chunk-relative
  std::vector<HubJob> jobs;
  for (PartChunk& C : P.chunks) {
    C.job_off = (int64_t)jobs.size();
    const int64_t b6 = C.bucket_off[kNumBuckets - 1], e6 = C.bucket_off[kNumBuckets];
    for (int64_t k = b6; k < e6;) {
      const int32_t v = P.h_edges[k].y;
      HubJob J{};
      J.v = v;
      J.begin = k - C.begin;
      J.count = 0;
      int64_t work = 0;
      while (k < e6 && P.h_edges[k].y == v) {
        const int64_t du = rp[P.h_edges[k].x + 1] - rp[P.h_edges[k].x];
        if (J.count > 0 && (J.count == kHubJobEdges || work + du > kHubJobWork)) {
          jobs.push_back(J);
          J.begin = k - C.begin;
          J.count = 0;
          work = 0;
        }
        ++J.count;
        work += du;
        ++k;
      }
      jobs.push_back(J);
    }
    C.job_cnt = (int64_t)jobs.size() - C.job_off;
    std::stable_sort(jobs.begin() + C.job_off, jobs.end(), [&](const HubJob& a, const HubJob& b) {
      return rp[a.v + 1] - rp[a.v] > rp[b.v + 1] - rp[b.v];
    });
  }
  // windows of the hub rows (the raw rows: the kernel reads them as given here)
  std::vector<uint32_t> wtab;
  assign_hub_windows(jobs, rp, ci, wtab);
  P.row_cap = row_cap;
  P.chunk_cap = chunk_cap;
  // rows are read up to kColPad elements past their end by the LDS-hash kernel
  if ((e = hipMalloc((void**)&P.d_rows, sizeof(int32_t) * (size_t)(std::max<int64_t>(row_cap, 1) + kColPad))) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_jobs, sizeof(HubJob) * std::max<size_t>(jobs.size(), 1))) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_wtab, sizeof(uint32_t) * std::max<size_t>(wtab.size(), 1))) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_worklist, sizeof(int32_t) * (size_t)chunk_cap)) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_jobctr, sizeof(unsigned long long))) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_edges, sizeof(int2) * (size_t)chunk_cap)) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_state, (size_t)chunk_cap)) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_edges2, sizeof(int2) * (size_t)chunk_cap)) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_state2, (size_t)chunk_cap)) != hipSuccess ||
      (e = hipMalloc((void**)&P.d_ecount, sizeof(int32_t) * (size_t)chunk_cap)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&P.copy, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.up[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.up[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.done[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.done[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&P.rowcopy, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.rready[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.rready[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.rfree[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&P.rfree[1], hipEventDisableTiming)) != hipSuccess)
    return fail_hip(e, "device buffers");
  if (!jobs.empty() &&
      ((e = hipMemcpy(P.d_jobs, jobs.data(), sizeof(HubJob) * jobs.size(), hipMemcpyHostToDevice)) != hipSuccess ||
       (e = hipMemcpy(P.d_wtab, wtab.data(), sizeof(uint32_t) * wtab.size(), hipMemcpyHostToDevice)) != hipSuccess))
    return fail_hip(e, "job table");
  g->partitioned = true;
  g->m = m;
  return SCAN_OK;
}

namespace {

struct Streamer {
  scan_graph* g;
  hipStream_t s;  // compute stream
  int32_t li = -1;   // block whose rows are in the buffer's first half
  int32_t slot_unit[2] = {-1, -1};  // unit whose rows a slot holds (or is receiving)
  int32_t last_slot = -1;  // slot read by the previous run of chunks
  int32_t next_slot = 0;   // slot the next upload goes to

  int64_t slot_off(int k) const { return g->part.jcap * (g->part.nslots == 2 ? 2 : 1) + (int64_t)k * g->part.jcap; }

  // Unit j's rows into a slot, on the row stream once the slot's last reader
  // is done; returns the slot.  A unit already held is not sent again.
  int load_unit(int32_t j, int avoid, hipError_t& e) {
    PartPlan& P = g->part;
    for (int k = 0; k < P.nslots; ++k)
      if (slot_unit[k] == j) return k;
    int k = next_slot;
    if (k == avoid && P.nslots == 2) k ^= 1;
    next_slot = (k + 1) % P.nslots;
    const int32_t lo = P.unit_lo[(size_t)j], hi = P.unit_lo[(size_t)j + 1];
    const int64_t len = P.h_rp[(size_t)hi] - P.h_rp[(size_t)lo];
    if (e == hipSuccess) e = hipStreamWaitEvent(P.rowcopy, P.rfree[k], 0);
    if (e == hipSuccess && len > 0)
      e = hipMemcpyAsync(P.d_rows + slot_off(k), P.h_ci + P.h_rp[(size_t)lo], sizeof(int32_t) * (size_t)len,
                         hipMemcpyHostToDevice, P.rowcopy);
    if (e == hipSuccess) e = hipEventRecord(P.rready[k], P.rowcopy);
    P.h2d_bytes += 4ull * (uint64_t)len;
    slot_unit[k] = j;
    return k;
  }

  // Called for the first chunk of every run of chunks with the same pair
  // (i, j), before any of its work is enqueued: makes block i's rows and unit
  // j's rows resident, sets the row mapping, and starts uploading the unit of
  // the next run (next_j, -1 if none) into the other slot.
  hipError_t enter(int32_t i, int32_t j, int32_t next_j, EdgeArgs& A) {
    PartPlan& P = g->part;
    hipError_t e = hipSuccess;
    if (last_slot >= 0) e = hipEventRecord(P.rfree[last_slot], s);  // the previous run's reads come first
    last_slot = -1;
    const int32_t lo_i = P.block_lo[(size_t)i], hi_i = P.block_lo[(size_t)i + 1];
    if (e == hipSuccess && i != li) {
      // block rows on the compute stream (every earlier chunk has read the old
      // ones), unit by unit: a unit a slot holds is copied on the device
      const int32_t u_end = std::min<int32_t>((i + 1) * P.upb, (int32_t)P.unit_lo.size() - 1);
      for (int32_t u = i * P.upb; u < u_end && e == hipSuccess; ++u) {
        const int64_t b = P.h_rp[(size_t)P.unit_lo[(size_t)u]], len = P.h_rp[(size_t)P.unit_lo[(size_t)u + 1]] - b;
        const int64_t at = b - P.h_rp[(size_t)lo_i];
        if (len <= 0) continue;
        int k = -1;
        for (int q = 0; q < P.nslots; ++q)
          if (slot_unit[q] == u) k = q;
        if (k >= 0) {
          // the slot's upload has been waited for already (every unit a slot
          // receives is the unit of a later run of the same block, entered
          // before this block comes up); the wait is repeated here so that the
          // copy does not depend on that order
          e = hipStreamWaitEvent(s, P.rready[k], 0);
          if (e == hipSuccess)
            e = hipMemcpyAsync(P.d_rows + at, P.d_rows + slot_off(k), sizeof(int32_t) * (size_t)len,
                               hipMemcpyDeviceToDevice, s);
        } else {
          e = hipMemcpyAsync(P.d_rows + at, P.h_ci + b, sizeof(int32_t) * (size_t)len, hipMemcpyHostToDevice, s);
          P.h2d_bytes += 4ull * (uint64_t)len;
        }
      }
      // the slots' next uploads wait for these copies
      for (int q = 0; q < P.nslots && e == hipSuccess; ++q) e = hipEventRecord(P.rfree[q], s);
      li = i;
    }
    A.ci = P.d_rows;
    A.hci = P.d_rows;
    A.a_lo = lo_i;
    A.a_hi = hi_i;
    A.delta_a = P.h_rp[(size_t)lo_i];
    A.delta_b = A.delta_a;
    if (j >= 0) {
      const int k = load_unit(j, -1, e);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, P.rready[k], 0);
      A.delta_b = P.h_rp[(size_t)P.unit_lo[(size_t)j]] - slot_off(k);
      last_slot = k;
    }
    if (next_j >= 0 && next_j != j && P.nslots == 2) (void)load_unit(next_j, last_slot, e);
    return e;
  }

  // After the last chunk: the slots' last readers are the chunks enqueued so far.
  hipError_t finish() {
    hipError_t e = hipSuccess;
    if (last_slot >= 0) e = hipEventRecord(g->part.rfree[last_slot], s);
    last_slot = -1;
    return e;
  }
};

// The unit of the first run after chunk list[idx]'s run that reads one, in
// the same block (-1: none; the slots may hold the next block's units, which
// are copied from them when it comes up).
int32_t next_unit(const PartPlan& P, const std::vector<int32_t>& list, size_t idx) {
  const PartChunk& C = P.chunks[(size_t)list[idx]];
  for (size_t k = idx + 1; k < list.size(); ++k) {
    const PartChunk& D = P.chunks[(size_t)list[k]];
    if (D.bi != C.bi) return -1;
    if (D.bj >= 0 && D.bj != C.bj) return D.bj;
  }
  return -1;
}

}  // namespace

namespace {

// The kernels of one resident chunk: group kernels for buckets 0-5, the
// LDS-hash kernel with the chunk's own jobs for the last bucket.
void launch_chunk(hipStream_t s, int mode, const PartChunk& C, EdgeArgs& A, PartPlan& P) {
  for (int k = 0; k < kNumBuckets; ++k) {
    A.e_begin = C.bucket_off[k] - C.begin;
    A.e_end = C.bucket_off[k + 1] - C.begin;
    A.bucket = k;
    if (k < kNumBuckets - 1) {
      launch_edges(s, mode, k, A);
    } else if (C.job_cnt > 0) {
      launch_zero_u64(s, P.d_jobctr, 1);
      launch_hub(s, mode, A, P.d_jobs + C.job_off, C.job_cnt, P.d_jobctr, P.d_worklist);
    }
  }
}

// Chunks the merge pass (some edge with two core endpoints) and the attach pass
// (some edge with exactly one core endpoint whose state is not dissimilar) must
// stream; host threads over the chunks.
void select_chunks(const PartPlan& P, const uint8_t* role, std::vector<int32_t>& merge_list,
                   std::vector<int32_t>& attach_list) {
  const size_t nc = P.chunks.size();
  std::vector<uint8_t> need_m(nc, 0), need_a(nc, 0);
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // units and blocks holding a core: a chunk whose block and unit hold none
  // has nothing to do
  const int32_t U = (int32_t)P.unit_lo.size() - 1;
  const int32_t K = (int32_t)P.block_lo.size() - 1;
  std::vector<uint8_t> unit_core((size_t)(U > 0 ? U : 1), 0), block_core((size_t)(K > 0 ? K : 1), 0);
  {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        for (int32_t b = (int32_t)t; b < U; b += (int32_t)nth)
          for (int32_t v = P.unit_lo[(size_t)b]; v < P.unit_lo[(size_t)b + 1]; ++v)
            if (role[v] == ROLE_CORE) {
              unit_core[(size_t)b] = 1;
              break;
            }
      });
    for (auto& x : th) x.join();
    for (int32_t b = 0; b < U; ++b)
      if (unit_core[(size_t)b]) block_core[(size_t)(b / P.upb)] = 1;
  }
  // slices of kSlice edges, taken by the threads from a shared counter, so
  // that a chunk needing a full scan (no qualifying edge early on) is spread
  // over all of them; a slice stops once both of its chunk's flags are set
  constexpr int64_t kSlice = 1 << 20;
  std::vector<int64_t> first_slice(nc + 1, 0);
  for (size_t c = 0; c < nc; ++c) {
    const PartChunk& C = P.chunks[c];
    const bool live = block_core[(size_t)C.bi] || (C.bj >= 0 && unit_core[(size_t)C.bj]);
    first_slice[c + 1] = first_slice[c] + (live ? (C.end - C.begin + kSlice - 1) / kSlice : 0);
  }
  std::vector<std::atomic<uint8_t>> fm(nc), fa(nc);
  for (size_t c = 0; c < nc; ++c) {
    fm[c].store(0, std::memory_order_relaxed);
    fa[c].store(0, std::memory_order_relaxed);
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nth; ++t)
    th.emplace_back([&]() {
      for (int64_t k = next.fetch_add(1); k < first_slice[nc]; k = next.fetch_add(1)) {
        const size_t c = (size_t)(std::upper_bound(first_slice.begin(), first_slice.end(), k) - first_slice.begin()) - 1;
        const PartChunk& C = P.chunks[c];
        const int64_t b = C.begin + (k - first_slice[c]) * kSlice, e_end = std::min(C.end, b + kSlice);
        bool m = fm[c].load(std::memory_order_relaxed) != 0, a = fa[c].load(std::memory_order_relaxed) != 0;
        for (int64_t e = b; e < e_end && !(m && a); ++e) {
          const int2 uv = P.h_edges[e];
          const bool cu = role[uv.x] == ROLE_CORE, cv = role[uv.y] == ROLE_CORE;
          m = m || (cu && cv);
          a = a || (cu != cv && P.h_state[e] != SIM_NO);
          if ((e & 4095) == 4095) {  // another slice of the chunk may have found what is missing
            m = m || fm[c].load(std::memory_order_relaxed) != 0;
            a = a || fa[c].load(std::memory_order_relaxed) != 0;
          }
        }
        if (m) fm[c].store(1, std::memory_order_relaxed);
        if (a) fa[c].store(1, std::memory_order_relaxed);
      }
    });
  for (auto& x : th) x.join();
  for (size_t c = 0; c < nc; ++c) {
    need_m[c] = fm[c].load();
    need_a[c] = fa[c].load();
  }
  merge_list.clear();
  attach_list.clear();
  for (size_t c = 0; c < nc; ++c) {
    if (need_m[c]) merge_list.push_back((int32_t)c);
    if (need_a[c]) attach_list.push_back((int32_t)c);
  }
}

}  // namespace

int part_run(scan_graph* g, uint64_t p, uint64_t q, int32_t mu, int32_t* d_labels, uint8_t* d_roles,
             hipStream_t s) {
  PartPlan& P = g->part;
  const bool timing = g->opts.timing != 0;
  auto mark = [&](int k) {
    if (timing) (void)hipEventRecord(g->ev[k], s);
  };
  P.h2d_bytes = 0;
  const int32_t n = g->n;
  HIP_TRY(hipMemsetAsync(g->d_stats, 0, sizeof(unsigned long long) * ST_COUNT, s), "hipMemsetAsync");
  EdgeArgs A{};
  A.rp = g->d_rp;
  A.edges = P.d_edges;
  A.wtab = P.d_wtab;
  A.state = P.d_state;
  A.lower = g->d_lower;
  A.upper = g->d_upper;
  A.role = g->d_role;
  A.parent = g->d_parent;
  A.label = g->d_label;
  A.stats = g->d_stats;
  A.p = p;
  A.q = q;
  A.mu = mu;
  A.pruning = g->opts.pruning;
  mark(0);
  launch_init(s, n, g->d_rp, mu, g->d_lower, g->d_upper, g->d_role, g->d_parent);
  launch_zero_u64(s, g->d_counters, kCounters);
  mark(1);
  // Chunks each pass streams: all of them for the cores pass; after it, only
  // those holding an edge the pass can act on (merge: both endpoints cores;
  // attach: one core, one non-core, not known dissimilar), found on the host
  // from the final roles and the edge states.
  std::vector<int32_t> all((size_t)P.chunks.size()), merge_list, attach_list;
  for (size_t c = 0; c < all.size(); ++c) all[c] = (int32_t)c;
  P.chunks_streamed = 0;
  const int modes[3] = {MODE_CORES, MODE_MERGE, MODE_ATTACH};
  for (int mi = 0; mi < 3; ++mi) {
    const int mode = modes[mi];
    if (mode == MODE_MERGE) {
      mark(2);
      launch_finalize_roles(s, n, mu, g->d_lower, g->d_role, nullptr, nullptr, g->d_counters + 4);
      mark(3);
      unsigned long long ncores = 0;
      HIP_TRY(hipMemcpyAsync(&ncores, g->d_counters + 4, sizeof(ncores), hipMemcpyDeviceToHost, s), "cores D2H");
      HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
      if (ncores > 0) {  // no core: no cluster, and the merge and attach passes have nothing to do
        std::vector<uint8_t> role((size_t)n);
        if (n > 0) HIP_TRY(hipMemcpyAsync(role.data(), g->d_role, (size_t)n, hipMemcpyDeviceToHost, s), "roles D2H");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        select_chunks(P, role.data(), merge_list, attach_list);
      }
      mark(4);
    } else if (mode == MODE_ATTACH) {
      mark(5);
      launch_flatten(s, n, g->d_role, g->d_parent, g->d_label);
      mark(6);
    }
    const std::vector<int32_t>& list = mode == MODE_CORES ? all : mode == MODE_MERGE ? merge_list : attach_list;
    Streamer st{g, s};
    int idx = 0;
    for (const int32_t ci : list) {
      const PartChunk& C = P.chunks[(size_t)ci];
      if (idx == 0 || C.bi != P.chunks[(size_t)list[(size_t)idx - 1]].bi ||
          C.bj != P.chunks[(size_t)list[(size_t)idx - 1]].bj)
        HIP_TRY(st.enter(C.bi, C.bj, next_unit(P, list, (size_t)idx), A), "rows H2D");
      const int64_t ne = C.end - C.begin;
      const int b = idx & 1;
      int2* de = b ? P.d_edges2 : P.d_edges;
      uint8_t* ds = b ? P.d_state2 : P.d_state;
      // upload on the copy stream once the chunk that last used this buffer is done;
      // the cores pass starts every state at ? on the device (nothing to send)
      if (idx >= 2) HIP_TRY(hipStreamWaitEvent(P.copy, P.done[b], 0), "hipStreamWaitEvent");
      HIP_TRY(hipMemcpyAsync(de, P.h_edges + C.begin, sizeof(int2) * (size_t)ne, hipMemcpyHostToDevice, P.copy),
              "edges H2D");
      if (mode != MODE_CORES)
        HIP_TRY(hipMemcpyAsync(ds, P.h_state + C.begin, (size_t)ne, hipMemcpyHostToDevice, P.copy), "state H2D");
      HIP_TRY(hipEventRecord(P.up[b], P.copy), "hipEventRecord");
      P.h2d_bytes += (mode != MODE_CORES ? 9ull : 8ull) * (uint64_t)ne;
      ++P.chunks_streamed;
      HIP_TRY(hipStreamWaitEvent(s, P.up[b], 0), "hipStreamWaitEvent");
      A.edges = de;
      A.state = ds;
      if (mode == MODE_CORES) launch_fill_u8(s, ds, ne, SIM_UNK);
      if (mode == MODE_MERGE) launch_hook(s, ne, de, ds, g->d_role, g->d_parent);
      launch_chunk(s, mode, C, A, P);
      if (mode != MODE_ATTACH)
        HIP_TRY(hipMemcpyAsync(P.h_state + C.begin, ds, (size_t)ne, hipMemcpyDeviceToHost, s), "state D2H");
      HIP_TRY(hipEventRecord(P.done[b], s), "hipEventRecord");
      ++idx;
    }
    HIP_TRY(st.finish(), "hipEventRecord");
    // the states copied back are read by the next pass's uploads and chunk selection
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    HIP_TRY(hipStreamSynchronize(P.copy), "hipStreamSynchronize");
  }
  mark(7);
  const int32_t split = g->opts.hub_outlier ? 1 : 0;
  if (split) {  // Def 2.7: one more pass over the edges, endpoints only
    launch_fill_i32(s, g->d_upper, n, -1);
    for (const PartChunk& C : P.chunks) {
      const int64_t ne = C.end - C.begin;
      HIP_TRY(hipMemcpyAsync(P.d_edges, P.h_edges + C.begin, sizeof(int2) * (size_t)ne, hipMemcpyHostToDevice, s),
              "edges H2D");
      P.h2d_bytes += 8ull * (uint64_t)ne;
      launch_hub_outlier_edges(s, ne, P.d_edges, g->d_label, g->d_upper, g->d_role);
    }
  }
  launch_output(s, n, g->d_role, g->d_label, d_labels, d_roles, split);
  mark(8);
  HIP_TRY(hipGetLastError(), "kernel launch");
  unsigned long long stv[ST_COUNT];
  HIP_TRY(hipMemcpyAsync(stv, g->d_stats, sizeof(stv), hipMemcpyDeviceToHost, s), "stats copy");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  scan_stats L;
  memset(&L, 0, sizeof(L));
  L.edges = g->m;
  const int phase_of_mode[3] = {SCAN_PHASE_CORES, SCAN_PHASE_MERGE, SCAN_PHASE_ATTACH};
  for (int md = 0; md < 3; ++md) {
    L.evaluated[phase_of_mode[md]] = (int64_t)stv[ST_EVAL + md];
    L.bounded[phase_of_mode[md]] = (int64_t)stv[ST_BOUND + md];
    L.probes[phase_of_mode[md]] = (int64_t)stv[ST_PROBES + md];
  }
  for (int k = 0; k < kNumBuckets; ++k) {
    L.cores_bucket_evaluated[k] = (int64_t)stv[ST_BUCKET_EVAL + k];
    L.cores_bucket_probes[k] = (int64_t)stv[ST_BUCKET_PROBES + k];
  }
  L.h2d_bytes = (int64_t)P.h2d_bytes;
  L.group_split = (int64_t)stv[ST_GROUP_SPLIT];
  if (timing) {
    float ms = 0;
    for (int ph = 0; ph < SCAN_NUM_PHASES; ++ph) {
      (void)hipEventElapsedTime(&ms, g->ev[ph], g->ev[ph + 1]);
      L.ms_phase[ph] = ms;
    }
    (void)hipEventElapsedTime(&ms, g->ev[0], g->ev[SCAN_NUM_PHASES]);
    L.ms_total = ms;
  }
  set_last(g, L);
  return SCAN_OK;
}

int part_counts(scan_graph* g, int32_t* h_counts, hipStream_t s) {
  PartPlan& P = g->part;
  P.h2d_bytes = 0;
  HIP_TRY(hipMemsetAsync(g->d_stats, 0, sizeof(unsigned long long) * ST_COUNT, s), "hipMemsetAsync");
  EdgeArgs A{};
  A.rp = g->d_rp;
  A.edges = P.d_edges;
  A.wtab = P.d_wtab;
  A.edge_counts = P.d_ecount;
  A.stats = g->d_stats;
  A.p = 1;
  A.q = 1;
  A.mu = 2;
  A.pruning = 0;
  Streamer st{g, s};
  std::vector<int32_t> all(P.chunks.size());
  for (size_t c = 0; c < all.size(); ++c) all[c] = (int32_t)c;
  for (size_t idx = 0; idx < all.size(); ++idx) {
    const PartChunk& C = P.chunks[idx];
    const int64_t ne = C.end - C.begin;
    if (idx == 0 || C.bi != P.chunks[idx - 1].bi || C.bj != P.chunks[idx - 1].bj)
      HIP_TRY(st.enter(C.bi, C.bj, next_unit(P, all, idx), A), "rows H2D");
    HIP_TRY(hipMemcpyAsync(P.d_edges, P.h_edges + C.begin, sizeof(int2) * (size_t)ne, hipMemcpyHostToDevice, s),
            "edges H2D");
    launch_chunk(s, MODE_COUNTS, C, A, P);
    HIP_TRY(hipMemcpyAsync(P.h_ecount + C.begin, P.d_ecount, sizeof(int32_t) * (size_t)ne, hipMemcpyDeviceToHost, s),
            "counts D2H");
  }
  HIP_TRY(st.finish(), "hipEventRecord");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  // per-edge counts to both arcs (CSR order)
  const int64_t m = g->m;
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      for (int64_t k = t; k < m; k += nth) {
        const int2 uv = P.h_edges[k];
        const int32_t* ru = P.h_ci + P.h_rp[(size_t)uv.x];
        const int32_t* rv = P.h_ci + P.h_rp[(size_t)uv.y];
        const int64_t du = P.h_rp[(size_t)uv.x + 1] - P.h_rp[(size_t)uv.x];
        const int64_t dv = P.h_rp[(size_t)uv.y + 1] - P.h_rp[(size_t)uv.y];
        const int64_t pu = std::lower_bound(ru, ru + du, uv.y) - ru;
        const int64_t pv = std::lower_bound(rv, rv + dv, uv.x) - rv;
        h_counts[P.h_rp[(size_t)uv.x] + pu] = P.h_ecount[k];
        h_counts[P.h_rp[(size_t)uv.y] + pv] = P.h_ecount[k];
      }
    });
  for (auto& x : th) x.join();
  unsigned long long stv[ST_COUNT];
  HIP_TRY(hipMemcpy(stv, g->d_stats, sizeof(stv), hipMemcpyDeviceToHost), "stats copy");
  scan_stats L{};
  L.edges = m;
  L.h2d_bytes = (int64_t)P.h2d_bytes;
  L.group_split = (int64_t)stv[ST_GROUP_SPLIT];
  set_last(g, L);
  return SCAN_OK;
}

}  // namespace scan
