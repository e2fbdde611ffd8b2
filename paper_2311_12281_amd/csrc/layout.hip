// Graph ingest on the device: CSR validation and the degree-oriented edge
// list of GPUSCAN++ Section 4.1 ("degree-oriented edge array": every edge
// once as (u, v) with deg(u) < deg(v), or equal degrees and id(u) < id(v)),
// grouped by the degree bucket of its smaller side and, inside a bucket, in
// CSR order of the larger side.  The grouping is a stable multi-way
// partition: per-block bucket counts, one exclusive scan, ordered scatter.
#include "scan_internal.h"

#include <algorithm>
#include <thread>
#include <vector>

namespace scan {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 4;                 // arcs per thread per block
constexpr int kTile = kBlock * kItems;    // arcs per block

enum : int {
  ERR_OFFSETS = 1,
  ERR_RANGE = 2,
  ERR_SELFLOOP = 4,
  ERR_ORDER = 8,
  ERR_ASYM = 16,
};

__global__ void k_check_offsets(int32_t n, int64_t nnz, const int64_t* rp, int32_t* err,
                                int32_t* maxdeg) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > n) return;
  if (u == 0 && rp[0] != 0) atomicOr(err, ERR_OFFSETS);
  if (u == n && rp[n] != nnz) atomicOr(err, ERR_OFFSETS);
  if (u < n) {
    int64_t d = rp[u + 1] - rp[u];
    if (d < 0 || rp[u] < 0 || rp[u + 1] > nnz) atomicOr(err, ERR_OFFSETS);
    else if (d > 0) atomicMax(maxdeg, (int32_t)(d > 0x7fffffff ? 0x7fffffff : d));
  }
}

// Row id of every arc (rows are processed one wave per vertex).
__global__ void k_arc_rows(int32_t n, const int64_t* rp, int32_t* src) {
  const int lane = threadIdx.x & 63;
  int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = w; u < n; u += nw) {
    for (int64_t i = rp[u] + lane; i < rp[u + 1]; i += 64) src[i] = (int32_t)u;
  }
}

__device__ inline bool row_contains(const int32_t* row, int64_t len, int32_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int32_t y = row[mid];
    if (y < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && row[lo] == x;
}

__global__ void k_check_arcs(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                             const int32_t* src, int32_t* err, int full) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t e = 0;
  for (; i < nnz; i += stride) {
    const int32_t u = src[i];
    const int32_t v = ci[i];
    if (v < 0 || v >= n) { e |= ERR_RANGE; continue; }
    if (!full) continue;
    if (v == u) e |= ERR_SELFLOOP;
    if (i > rp[u] && ci[i - 1] >= v) e |= ERR_ORDER;
    if (!row_contains(ci + rp[v], rp[v + 1] - rp[v], u)) e |= ERR_ASYM;
  }
  if (e) atomicOr(err, e);
}

// Owner arc of each undirected edge, and its bucket (or -1 if arc i does not
// own its edge).  With x = row of arc i and y = its neighbour, the edge's
// smaller side by (degree, id) is u and the larger is v.  Every edge is owned
// by the arc in v's row, so each bucket lists its edges grouped by the larger
// side: consecutive edges share v's degree, role, bounds and row (the larger
// list that the intersections search), and in bucket 6 each job of the
// LDS-hash kernel stages one larger list and streams the smaller lists of its
// in-edges.
__device__ inline int arc_bucket(const int64_t* rp, const int32_t* ci, const int32_t* src, int64_t i) {
  const int32_t x = src[i], y = ci[i];
  const int64_t dx = rp[x + 1] - rp[x], dy = rp[y + 1] - rp[y];
  const bool x_smaller = dx < dy || (dx == dy && x < y);
  const int64_t ds = x_smaller ? dx : dy, dl = x_smaller ? dy : dx;
  int b = bucket_of(ds);
  if (b == 5 && dl > kHubMinDegree) b = 6;
  return x_smaller ? -1 : b;  // the larger side's arc owns the edge
}

__global__ __launch_bounds__(kBlock) void k_bucket_counts(int64_t nnz, const int64_t* rp,
                                                          const int32_t* ci, const int32_t* src,
                                                          int64_t nblocks, int64_t* counts) {
  __shared__ int32_t c[kNumBuckets];
  if (threadIdx.x < kNumBuckets) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
    if (i < nnz) {
      int b = arc_bucket(rp, ci, src, i);
      if (b >= 0) atomicAdd(&c[b], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < kNumBuckets) counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = c[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_bucket_scatter(int64_t nnz, const int64_t* rp,
                                                           const int32_t* ci, const int32_t* src,
                                                           int64_t nblocks, const int64_t* offsets,
                                                           int2* edges) {
  __shared__ int32_t wave_cnt[kNumBuckets][kBlock / 64];
  __shared__ int64_t running[kNumBuckets];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < kNumBuckets) running[threadIdx.x] = offsets[(int64_t)threadIdx.x * nblocks + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
    const int b = (i < nnz) ? arc_bucket(rp, ci, src, i) : -1;
    int myrank = 0;
    __syncthreads();
    for (int k = 0; k < kNumBuckets; ++k) {
      const uint64_t mask = __ballot(b == k);
      if (b == k) myrank = __popcll(mask & lt);
      if (lane == 0) wave_cnt[k][wave] = __popcll(mask);
    }
    __syncthreads();
    if (b >= 0) {
      int64_t pos = running[b] + myrank;
      for (int w = 0; w < wave; ++w) pos += wave_cnt[b][w];
      // stored as (smaller side, larger side); arc i lies in the larger side's row
      edges[pos] = make_int2(ci[i], src[i]);
    }
    __syncthreads();
    if (threadIdx.x < kNumBuckets) {
      int64_t t = 0;
      for (int w = 0; w < kBlock / 64; ++w) t += wave_cnt[threadIdx.x][w];
      running[threadIdx.x] += t;
    }
  }
}

// Exclusive scan of int64, 1024 elements per block; block totals to sums.
__global__ __launch_bounds__(kBlock) void k_scan_block(const int64_t* in, int64_t* out, int64_t n,
                                                       int64_t* sums) {
  __shared__ int64_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t v[kItems];
  int64_t t = 0;
  for (int k = 0; k < kItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    t += v[k];
  }
  int64_t incl = t;
  for (int d = 1; d < 64; d <<= 1) {
    int64_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += wsum[w];
  int64_t run = woff + incl - t;
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1 && sums) sums[blockIdx.x] = woff + incl;
}

__global__ void k_scan_add(int64_t* data, int64_t n, const int64_t* add) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) data[i] += add[i / kTile];
}

hipError_t exclusive_scan(hipStream_t s, const int64_t* in, int64_t* out, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kTile - 1) / kTile;
  if (nb == 1) {
    k_scan_block<<<1, kBlock, 0, s>>>(in, out, n, nullptr);
    return hipGetLastError();
  }
  int64_t* sums = nullptr;
  hipError_t e = hipMalloc((void**)&sums, sizeof(int64_t) * nb * 2);
  if (e != hipSuccess) return e;
  k_scan_block<<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, sums);
  e = exclusive_scan(s, sums, sums + nb, nb);
  if (e == hipSuccess) {
    k_scan_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n, sums + nb);
    e = hipGetLastError();
  }
  hipError_t f = hipStreamSynchronize(s);
  hipFree(sums);
  return e != hipSuccess ? e : f;
}


}  // namespace

int64_t hub_windows(const int32_t* row, int64_t dv, std::vector<uint32_t>& out) {
  // The same windows the LDS-hash kernel would find: a bitmap of the ids
  // row[w0] .. row[w0] + kHubBitmapBits - 1 where that range holds at least
  // kHubBitmapMin elements from w0 on, else a hash set of the next kHubWindow
  // elements, cut where the longest suffix that one bitmap covers begins (if
  // that suffix holds at least kHubBitmapMin elements).
  int64_t wsuf = dv;
  if (dv >= kHubBitmapMin) {
    const int64_t T = (int64_t)row[dv - 1] - kHubBitmapBits + 1;
    const int64_t ws = std::lower_bound(row, row + dv, T, [](int32_t a, int64_t b) { return (int64_t)a < b; }) - row;
    if (dv - ws >= kHubBitmapMin) wsuf = ws;
  }
  int64_t cnt = 0;
  for (int64_t w0 = 0, w1 = 0; w0 < dv; w0 = w1, ++cnt) {
    w1 = (dv - w0 > kHubWindow) ? w0 + kHubWindow : dv;
    if (w0 < wsuf && w1 > wsuf) w1 = wsuf;
    bool bitmap = false;
    if (dv - w0 >= kHubBitmapMin) {
      const int64_t lim = (int64_t)row[w0] + kHubBitmapBits;
      const int64_t wb = std::lower_bound(row + w0 + 1, row + dv, lim,
                                          [](int32_t a, int64_t b) { return (int64_t)a < b; }) - row;
      if (wb - w0 >= kHubBitmapMin) {
        bitmap = true;
        w1 = wb;
      }
    }
    out.push_back(((uint32_t)w1 << 1) | (bitmap ? 1u : 0u));
  }
  return cnt;
}

void assign_hub_windows(std::vector<HubJob>& jobs, const int64_t* rp, const int32_t* rows,
                        std::vector<uint32_t>& table) {
  table.clear();
  std::vector<std::pair<int32_t, size_t>> order(jobs.size());
  for (size_t k = 0; k < jobs.size(); ++k) order[k] = {jobs[k].v, k};
  std::sort(order.begin(), order.end());
  for (size_t k = 0; k < order.size();) {
    const int32_t v = order[k].first;
    const int32_t wbeg = (int32_t)table.size();
    const int32_t wcnt = (int32_t)hub_windows(rows + rp[v], rp[v + 1] - rp[v], table);
    for (; k < order.size() && order[k].first == v; ++k) {
      jobs[order[k].second].wbeg = wbeg;
      jobs[order[k].second].wcnt = wcnt;
    }
  }
}

hipError_t build_ranked_rows(hipStream_t s, int32_t n, int64_t nnz, const int64_t* h_rp,
                             const int32_t* h_ci, int32_t* d_hci, std::vector<int32_t>* h_hci) {
  if (nnz <= 0 || n <= 0) return hipSuccess;
  // rank: counting sort of the vertices by increasing degree, ties by id
  int64_t maxd = 0;
  for (int32_t v = 0; v < n; ++v) maxd = std::max(maxd, h_rp[v + 1] - h_rp[v]);
  std::vector<int64_t> first((size_t)maxd + 2, 0);
  for (int32_t v = 0; v < n; ++v) ++first[(size_t)(h_rp[v + 1] - h_rp[v])];
  int64_t acc = 0;
  for (auto& c : first) {
    const int64_t t = c;
    c = acc;
    acc += t;
  }
  std::vector<int32_t> rank((size_t)n);
  for (int32_t v = 0; v < n; ++v) rank[(size_t)v] = (int32_t)first[(size_t)(h_rp[v + 1] - h_rp[v])]++;
  // renamed rows, each sorted again; threads take row ranges of about equal arc counts
  std::vector<int32_t> out((size_t)nnz);
  const int nth = 16;
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      // rows whose start lies in [nnz t / nth, nnz (t + 1) / nth): every row once
      auto first_row = [&](int k) -> int32_t {
        if (k >= nth) return n;
        return (int32_t)(std::lower_bound(h_rp, h_rp + n, nnz * k / nth) - h_rp);
      };
      const int32_t r0 = first_row(t), r1 = first_row(t + 1);
      for (int32_t v = r0; v < r1; ++v) {
        int32_t* r = out.data() + h_rp[v];
        for (int64_t k = h_rp[v]; k < h_rp[v + 1]; ++k) r[k - h_rp[v]] = rank[(size_t)h_ci[k]];
        std::sort(r, r + (h_rp[v + 1] - h_rp[v]));
      }
    });
  for (auto& x : th) x.join();
  hipError_t e = hipMemcpyAsync(d_hci, out.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (h_hci) h_hci->swap(out);
  return e;
}

hipError_t build_layout(hipStream_t s, int32_t n, int64_t nnz, const int64_t* h_rp,
                        const int32_t* h_ci, const int64_t* d_rp, const int32_t* d_ci, int validate,
                        int2** d_edges_out, std::vector<HubJob>* jobs_out, LayoutResult* out) {
  hipError_t e = hipSuccess;
  jobs_out->clear();
  out->hub_jobs = 0;
  int32_t* d_flags = nullptr;  // [0] = error bits, [1] = max degree
  int32_t* d_src = nullptr;
  int64_t* d_cnt = nullptr;
  int2* d_edges = nullptr;
  const int64_t nblocks = (nnz + kTile - 1) / kTile;
  const int64_t ncnt = nblocks * kNumBuckets;
  int32_t h_flags[2] = {0, 0};
  int64_t h_off[kNumBuckets];
  int64_t h_last[2] = {0, 0};
  *d_edges_out = nullptr;
  for (int k = 0; k <= kNumBuckets; ++k) out->bucket_off[k] = 0;
  out->error = 0;
  out->max_degree = 0;
#define LTRY(x) do { e = (x); if (e != hipSuccess) goto done; } while (0)
  LTRY(hipMalloc((void**)&d_flags, sizeof(int32_t) * 2));
  LTRY(hipMemsetAsync(d_flags, 0, sizeof(int32_t) * 2, s));
  k_check_offsets<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(n, nnz, d_rp, d_flags, d_flags + 1);
  LTRY(hipGetLastError());
  LTRY(hipMemcpyAsync(h_flags, d_flags, sizeof(h_flags), hipMemcpyDeviceToHost, s));
  LTRY(hipStreamSynchronize(s));
  out->error = h_flags[0];
  out->max_degree = h_flags[1];
  if (h_flags[0] != 0 || nnz == 0) goto done;  // offsets unusable, or no edges
  LTRY(hipMalloc((void**)&d_src, sizeof(int32_t) * nnz));
  k_arc_rows<<<4096, 256, 0, s>>>(n, d_rp, d_src);
  LTRY(hipGetLastError());
  // The id-range check always runs (every later kernel indexes rp by ids);
  // order and symmetry are checked when validation is on.
  k_check_arcs<<<8192, 256, 0, s>>>(n, nnz, d_rp, d_ci, d_src, d_flags, validate);
  LTRY(hipGetLastError());
  LTRY(hipMemcpyAsync(h_flags, d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LTRY(hipStreamSynchronize(s));
  out->error = h_flags[0];
  if (h_flags[0] != 0) goto done;
  LTRY(hipMalloc((void**)&d_cnt, sizeof(int64_t) * ncnt * 2));
  k_bucket_counts<<<(unsigned)nblocks, kBlock, 0, s>>>(nnz, d_rp, d_ci, d_src, nblocks, d_cnt);
  LTRY(hipGetLastError());
  LTRY(exclusive_scan(s, d_cnt, d_cnt + ncnt, ncnt));
  for (int k = 0; k < kNumBuckets; ++k)
    LTRY(hipMemcpyAsync(&h_off[k], d_cnt + ncnt + (int64_t)k * nblocks, sizeof(int64_t),
                        hipMemcpyDeviceToHost, s));
  LTRY(hipMemcpyAsync(&h_last[0], d_cnt + ncnt - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LTRY(hipMemcpyAsync(&h_last[1], d_cnt + 2 * ncnt - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LTRY(hipStreamSynchronize(s));
  for (int k = 0; k < kNumBuckets; ++k) out->bucket_off[k] = h_off[k];
  out->bucket_off[kNumBuckets] = h_last[0] + h_last[1];  // total owned arcs = edges
  LTRY(hipMalloc((void**)&d_edges, sizeof(int2) * (out->bucket_off[kNumBuckets] > 0 ? out->bucket_off[kNumBuckets] : 1)));
  k_bucket_scatter<<<(unsigned)nblocks, kBlock, 0, s>>>(nnz, d_rp, d_ci, d_src, nblocks,
                                                        d_cnt + ncnt, d_edges);
  LTRY(hipGetLastError());
  LTRY(hipStreamSynchronize(s));
  {
    // Jobs of the last bucket.  Its edges are listed by increasing larger
    // side v and, within v, in the order of v's row; a job is a run of one v's
    // in-edges holding at most kHubJobEdges edges and at most kHubJobWork
    // elements of smaller lists, so that the heaviest tables are shared by
    // many blocks.  The table is ordered by decreasing deg(v).  Computed on the
    // host from the caller's CSR with the predicate the device used.
    const int64_t b6 = out->bucket_off[kNumBuckets - 1], e6 = out->bucket_off[kNumBuckets];
    if (e6 > b6 && n > 0) {
      auto deg = [&](int32_t x) { return h_rp[x + 1] - h_rp[x]; };
      auto in_edge = [&](int32_t v, int32_t u) {  // edge (u, v) is in the last bucket, owned by v
        const int64_t dv = deg(v), du = deg(u);
        const bool u_smaller = du < dv || (du == dv && u < v);
        return u_smaller && du > 64 && dv > kHubMinDegree;
      };
      const int nth = 16;
      std::vector<std::vector<HubJob>> part(nth);
      std::vector<int64_t> cnt((size_t)n, 0);
      std::vector<std::thread> th;
      // pass 1: in-edge counts per v (for the segment starts)
      for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t]() {
          for (int32_t v = t; v < n; v += nth) {
            if (deg(v) <= kHubMinDegree) continue;
            int64_t c = 0;
            for (int64_t k = h_rp[v]; k < h_rp[v + 1]; ++k) c += in_edge(v, h_ci[k]);
            cnt[(size_t)v] = c;
          }
        });
      for (auto& x : th) x.join();
      th.clear();
      std::vector<int64_t> start((size_t)n);
      int64_t acc = 0;
      for (int32_t v = 0; v < n; ++v) {
        start[(size_t)v] = acc;
        acc += cnt[(size_t)v];
      }
      if (acc != e6 - b6) {
        out->error = 32;  // host and device disagree on the bucket (cannot happen for a valid CSR)
        goto done;
      }
      // pass 2: cut each v's in-edges into jobs
      for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t]() {
          for (int32_t v = t; v < n; v += nth) {
            if (cnt[(size_t)v] == 0) continue;
            HubJob J{};
            J.v = v;
            J.begin = b6 + start[(size_t)v];
            J.count = 0;
            int64_t work = 0;
            for (int64_t k = h_rp[v]; k < h_rp[v + 1]; ++k) {
              const int32_t u = h_ci[k];
              if (!in_edge(v, u)) continue;
              if (J.count > 0 && (J.count == kHubJobEdges || work + deg(u) > kHubJobWork)) {
                part[(size_t)t].push_back(J);
                J.begin += J.count;
                J.count = 0;
                work = 0;
              }
              ++J.count;
              work += deg(u);
            }
            part[(size_t)t].push_back(J);
          }
        });
      for (auto& x : th) x.join();
      std::vector<HubJob>& jobs = *jobs_out;
      for (auto& p : part) jobs.insert(jobs.end(), p.begin(), p.end());
      std::stable_sort(jobs.begin(), jobs.end(), [&](const HubJob& a, const HubJob& b) {
        const int64_t da = deg(a.v), db = deg(b.v);
        return da != db ? da > db : a.begin < b.begin;
      });
      out->hub_jobs = (int64_t)jobs.size();
    }
  }
  *d_edges_out = d_edges;
  d_edges = nullptr;
done:
  hipStreamSynchronize(s);
  if (d_edges) hipFree(d_edges);
  if (d_cnt) hipFree(d_cnt);
  if (d_src) hipFree(d_src);
  if (d_flags) hipFree(d_flags);
#undef LTRY
  return e;
}

}  // namespace scan
