// Clustering kernels for gfx950 (wave64).
//
// The run follows GPUSCAN++ Algorithms 1-3:
//   init          bounds lower = 1, upper = deg + 1, role ?, sim ?   (Alg. 1; Sec. 4.2 text)
//   CORES pass    identifyCore: for every oriented edge with a role still
//                 unknown, test sigma >= eps and move the bounds; Lemma 4.1
//                 decides a role as soon as lower >= mu or upper < mu  (Alg. 2)
//   finalize      a role still unknown after the pass is decided by its now
//                 exact count
//   hook          union along core-core edges already known similar  (Alg. 3, first loop)
//   MERGE pass    core-core edges of unknown similarity are tested only when
//                 their endpoints are still in different trees        (Alg. 3, second loop)
//   flatten       label = root = minimum core id of the tree          (Alg. 3, third loop)
//   ATTACH pass   a non-core similar to a core takes the smallest label (Alg. 3, last loop)
//
// The similarity test is exact: |N[u] & N[v]| = |nbr(u) & nbr(v)| + 2 for
// adjacent u, v (each endpoint lies in the other's closed set and in its
// own), compared with the integer threshold closed_needed(p, q, a, b).
//
// Edges are processed in degree buckets of the smaller side d_s:
//   d_s <= 64 : k_group - lanes classify 64 edges at once, then groups of
//               G in {4, 8, 16, 32, 64} lanes intersect the edges that need
//               it, one lane per element of the smaller list binary-searching
//               the larger list; the group's count is a ballot popcount.
//   d_s  > 64 : k_hub - edges grouped by their larger side v, whose
//               neighbours are staged in an LDS hash table that the smaller
//               lists are streamed through (strategy 1 uses k_group with G = 64
//               instead).
// Every intersection stops as soon as the verdict is known (count reached or
// unreachable), except when exact counts are requested.
#include "scan_internal.h"

#include <climits>

namespace scan {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint8_t ld_u8(const uint8_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u8(uint8_t* p, uint8_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_i32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_i32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union-find with min-id hooking: a root is only ever linked below a smaller
// root, so parent[x] <= x always holds, no cycle can form, and the final root
// of every tree is its minimum member.  find() halves paths; every value it
// writes is an ancestor of x, which stays an ancestor forever.
__device__ int32_t uf_find(int32_t* parent, int32_t x) {
  while (true) {
    const int32_t p = ld_i32(parent + x);
    if (p == x) return x;
    const int32_t gp = ld_i32(parent + p);
    if (gp == p) return p;
    st_i32(parent + x, gp);
    x = gp;
  }
}

__device__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) { int32_t t = a; a = b; b = t; }
    const int32_t old = atomicCAS(parent + b, b, a);
    if (old == b) return;
  }
}

// First position in row[lo, hi) whose value is >= x.
__device__ __forceinline__ int64_t lower_bound(const int32_t* row, int64_t lo, int64_t hi, int32_t x) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (row[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Position of x's row in A.ci.  In memory this is rp[x]; on the partitioned
// path A.ci holds the rows of two vertex ranges side by side, and each range
// is shifted by its own delta.
__device__ __forceinline__ int64_t row_start(const EdgeArgs& A, int32_t x) {
  return A.rp[x] - ((x >= A.a_lo && x < A.a_hi) ? A.delta_a : A.delta_b);
}

// Per-edge decision taken before any intersection.
struct EdgeView {
  int32_t u, v;       // u = smaller side
  int64_t bu, bv;     // row starts
  int64_t du, dv;     // degrees
  int32_t need;       // closed count needed for similarity
  int32_t core_side;  // ATTACH: endpoint that is the core (u or v)
  int32_t other;      // ATTACH: the non-core endpoint
  int32_t core_label; // ATTACH
  int32_t mu;         // the edge's graph's mu
  uint8_t work;       // 1: run the intersection
  uint8_t open_u, open_v;  // cores pass: the endpoint's role was still unknown when read, so
                           // its bounds still matter (a known role never changes again)
};

// eps = p/q and mu of the graph holding vertex x (one graph, or a batch of
// graphs with per-graph parameters looked up through the vertex's graph id).
__device__ __forceinline__ void graph_params(const EdgeArgs& A, int32_t x, uint64_t& p, uint64_t& q,
                                             int32_t& mu) {
  if (A.gid) {
    const int32_t g = A.gid[x];
    p = A.gp[g];
    q = A.gq[g];
    mu = A.gmu[g];
  } else {
    p = A.p;
    q = A.q;
    mu = A.mu;
  }
}

template <int MODE>
__device__ __forceinline__ void classify(const EdgeArgs& A, int64_t e, bool active, EdgeView& ev,
                                         unsigned long long& n_bound) {
  ev = EdgeView{};
  ev.open_u = ev.open_v = 1;
  if (!active) return;
  const int2 uv = A.edges[e];
  ev.u = uv.x;
  ev.v = uv.y;
  if (A.edeg) {  // both degrees with the edge: no row offsets unless the edge is intersected
    const int2 d = A.edeg[e];
    ev.du = d.x;
    ev.dv = d.y;
  } else {
    ev.du = A.rp[ev.u + 1] - A.rp[ev.u];
    ev.dv = A.rp[ev.v + 1] - A.rp[ev.v];
  }
  const uint64_t a = (uint64_t)ev.du + 1, b = (uint64_t)ev.dv + 1;
  if (MODE == MODE_COUNTS) {
    ev.bu = row_start(A, ev.u);
    ev.bv = row_start(A, ev.v);
    ev.need = 0;
    ev.work = 1;
    return;
  }
  uint64_t p, q;
  graph_params(A, ev.u, p, q, ev.mu);
  if (MODE == MODE_CORES) {
    if (A.pruning) {
      const uint8_t ru = ld_u8(A.role + ev.u), rv = ld_u8(A.role + ev.v);
      if (ru != ROLE_UNK && rv != ROLE_UNK) return;  // Alg. 2: both roles known, defer
      ev.open_u = ru == ROLE_UNK;
      ev.open_v = rv == ROLE_UNK;
    }
  } else if (MODE == MODE_MERGE) {
    if (A.state[e] != SIM_UNK) return;
    if (ld_u8(A.role + ev.u) != ROLE_CORE || ld_u8(A.role + ev.v) != ROLE_CORE) return;
    if (A.pruning && uf_find(A.parent, ev.u) == uf_find(A.parent, ev.v)) return;  // already one cluster
  } else {  // MODE_ATTACH
    const bool cu = ld_u8(A.role + ev.u) == ROLE_CORE, cv = ld_u8(A.role + ev.v) == ROLE_CORE;
    if (cu == cv) return;
    const uint8_t st = A.state[e];
    if (st == SIM_NO) return;
    ev.core_side = cu ? ev.u : ev.v;
    ev.other = cu ? ev.v : ev.u;
    ev.core_label = A.label[ev.core_side];
    if (st == SIM_YES) {
      ev.work = 2;  // known similar: attach without intersecting
      return;
    }
    if (A.pruning && ld_i32(A.label + ev.other) <= ev.core_label) return;  // no smaller label possible
  }
  // |N[u] & N[v]| <= min(a, b) = a, so a q^2 < p^2 b already means dissimilar.
  if (A.pruning && a * q * q < p * p * b) {
    ev.work = 3;
    ++n_bound;
    return;
  }
  ev.need = (int32_t)closed_needed(p, q, a, b);
  ev.bu = row_start(A, ev.u);
  ev.bv = row_start(A, ev.v);
  ev.work = 1;
}

// Fields of an edge already known to need an intersection (phase B of the
// LDS-hash kernel).  Returns false for a cores-pass edge whose two roles have
// become known in the meantime: it is deferred like any other such edge.
template <int MODE>
__device__ __forceinline__ bool load_survivor(const EdgeArgs& A, int64_t e, EdgeView& ev) {
  const int2 uv = A.edges[e];
  ev.u = uv.x;
  ev.v = uv.y;
  ev.du = A.rp[ev.u + 1] - A.rp[ev.u];
  ev.dv = A.rp[ev.v + 1] - A.rp[ev.v];
  ev.bu = row_start(A, ev.u);
  ev.bv = row_start(A, ev.v);
  ev.need = 0;
  ev.work = 1;
  ev.open_u = ev.open_v = 1;
  if (MODE == MODE_COUNTS) return true;
  uint64_t p, q;
  graph_params(A, ev.u, p, q, ev.mu);
  ev.need = (int32_t)closed_needed(p, q, (uint64_t)ev.du + 1, (uint64_t)ev.dv + 1);
  if (MODE == MODE_CORES) {
    if (A.pruning) {
      const uint8_t ru = ld_u8(A.role + ev.u), rv = ld_u8(A.role + ev.v);
      if (ru != ROLE_UNK && rv != ROLE_UNK) return false;
      ev.open_u = ru == ROLE_UNK;
      ev.open_v = rv == ROLE_UNK;
    }
  } else if (MODE == MODE_ATTACH) {
    const bool cu = ld_u8(A.role + ev.u) == ROLE_CORE;
    ev.core_side = cu ? ev.u : ev.v;
    ev.other = cu ? ev.v : ev.u;
    ev.core_label = A.label[ev.core_side];
  }
  return true;
}

// Cores pass, effect of a decided edge in two halves, so that a thread can
// have the counter updates of several edges in flight before it needs their
// results: the bound moved on both endpoints (lower on a similar edge, upper on
// a dissimilar one; both atomics issued back to back, values before the update
// returned), then the roles those values settle (Lemma 4.1).
// Only endpoints whose role was unknown are updated (do_u, do_v): a known role
// never changes, and the final count is read only for roles still unknown.
// The upper bound is kept only for degrees up to kUpperMaxDegree: it serves
// just to mark a vertex non-core early (Lemma 4.1), which for a vertex of
// higher degree happens only after most of its edges were tested, while every
// one of its dissimilar edges costs a device-scope atomic on that vertex's
// counter; the few intersections an early mark saves do not pay for those
// beyond a few dozen neighbours.  Such a vertex keeps role ? and is settled
// from its exact lower bound at the end of the pass.
constexpr int64_t kUpperMaxDegree = 16;
static_assert(kUpperMaxDegree < kHubMinDegree, "the LDS-hash kernel keeps no upper bound for its larger side");
__device__ __forceinline__ void cores_count(const EdgeArgs& A, const EdgeView& ev, bool sim, bool do_u,
                                            bool do_v, int32_t& cu, int32_t& cv) {
  int32_t* c = sim ? A.lower : A.upper;
  const int32_t d = sim ? 1 : -1;
  do_u = do_u && (sim || ev.du <= kUpperMaxDegree);
  do_v = do_v && (sim || ev.dv <= kUpperMaxDegree);
  cu = do_u ? atomicAdd(c + ev.u, d) : 0;
  cv = do_v ? atomicAdd(c + ev.v, d) : 0;
}

__device__ __forceinline__ void cores_roles(const EdgeArgs& A, const EdgeView& ev, bool sim, bool do_u,
                                            bool do_v, int32_t cu, int32_t cv) {
  do_u = do_u && (sim || ev.du <= kUpperMaxDegree);
  do_v = do_v && (sim || ev.dv <= kUpperMaxDegree);
  if (sim) {
    if (do_u && cu + 1 >= ev.mu) st_u8(A.role + ev.u, ROLE_CORE);
    if (do_v && cv + 1 >= ev.mu) st_u8(A.role + ev.v, ROLE_CORE);
  } else {
    if (do_u && cu - 1 < ev.mu) st_u8(A.role + ev.u, ROLE_NONCORE);
    if (do_v && cv - 1 < ev.mu) st_u8(A.role + ev.v, ROLE_NONCORE);
  }
}

// Effect of a decided edge; executed by one lane.
template <int MODE>
__device__ __forceinline__ void apply(const EdgeArgs& A, int64_t e, const EdgeView& ev, bool sim,
                                      int32_t closed) {
  if (MODE == MODE_COUNTS) {
    if (A.edge_counts) A.edge_counts[e] = closed;
    if (A.counts) {
      const int64_t pu = lower_bound(A.ci, ev.bu, ev.bu + ev.du, ev.v);
      const int64_t pv = lower_bound(A.ci, ev.bv, ev.bv + ev.dv, ev.u);
      if (pu < ev.bu + ev.du && A.ci[pu] == ev.v) A.counts[pu] = closed;
      if (pv < ev.bv + ev.dv && A.ci[pv] == ev.u) A.counts[pv] = closed;
    }
    return;
  }
  if (MODE == MODE_CORES) {
    int32_t cu, cv;
    cores_count(A, ev, sim, ev.open_u, ev.open_v, cu, cv);
    A.state[e] = sim ? SIM_YES : SIM_NO;
    cores_roles(A, ev, sim, ev.open_u, ev.open_v, cu, cv);
  } else if (MODE == MODE_MERGE) {
    A.state[e] = sim ? SIM_YES : SIM_NO;
    if (sim) uf_union(A.parent, ev.u, ev.v);
  } else {
    if (sim) atomicMin(A.label + ev.other, ev.core_label);
  }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__device__ __forceinline__ void flush_stats(const EdgeArgs& A, int mode, unsigned long long ev,
                                            unsigned long long bd, unsigned long long pr) {
  ev = wave_sum(ev);
  bd = wave_sum(bd);
  pr = wave_sum(pr);
  if ((threadIdx.x & 63) == 0) {
    if (ev) atomicAdd(A.stats + ST_EVAL + mode, ev);
    if (bd) atomicAdd(A.stats + ST_BOUND + mode, bd);
    if (pr) atomicAdd(A.stats + ST_PROBES + mode, pr);
    if (mode == MODE_CORES) {
      if (ev) atomicAdd(A.stats + ST_BUCKET_EVAL + A.bucket, ev);
      if (pr) atomicAdd(A.stats + ST_BUCKET_PROBES + A.bucket, pr);
    }
  }
}

// The same totals summed over the block first (every thread of the block must
// call it): one set of atomics per block instead of one per wave, since many
// short-lived waves adding to the same few counters serialise on them.
template <int NW>
__device__ __forceinline__ void flush_stats_block(const EdgeArgs& A, int mode, unsigned long long ev,
                                                  unsigned long long bd, unsigned long long pr) {
  __shared__ unsigned long long part[3][NW];
  ev = wave_sum(ev);
  bd = wave_sum(bd);
  pr = wave_sum(pr);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][w] = ev;
    part[1][w] = bd;
    part[2][w] = pr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ev = bd = pr = 0;
    for (int k = 0; k < NW; ++k) {
      ev += part[0][k];
      bd += part[1][k];
      pr += part[2][k];
    }
    if (ev) atomicAdd(A.stats + ST_EVAL + mode, ev);
    if (bd) atomicAdd(A.stats + ST_BOUND + mode, bd);
    if (pr) atomicAdd(A.stats + ST_PROBES + mode, pr);
    if (mode == MODE_CORES) {
      if (ev) atomicAdd(A.stats + ST_BUCKET_EVAL + A.bucket, ev);
      if (pr) atomicAdd(A.stats + ST_BUCKET_PROBES + A.bucket, pr);
    }
  }
}

// A group of G lanes intersects the smaller list nbr(u) (length du) with the
// larger list nbr(v) (length dv): nbr(u) in tiles of G elements, every lane
// binary-searching its element in the unread remainder of nbr(v) (both lists
// are sorted, so the remainder only shrinks).  cnt receives the open common
// neighbours found, consumed the elements of nbr(u) read.  Unless `exact`,
// the loop stops as soon as the verdict against need_open is certain.
// Returns 2 (similar), 3 (dissimilar) or 1 (full count, undecided).
template <int G>
__device__ __forceinline__ int group_intersect(const int32_t* Arow, int64_t du, const int32_t* B,
                                               int64_t dv, int32_t need_open, bool exact, int sub,
                                               int gbase, uint64_t gmask, int32_t& cnt,
                                               int64_t& consumed) {
  cnt = 0;
  consumed = 0;
  int64_t lo = 0;
  for (int64_t t = 0; t < du; t += G) {
    const int64_t i = t + sub;
    int64_t pos = dv;
    bool f = false;
    if (i < du) {
      const int32_t x = Arow[i];
      pos = lower_bound(B, lo, dv, x);
      f = pos < dv && B[pos] == x;
    }
    cnt += __popcll(__ballot(f) & gmask);
    const int64_t take = du - t < G ? du - t : G;
    consumed += take;
    lo = __shfl(pos, gbase + (int)(take - 1), 64);
    if (!exact) {
      if (cnt >= need_open) return 2;
      int64_t rem = du - (t + take);
      if (dv - lo < rem) rem = dv - lo;
      if (cnt + rem < need_open) return 3;
    }
    if (lo >= dv) break;  // the larger list is exhausted
  }
  return 1;
}

template <typename T>
__device__ __forceinline__ T shfl_t(T x, int src) {
  return __shfl(x, src, 64);
}

// Per-wave LDS hash set for the staged bucket: kWaveSlots int32 slots in
// buckets of 4, two-choice placement (the emptier of two buckets from one
// multiplicative hash; both full: the first bucket after the second with
// room), at most half full for a list of kHubMinDegree elements.  Empty slots
// hold -1.  Slots of a bucket fill in order and are never freed while the set
// is in use, so a bucket that is not full at probe time was not full when any
// element was placed.
constexpr int kWaveSlots = 2 * kHubMinDegree;
constexpr int kWaveBuckets = kWaveSlots / 4;
constexpr int kWaveBucketBits = 8;
static_assert(kWaveBuckets == 1 << kWaveBucketBits, "bucket index width");

__device__ __forceinline__ void wave_buckets(int32_t x, uint32_t& b1, uint32_t& b2) {
  const uint32_t h = (uint32_t)x * 0x9E3779B1u;
  b1 = h >> (32 - kWaveBucketBits);
  b2 = ((h >> (32 - 2 * kWaveBucketBits)) ^ h) & (kWaveBuckets - 1);
}

__device__ __forceinline__ int wave_bucket_free(int4 q) {
  return (q.x == -1) + (q.y == -1) + (q.z == -1) + (q.w == -1);
}

__device__ __forceinline__ bool wave_bucket_put(int32_t* T, uint32_t b, int32_t x) {
  int32_t* slot = T + 4 * b;
  if (atomicCAS(slot + 0, -1, x) == -1) return true;
  if (atomicCAS(slot + 1, -1, x) == -1) return true;
  if (atomicCAS(slot + 2, -1, x) == -1) return true;
  return atomicCAS(slot + 3, -1, x) == -1;
}

__device__ __forceinline__ void wave_insert(int32_t* T, int32_t x) {
  uint32_t b1, b2;
  wave_buckets(x, b1, b2);
  const int4* T4 = reinterpret_cast<const int4*>(T);
  const bool second_first = wave_bucket_free(T4[b2]) > wave_bucket_free(T4[b1]);
  if (wave_bucket_put(T, second_first ? b2 : b1, x)) return;
  if (wave_bucket_put(T, second_first ? b1 : b2, x)) return;
  uint32_t b = (b2 + 1) & (kWaveBuckets - 1);
  while (!wave_bucket_put(T, b, x)) b = (b + 1) & (kWaveBuckets - 1);
}

__device__ __forceinline__ bool wave_has(const int32_t* T, int32_t x) {
  uint32_t b1, b2;
  wave_buckets(x, b1, b2);
  const int4* T4 = reinterpret_cast<const int4*>(T);
  const int4 q1 = T4[b1], q2 = T4[b2];
  const auto has = [](int4 q, int32_t y) { return q.x == y || q.y == y || q.z == y || q.w == y; };
  if (has(q1, x) || has(q2, x)) return true;
  if ((q1.w | q2.w) < 0) return false;  // one of the two buckets has room
  uint32_t b = (b2 + 1) & (kWaveBuckets - 1);
  while (true) {
    const int4 q = T4[b];
    if (has(q, x)) return true;
    if (q.w == -1) return false;
    b = (b + 1) & (kWaveBuckets - 1);
  }
}

// Staged-bucket intersection: the whole wave (64 lanes) probes the smaller
// list, one element per lane per step, against the wave's hash set of the
// larger list; the next step's elements are loaded while this one is probed.
// Early exit as in group_intersect.
__device__ __forceinline__ int wave_intersect(const int32_t* Arow, int64_t du, const int32_t* T,
                                              int32_t need_open, bool exact, int lane, int32_t& cnt,
                                              int64_t& consumed) {
  cnt = 0;
  consumed = 0;
  int32_t xn = (lane < du) ? Arow[lane] : -1;
  for (int64_t t = 0; t < du; t += 64) {
    const int32_t x = xn;
    const int64_t nx = t + 64 + lane;
    xn = (nx < du) ? Arow[nx] : -1;
    const bool f = (t + lane < du) && wave_has(T, x);
    cnt += __popcll(__ballot(f));
    const int64_t take = du - t < 64 ? du - t : 64;
    consumed += take;
    if (!exact) {
      if (cnt >= need_open) return 2;
      if (cnt + (du - (t + take)) < need_open) return 3;
    }
  }
  return 1;
}

// Edge counters of one pass, summed per lane and flushed once.
struct PassCounts {
  unsigned long long eval = 0, bound = 0, probe = 0;
};

// Every lane classifies one edge of a chunk of 64 and applies the edges that
// need no intersection; the edges that do are then taken 64/G at a time, one
// per group of G lanes (the edge's fields are broadcast from the lane that
// classified it).  Buckets 0-4 use G >= d_s (one tile); G = 64 also serves the
// last bucket when it runs without the LDS-hash kernel.
// STAGE (buckets 4 and 5, G = 64): for an edge whose larger side has at most
// kHubMinDegree neighbours, the wave loads nbr(v) into its own LDS hash set
// (T, kWaveSlots int32), and every element of the smaller list is one hash
// probe; edges with a larger side above that search nbr(v) in global memory.
// Wave `wave` of `nwaves` takes the chunks wave, wave + nwaves, ... of
// [begin, end).
template <int MODE, int G, bool STAGE>
__device__ __forceinline__ void group_edges(const EdgeArgs& A, int64_t begin, int64_t end, int64_t wave,
                                            int64_t nwaves, int32_t* T, PassCounts& pc) {
  static_assert(!STAGE || G == 64, "staging is per wave");
  constexpr int kGroups = 64 / G;
  const int lane = threadIdx.x & 63;
  const int grp = lane / G, sub = lane & (G - 1), gbase = lane & ~(G - 1);
  const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
  const bool exact = (MODE == MODE_COUNTS) || !A.pruning;
  int32_t staged_v = -1;  // STAGE: the vertex whose list the wave's LDS slot holds
  for (int64_t base = begin + wave * 64; base < end; base += nwaves * 64) {
    const int64_t e = base + lane;
    EdgeView ev;
    unsigned long long nb = 0;
    classify<MODE>(A, e, e < end, ev, nb);
    pc.bound += nb;
    bool surv = false;
    if (ev.work == 2) {
      apply<MODE>(A, e, ev, true, 0);
    } else if (ev.work == 3) {
      if (MODE != MODE_ATTACH) apply<MODE>(A, e, ev, false, 0);
    } else if (ev.work == 1) {
      if (!exact && ev.need - 2 <= 0) {
        ++pc.eval;
        apply<MODE>(A, e, ev, true, 0);
      } else {
        surv = true;
      }
    }
    uint64_t pending = __ballot(surv);
    while (pending) {
      uint64_t mk = pending;
      for (int j = 0; j < grp; ++j) mk &= mk - 1;
      const bool act = mk != 0;
      const int src = act ? __ffsll((unsigned long long)mk) - 1 : lane;
      EdgeView w;
      w.u = shfl_t(ev.u, src);
      w.v = shfl_t(ev.v, src);
      w.bu = shfl_t(ev.bu, src);
      w.bv = shfl_t(ev.bv, src);
      w.du = shfl_t(ev.du, src);
      w.dv = shfl_t(ev.dv, src);
      w.need = shfl_t(ev.need, src);
      w.core_side = shfl_t(ev.core_side, src);
      w.other = shfl_t(ev.other, src);
      w.core_label = shfl_t(ev.core_label, src);
      w.mu = shfl_t(ev.mu, src);
      w.open_u = (uint8_t)shfl_t((int32_t)ev.open_u, src);
      w.open_v = (uint8_t)shfl_t((int32_t)ev.open_v, src);
      const int64_t we = shfl_t(e, src);
      if (act) {
        int32_t cnt;
        int64_t consumed;
        int verdict;
        if (STAGE && w.dv <= kHubMinDegree) {  // uniform over the wave (G = 64)
          // edges are grouped by the larger side, so consecutive edges of a
          // wave mostly share it and its set is built once
          if (w.v != staged_v) {
            // the wave's probes of the previous edge's set come first
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int i = lane; i < kWaveBuckets; i += 64)
              reinterpret_cast<int4*>(T)[i] = make_int4(-1, -1, -1, -1);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // two loads in flight per lane, then their inserts: holding all
            // eight of a 512-element list spilled registers in the fused
            // batch kernel
            for (int k0 = 0; k0 < kHubMinDegree / 64 && k0 * 64 < w.dv; k0 += 2) {
              int32_t y[2];
#pragma unroll
              for (int k = 0; k < 2; ++k)
                y[k] = ((k0 + k) * 64 + lane < w.dv) ? A.ci[w.bv + (k0 + k) * 64 + lane] : -1;
#pragma unroll
              for (int k = 0; k < 2; ++k)
                if (y[k] >= 0) wave_insert(T, y[k]);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            staged_v = w.v;
          }
          verdict = wave_intersect(A.ci + w.bu, w.du, T, w.need - 2, exact, lane, cnt, consumed);
        } else {
          verdict = group_intersect<G>(A.ci + w.bu, w.du, A.ci + w.bv, w.dv, w.need - 2, exact, sub, gbase,
                                       gmask, cnt, consumed);
        }
        if (sub == 0) {
          ++pc.eval;
          pc.probe += (unsigned long long)consumed;
          const bool sim = verdict == 2 ? true : verdict == 3 ? false : (cnt + 2 >= w.need);
          apply<MODE>(A, we, w, MODE == MODE_COUNTS ? false : sim, cnt + 2);
        }
      }
      for (int j = 0; j < kGroups && pending; ++j) pending &= pending - 1;
    }
  }
}

// One bucket's pass over [A.e_begin, A.e_end), grid-stride over 64-edge chunks.
template <int MODE, int G, bool STAGE = false>
__global__ __launch_bounds__(kBlock) void k_group(EdgeArgs A) {
  if ((MODE == MODE_MERGE || MODE == MODE_ATTACH) && A.ncores && *A.ncores == 0) return;  // no cluster
  __shared__ __align__(16) int32_t stage[STAGE ? (kBlock / 64) * kWaveSlots : 1];
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  PassCounts pc;
  group_edges<MODE, G, STAGE>(A, A.e_begin, A.e_end, wave, nwaves, stage + (STAGE ? (threadIdx.x >> 6) * kWaveSlots : 0),
                              pc);
  flush_stats_block<kBlock / 64>(A, MODE, pc.eval, pc.bound, pc.probe);
}

// Last bucket (d_u > 64), grouped by the larger side v.  A job is up to
// kHubJobEdges consecutive in-edges (u_i, v) of one v; blocks take jobs from a
// device counter, heaviest v first.
//   Phase A: every thread classifies in-edges; those needing an intersection
//            are appended to the job's slice of the worklist.
//   Phase B: the survivors are processed kHubBatch at a time.  For each batch
//            the block loads nbr(v) into LDS, window by window, and groups of
//            kHubGroup lanes stream the smaller lists nbr(u_i) of the
//            survivors through it.  A window is a run of consecutive elements
//            of nbr(v) and stands for the ids from its first element up to
//            the first element of the next window, so each survivor keeps its
//            read position and next element in LDS, nbr(u_i) is read once in
//            total, and windows below every survivor's next element are not
//            built at all.  Where kHubBitmapBits ids from the window's first
//            element on hold at least kHubBitmapMin elements of nbr(v), the
//            window is all of them, kept as a bitmap (a probe is one bit
//            test); otherwise it is the next kHubWindow elements, kept as a
//            hash set, cut short where the longest suffix of nbr(v) that one
//            bitmap covers begins.  A survivor stops as soon as its verdict
//            is certain.  The windows that the first batch of a job finds are
//            kept in LDS for its later batches.  The rows may be given with
//            vertices renamed by degree rank (A.hci), which packs most of a
//            long row into the last bitmap window.
// LDS hash set: kHubSlots int32 slots viewed as buckets of 4 (one 16-byte
// LDS load each).  Two-choice placement: every element has two buckets, both
// derived from one multiplicative hash, and goes to the emptier one; only when
// both are full does it go on to the first bucket after its second one that
// has room.  A probe reads both buckets at once; it has to look further only
// when both are full and neither holds the element, which two-choice placement
// at half load makes rare.  A window of at most kHubSparseMax elements places
// first fit instead (first bucket, else second, else onwards), and a probe
// reads the second bucket only when the first is full without the element.
// Slots of a bucket fill in order (each insert takes its first free slot), so
// a bucket is full exactly when its last slot is set, and slots are never
// freed while a table is in use: a bucket that is not full at probe time was
// not full when any later element was placed.
constexpr int kHubBucketBits = kHubLog2Slots - 2;
constexpr int kHubBuckets = 1 << kHubBucketBits;
static_assert(2 * kHubBucketBits <= 32, "both bucket indices come from one 32-bit product");
__device__ __forceinline__ void hub_buckets(int32_t x, uint32_t& b1, uint32_t& b2) {
  const uint32_t h = (uint32_t)x * 0x9E3779B1u;
  b1 = h >> (32 - kHubBucketBits);
  b2 = ((h >> (32 - 2 * kHubBucketBits)) ^ h) & (kHubBuckets - 1);
}

__device__ __forceinline__ int bucket_free(int4 q) {
  return (q.x == -1) + (q.y == -1) + (q.z == -1) + (q.w == -1);
}

__device__ __forceinline__ bool bucket_put(int32_t* table, uint32_t b, int32_t x) {
  int32_t* slot = table + 4 * b;
  if (atomicCAS(slot + 0, -1, x) == -1) return true;
  if (atomicCAS(slot + 1, -1, x) == -1) return true;
  if (atomicCAS(slot + 2, -1, x) == -1) return true;
  return atomicCAS(slot + 3, -1, x) == -1;
}

__device__ __forceinline__ void hub_insert(int32_t* table, int32_t x) {
  uint32_t b1, b2;
  hub_buckets(x, b1, b2);
  const int4* T = reinterpret_cast<const int4*>(table);
  // the loads only steer the choice; the CAS loops decide where x lands
  const bool second_first = bucket_free(T[b2]) > bucket_free(T[b1]);
  if (bucket_put(table, second_first ? b2 : b1, x)) return;
  if (bucket_put(table, second_first ? b1 : b2, x)) return;
  uint32_t b = (b2 + 1) & (kHubBuckets - 1);
  while (!bucket_put(table, b, x)) b = (b + 1) & (kHubBuckets - 1);
}

// First-fit placement for a sparse set (at most kHubSparseMax elements, a
// quarter of the slots): the first bucket if it has room, else the second,
// else the first bucket after the second with room.  A probe then needs the
// second bucket only when the first is full, which at this load is rare.
__device__ __forceinline__ void hub_insert_sparse(int32_t* table, int32_t x) {
  uint32_t b1, b2;
  hub_buckets(x, b1, b2);
  if (bucket_put(table, b1, x)) return;
  if (bucket_put(table, b2, x)) return;
  uint32_t b = (b2 + 1) & (kHubBuckets - 1);
  while (!bucket_put(table, b, x)) b = (b + 1) & (kHubBuckets - 1);
}

// Stands for "no element" in a probe: matches no slot (empty slots hold -1).
constexpr int32_t kHubNone = -2;

__device__ __forceinline__ bool bucket_has(int4 q, int32_t x) {
  return q.x == x || q.y == x || q.z == x || q.w == x;
}

// Rest of a probe whose two buckets were both full.
__device__ __noinline__ bool hub_probe_tail(const int4* T, int32_t x) {
  uint32_t b1, b2;
  hub_buckets(x, b1, b2);
  uint32_t b = (b2 + 1) & (kHubBuckets - 1);
  while (true) {
    const int4 q = T[b];
    if (bucket_has(q, x)) return true;
    if (q.w == -1) return false;
    b = (b + 1) & (kHubBuckets - 1);
  }
}

// Exclusive prefix sum of one int64 per thread over a block of kHubBlock
// threads; returns the sum of all values through *total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t* wsum, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t incl = x;
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int w = 0; w < kHubBlock / 64; ++w) {
    const int64_t t = wsum[w];
    off += (w < wave) ? t : 0;
    tot += t;
  }
  *total = tot;
  return off + incl - x;
}

// Kinds of window: 0 hash set (two-choice), 1 bitmap, 2 sparse hash set
// (first fit).
template <int K>
struct KindTag {
  static constexpr int value = K;
};

// First index in (lo, hi) whose value is at least T in the ascending array
// row, or hi if there is none; row[lo] < T.  The whole block searches
// together, one load per thread per round, each round narrowing the range
// kHubBlock-fold.  Every thread must call it with the same arguments.
__device__ __forceinline__ int64_t block_find(const int32_t* row, int64_t lo, int64_t hi, int64_t T,
                                              int32_t* s_first) {
  while (hi - lo > 1) {
    const int64_t stride = (hi - lo - 1 + kHubBlock - 1) / kHubBlock;
    if (threadIdx.x == 0) *s_first = kHubBlock;
    __syncthreads();
    const int64_t p = lo + (int64_t)(threadIdx.x + 1) * stride;
    if (p < hi && (int64_t)row[p] >= T) atomicMin(s_first, (int32_t)threadIdx.x);
    __syncthreads();
    const int32_t t = *s_first;
    __syncthreads();  // s_first is reset at the top of the next round
    if (t < kHubBlock) {
      hi = lo + (int64_t)(t + 1) * stride;
      lo = lo + (int64_t)t * stride;
    } else {
      lo = lo + ((hi - 1 - lo) / stride) * stride;  // the last probe below hi
    }
  }
  return hi;
}

template <int MODE>
__global__ __launch_bounds__(kHubBlock)
__attribute__((amdgpu_waves_per_eu(kHubWavesPerSimd, kHubWavesPerSimd)))  // kHubBlocksPerCU blocks fit
void k_hub(EdgeArgs A, const HubJob* jobs, int64_t njobs, unsigned long long* counter, int32_t* wl) {
  constexpr int kGroups = kHubBlock / kHubGroup;
  constexpr int kStep = kHubGroup * kHubUnroll;  // elements per group step
  // hash set, or bitmap plus one zero word that out-of-range probes read
  __shared__ __align__(16) int32_t table[kHubSlots + 4];
  __shared__ int64_t q_bu[kHubBatch];
  __shared__ unsigned long long q_acc[kHubBatch];  // (consumed in this window) << 32 | hits
  __shared__ int32_t q_du[kHubBatch];
  __shared__ int32_t q_need[kHubBatch];   // open common neighbours needed
  __shared__ int32_t q_cnt[kHubBatch];    // open common neighbours found before this window
  __shared__ int32_t q_pos[kHubBatch];    // elements of nbr(u) consumed before this window
  __shared__ int32_t q_end[kHubBatch];    // end of this window's part of nbr(u)
  __shared__ int32_t q_next[kHubBatch];   // next unread element of nbr(u) (INT_MAX at the end)
  __shared__ int32_t q_first[kHubBatch + 1];  // index of the survivor's first chunk among first chunks
  __shared__ int32_t q_rest[kHubBatch + 1];   // index of its second chunk among the later chunks
  __shared__ uint8_t q_st[kHubBatch];     // 0 skipped, 1 active, 2 similar, 3 dissimilar
  __shared__ int64_t wsum[kHubBlock / 64];
  __shared__ int64_t s_job;
  __shared__ int32_t s_n, s_min, s_chunk, s_first;
  // the job's windows found so far (every batch of a job has the same ones):
  // window k is elements s_wend[k - 1] .. s_wend[k] - 1 of nbr(v) (s_wend[-1] = 0)
  __shared__ int64_t s_wend[kHubMaxWindows];
  __shared__ uint8_t s_wbitmap[kHubMaxWindows];
  // cores pass: similar verdicts of this job's edges on the common larger side
  // v, added to v's lower bound once per job (all of a job's edges would
  // otherwise update the same counter one by one); v's degree is above
  // kUpperMaxDegree, so its upper bound is not kept
  __shared__ int32_t s_vsim;
  const int tid = threadIdx.x;
  const int sub = tid & (kHubGroup - 1);  // lane within its group
  const bool exact = (MODE == MODE_COUNTS) || !A.pruning;
  const int4* T4 = reinterpret_cast<const int4*>(table);
  unsigned long long n_eval = 0, n_bound = 0, n_probe = 0;
  uint32_t n_split = 0;
  if ((MODE == MODE_MERGE || MODE == MODE_ATTACH) && A.ncores && *A.ncores == 0) return;  // no cluster
  while (true) {
    if (tid == 0) {
      s_job = (int64_t)atomicAdd(counter, 1ull);
      s_n = 0;
      s_vsim = 0;
    }
    __syncthreads();
    const int64_t job = s_job;
    if (job >= njobs) break;
    const HubJob J = jobs[job];
    const int64_t region = J.begin - A.e_begin;
    // Phase A: each thread classifies kHubPerThread in-edges, all of their
    // loads first (classification only reads), then acts on them.
    for (int32_t base = 0; base < J.count; base += kHubBlock * kHubPerThread) {
      EdgeView ev[kHubPerThread];
      unsigned long long nb[kHubPerThread];
#pragma unroll
      for (int i = 0; i < kHubPerThread; ++i) {
        const int32_t off = base + i * kHubBlock + tid;
        nb[i] = 0;
        classify<MODE>(A, J.begin + off, off < J.count, ev[i], nb[i]);
      }
      // edges decided without an intersection: dissimilar by the degree
      // bound (3), similar because two closed neighbours suffice, or already
      // known similar (2, attach pass)
      bool act[kHubPerThread], sim[kHubPerThread];
#pragma unroll
      for (int i = 0; i < kHubPerThread; ++i) {
        n_bound += nb[i];
        const bool trivial = ev[i].work == 1 && !exact && ev[i].need - 2 <= 0;
        act[i] = ev[i].work == 2 || (ev[i].work == 3 && MODE != MODE_ATTACH) || trivial;
        sim[i] = ev[i].work == 2 || trivial;
        n_eval += trivial ? 1 : 0;
      }
      if (MODE == MODE_CORES) {
        int32_t cu[kHubPerThread], cv[kHubPerThread], vsim = 0;
#pragma unroll
        for (int i = 0; i < kHubPerThread; ++i)
          if (act[i]) cores_count(A, ev[i], sim[i], ev[i].open_u, false, cu[i], cv[i]);
#pragma unroll
        for (int i = 0; i < kHubPerThread; ++i) {
          if (!act[i]) continue;
          A.state[J.begin + base + i * kHubBlock + tid] = sim[i] ? SIM_YES : SIM_NO;
          cores_roles(A, ev[i], sim[i], ev[i].open_u, false, cu[i], cv[i]);
          if (ev[i].open_v && sim[i]) ++vsim;
        }
        if (vsim) atomicAdd(&s_vsim, vsim);
      } else {
#pragma unroll
        for (int i = 0; i < kHubPerThread; ++i)
          if (act[i]) apply<MODE>(A, J.begin + base + i * kHubBlock + tid, ev[i], sim[i], 0);
      }
#pragma unroll
      for (int i = 0; i < kHubPerThread; ++i) {
        const int32_t off = base + i * kHubBlock + tid;
        if (ev[i].work == 1 && !act[i]) wl[region + atomicAdd(&s_n, 1)] = off;
      }
    }
    __syncthreads();
    const int32_t S = s_n;
    const int64_t bv = row_start(A, J.v);
    const int64_t dv = A.rp[J.v + 1] - A.rp[J.v];
    // v's windows as computed when the graph was created (the first
    // kHubMaxWindows of them); any further ones are found below as they come
    int32_t n_known = 0;  // windows of this job in s_wend / s_wbitmap
    if (S > 0 && J.wcnt > 0) {
      n_known = min(J.wcnt, kHubMaxWindows);
      for (int k = tid; k < n_known; k += kHubBlock) {
        const uint32_t w = A.wtab[J.wbeg + k];
        s_wend[k] = (int64_t)(w >> 1);
        s_wbitmap[k] = (uint8_t)(w & 1u);
      }
      __syncthreads();
    }
    // Start of the longest suffix of nbr(v) that one bitmap covers; when it
    // holds at least kHubBitmapMin elements, hash windows stop at it, so that
    // the suffix becomes a single bitmap window.  (Needed only to find windows
    // here.)
    int64_t wsuf = dv;
    if (S > 0 && dv >= kHubBitmapMin && (J.wcnt <= 0 || J.wcnt > kHubMaxWindows)) {
      const int64_t T = (int64_t)A.hci[bv + dv - 1] - kHubBitmapBits + 1;
      const int64_t ws = ((int64_t)A.hci[bv] >= T) ? 0 : block_find(A.hci + bv, 0, dv, T, &s_first);
      if (dv - ws >= kHubBitmapMin) wsuf = ws;
    }
    // Phase B
    for (int32_t b0 = 0; b0 < S; b0 += kHubBatch) {
      const int32_t nbatch = (S - b0 < kHubBatch) ? S - b0 : kHubBatch;
      EdgeView ev;
      int64_t e = 0;
      if (tid < nbatch) {
        e = J.begin + wl[region + b0 + tid];
        const bool keep = load_survivor<MODE>(A, e, ev);
        q_bu[tid] = ev.bu;
        q_du[tid] = (int32_t)ev.du;
        q_need[tid] = ev.need - 2;
        q_cnt[tid] = 0;
        q_pos[tid] = 0;
        q_next[tid] = (keep && ev.du > 0) ? A.hci[ev.bu] : INT_MAX;
        q_st[tid] = keep ? 1 : 0;
      }
      int32_t wi = 0;
      for (int64_t w0 = 0, w1 = 0; w0 < dv; w0 = w1, ++wi) {
        // This window is a bitmap of the ids L .. L + kHubBitmapBits - 1 if
        // that range holds at least kHubBitmapMin elements of nbr(v) from w0
        // on, else a hash set of the next kHubWindow elements (at most up to
        // the bitmap suffix).  A window an earlier batch of the job found is
        // taken from LDS.
        const int32_t L = A.hci[bv + w0];
        bool bitmap = false;
        if (wi < n_known) {
          w1 = s_wend[wi];
          bitmap = s_wbitmap[wi] != 0;
        } else {
          w1 = (dv - w0 > kHubWindow) ? w0 + kHubWindow : dv;
          if (w0 < wsuf && w1 > wsuf) w1 = wsuf;
          if (dv - w0 >= kHubBitmapMin) {
            const int64_t wb = block_find(A.hci + bv, w0, dv, (int64_t)L + kHubBitmapBits, &s_first);
            if (wb - w0 >= kHubBitmapMin) {
              bitmap = true;
              w1 = wb;
            }
          }
          if (wi < kHubMaxWindows) {
            // every thread found the same window; the first records it (read
            // by the next batch, after the barriers below)
            if (tid == 0) {
              s_wend[wi] = w1;
              s_wbitmap[wi] = bitmap ? 1 : 0;
            }
            n_known = wi + 1;
          }
        }
        const int32_t hi = (w1 < dv) ? A.hci[bv + w1] : INT_MAX;
        const bool sparse = !bitmap && w1 - w0 <= kHubSparseMax;
        if (tid == 0) {
          s_min = INT_MAX;
          s_chunk = 0;
        }
        __syncthreads();
        if (tid < nbatch && q_st[tid] == 1) atomicMin(&s_min, q_next[tid]);
        __syncthreads();
        const int32_t mn = s_min;
        __syncthreads();           // s_min is reset at the top of the next window
        if (mn == INT_MAX) break;  // every survivor decided or fully read
        if (mn >= hi) continue;    // no survivor has an element in this window
        if (bitmap) {
          for (int k = tid; k < kHubSlots + 4; k += kHubBlock) table[k] = 0;
        } else {
          for (int k = tid; k < kHubSlots; k += kHubBlock) table[k] = -1;
        }
        // This window's part of every active survivor, cut into chunks of
        // kHubChunk.  Chunks are handed out first-chunk-of-every-survivor
        // first, then the remaining chunks survivor by survivor, so that most
        // verdicts (usually reached inside the first chunk) come before any
        // group starts on a survivor's later chunks.  Per survivor, packed as
        // (1 << 32) | (chunks - 1) so that one scan yields both offsets.
        int64_t packed = 0;
        if (tid < nbatch) {
          q_acc[tid] = 0;
          if (q_st[tid] == 1 && q_next[tid] < hi) {
            const int32_t* Arow = A.hci + q_bu[tid];
            int32_t lo = q_pos[tid], hi2 = q_du[tid];
            if (hi != INT_MAX && A.hsamp) {
              // The part ends at the first 128-byte line past the survivor's
              // position whose first element is >= hi, found in the line
              // samples (an array of nnz/32 ids, read through the caches)
              // rather than in the row itself, whose lines would be fetched
              // here and again, after eviction, by the chunks.  The chunks
              // then also read up to 31 elements of the part's last line that
              // are >= hi, and skip them by value.
              const int64_t bu = q_bu[tid];
              const int64_t kb = (bu + hi2 - 1) >> 5;  // the row's last line
              // lines in (a0, a] start below hi; line b starts at or above it
              // (b = kb + 1: none does), galloping from the position's line a0
              int64_t a = (bu + lo) >> 5, step = 1;
              while (a + step <= kb && A.hsamp[a + step] < hi) {
                a += step;
                step *= 2;
              }
              int64_t b = (a + step <= kb) ? a + step : kb + 1;
              while (b - a > 1) {
                const int64_t mid = (a + b) >> 1;
                if (A.hsamp[mid] < hi) a = mid;
                else b = mid;
              }
              q_end[tid] = (b <= kb) ? (int32_t)((b << 5) - bu) : hi2;
            } else if (hi != INT_MAX) {
              // first element >= hi, found by galloping from the survivor's
              // position (Arow[lo] < hi): the probes fall on lines of this
              // window's part, which the chunks read next, and at most one past it
              int64_t a = lo, b = hi2, step = 32;
              while (a + step < b && Arow[a + step] < hi) {
                a += step;
                step *= 2;
              }
              if (a + step < b) b = a + step;
              ++a;  // Arow[a - 1] < hi
              while (a < b) {
                const int64_t mid = (a + b) >> 1;
                if (Arow[mid] < hi) a = mid + 1;
                else b = mid;
              }
              q_end[tid] = (int32_t)a;
            } else {
              q_end[tid] = hi2;
            }
            packed = (1ll << 32) | (int64_t)((q_end[tid] - q_pos[tid] - 1) / kHubChunk);
          }
        }
        int64_t total;
        const int64_t off = block_exclusive_scan(packed, wsum, &total);
        const int32_t n_first = (int32_t)(total >> 32);
        const int32_t n_rest = (int32_t)(total & 0xffffffffll);
        const int32_t n_chunks = n_first + n_rest;
        if (tid < nbatch) {
          q_first[tid] = (int32_t)(off >> 32);
          q_rest[tid] = (int32_t)(off & 0xffffffffll);
        }
        if (tid == 0) {
          q_first[nbatch] = n_first;
          q_rest[nbatch] = n_rest;
        }
        __syncthreads();
        // this window of nbr(v) into the table, kHubInsertBatch loads in flight per thread
        for (int64_t k0 = w0 + tid; k0 < w1; k0 += (int64_t)kHubBlock * kHubInsertBatch) {
          int32_t y[kHubInsertBatch];
#pragma unroll
          for (int i = 0; i < kHubInsertBatch; ++i) {
            const int64_t k = k0 + (int64_t)i * kHubBlock;
            y[i] = (k < w1) ? A.hci[bv + k] : kHubNone;
          }
#pragma unroll
          for (int i = 0; i < kHubInsertBatch; ++i) {
            if (y[i] == kHubNone) continue;
            if (bitmap) {
              const uint32_t off = (uint32_t)y[i] - (uint32_t)L;
              atomicOr(reinterpret_cast<uint32_t*>(table) + (off >> 5), 1u << (off & 31));
            } else if (sparse) {
              hub_insert_sparse(table, y[i]);
            } else {
              hub_insert(table, y[i]);
            }
          }
        }
        __syncthreads();
        // Groups of kHubGroup lanes take chunks until none are left.  The loop
        // body branches on nothing that differs between the lanes of a group
        // (the group's first lane alone adds, through a select, not a branch):
        // a branch on the lane index would let the compiler run the group's
        // lanes around the loop separately, and the shuffles need the whole
        // group together.
        // the chunk loop, compiled once per kind of window
        auto chunk_loop = [&](auto kind) {
        constexpr int kKind = decltype(kind)::value;
        while (true) {
          // every lane adds 1, so a group's lanes receive kHubGroup consecutive
          // values starting at a multiple of kHubGroup: value / kHubGroup is
          // the group's chunk (a uniform addend keeps this a single atomic per
          // wave and avoids any branch on the lane index)
          const int32_t c = atomicAdd(&s_chunk, 1) / kHubGroup;
          // every lane of a group must have the same chunk (the totals below
          // are read back for the whole group); each lane compares its chunk
          // with its left neighbour's (one DPP row shift, no branch), and a
          // lane whose neighbour in the group differs is counted.  All seven
          // neighbour pairs equal means the whole group agrees; the parity
          // tests require the count to stay zero.
          static_assert(kHubGroup <= 16, "a group lies in one DPP row");
          const int32_t left = __builtin_amdgcn_update_dpp(c, c, 0x111 /* row_shr:1 */, 0xF, 0xF, false);
          n_split += ((tid & (kHubGroup - 1)) != 0 && left != c) ? 1u : 0u;
          if (c >= n_chunks) break;
          const bool first = c < n_first;
          const int32_t cc = first ? c : c - n_first;
          const int32_t* pre = first ? q_first : q_rest;
          int32_t lo = 0, hi2 = nbatch;  // survivor k: pre[k] <= cc < pre[k + 1]
          while (hi2 - lo > 1) {
            const int32_t mid = (lo + hi2) >> 1;
            if (pre[mid] <= cc) lo = mid;
            else hi2 = mid;
          }
          const int k = lo;
          if (q_st[k] != 1) continue;  // already decided
          const int32_t* Arow = A.hci + q_bu[k];
          const int32_t base = q_pos[k], du = q_du[k], need = q_need[k], cnt0 = q_cnt[k];
          const int32_t cs = first ? base : base + (1 + cc - pre[k]) * kHubChunk;
          const int32_t ce = (q_end[k] - cs < kHubChunk) ? q_end[k] : cs + kHubChunk;
          // Each lane counts its own elements and hits and adds them to the
          // survivor's running totals itself, so no step needs a reduction
          // across the group.
          uint32_t my_hits = 0, my_seen = 0;
          // elements of the next step are loaded while this one is probed
          // (the last step loads its own elements again, from lines already
          // fetched, rather than the next ones past the chunk); loads may run
          // up to one step past the chunk (col_idx is padded), values at or
          // beyond ce are ignored
          const int32_t* P = Arow + cs + sub;
          int32_t xn[kHubUnroll];
#pragma unroll
          for (int j = 0; j < kHubUnroll; ++j) xn[j] = P[j * kHubGroup];
          for (int32_t p = cs; p < ce; p += kStep) {
            P = (p + kStep < ce) ? P + kStep : P;
            const int32_t left = ce - p - sub;  // this lane's elements from here on
            int32_t x[kHubUnroll];
            uint32_t step_seen = 0;  // elements of this window's part (below hi)
#pragma unroll
            for (int j = 0; j < kHubUnroll; ++j) {
              x[j] = (j * kHubGroup < left) ? xn[j] : kHubNone;
              xn[j] = P[j * kHubGroup];
              step_seen += ((uint32_t)x[j] < (uint32_t)hi) ? 1u : 0u;  // kHubNone is above every id
            }
            uint32_t step_hits = 0;
            if constexpr (kKind == 2) {
              // first buckets only; the second one (and beyond) just for
              // elements whose first bucket is full without them
              int4 q[kHubUnroll];
              uint32_t b2[kHubUnroll];
#pragma unroll
              for (int j = 0; j < kHubUnroll; ++j) {
                uint32_t b1;
                hub_buckets(x[j], b1, b2[j]);
                q[j] = T4[b1];
              }
#pragma unroll
              for (int j = 0; j < kHubUnroll; ++j) {
                const uint32_t xj = (uint32_t)x[j];
                const uint32_t dj = min(min((uint32_t)q[j].x ^ xj, (uint32_t)q[j].y ^ xj),
                                        min((uint32_t)q[j].z ^ xj, (uint32_t)q[j].w ^ xj));
                bool h = dj == 0u;
                if (!h && q[j].w >= 0) {  // first bucket full without x
                  const int4 r = T4[b2[j]];
                  h = bucket_has(r, x[j]);
                  if (!h && r.w >= 0) h = hub_probe_tail(T4, x[j]);
                }
                step_hits += h ? 1u : 0u;
              }
            } else if constexpr (kKind == 1) {
              // ids outside L .. L + kHubBitmapBits - 1 (kHubNone included)
              // read the zero word just past the bitmap
              const uint32_t* bm = reinterpret_cast<const uint32_t*>(table);
#pragma unroll
              for (int j = 0; j < kHubUnroll; ++j) {
                const uint32_t off = min((uint32_t)x[j] - (uint32_t)L, (uint32_t)kHubBitmapBits);
                step_hits += (bm[off >> 5] >> (off & 31)) & 1u;
              }
            } else {
            // first buckets of all elements, then second buckets, in the same
            // registers; slot compares give per-lane bits, which combine on the
            // scalar unit
            int4 q[kHubUnroll];
            uint32_t b2[kHubUnroll];
            int32_t w1[kHubUnroll];
            bool found[kHubUnroll];
#pragma unroll
            for (int j = 0; j < kHubUnroll; ++j) {
              uint32_t b1;
              hub_buckets(x[j], b1, b2[j]);
              q[j] = T4[b1];
            }
#pragma unroll
            for (int j = 0; j < kHubUnroll; ++j) {
              const int32_t xj = x[j];
              found[j] = (q[j].x == xj) | (q[j].y == xj) | (q[j].z == xj) | (q[j].w == xj);
              w1[j] = q[j].w;
            }
#pragma unroll
            for (int j = 0; j < kHubUnroll; ++j) q[j] = T4[b2[j]];
            int32_t both_full = -1;  // >= 0 once some element had both buckets full
#pragma unroll
            for (int j = 0; j < kHubUnroll; ++j) {
              const int32_t xj = x[j];
              found[j] = found[j] | (q[j].x == xj) | (q[j].y == xj) | (q[j].z == xj) | (q[j].w == xj);
              step_hits += found[j] ? 1u : 0u;
              // a bucket is full when its last slot holds an id (>= 0); empty slots hold -1
              both_full = max(both_full, w1[j] | q[j].w);
            }
            if (__ballot(both_full >= 0)) {  // rare: both of some element's buckets full
#pragma unroll
              for (int j = 0; j < kHubUnroll; ++j)
                if (!found[j] && (w1[j] | q[j].w) >= 0) step_hits += hub_probe_tail(T4, x[j]) ? 1u : 0u;
            }
            }
            if (exact) {
              my_hits += step_hits;
              my_seen += step_seen;
            } else {
              // fold this step into the survivor's running totals and stop as
              // soon as its verdict is certain, or another group reached it;
              // the totals are read back by one load for the whole group, so
              // the verdict and the exit are the same on all of its lanes
              atomicAdd(&q_acc[k], ((unsigned long long)step_seen << 32) | step_hits);
              const unsigned long long now = q_acc[k];
              const int32_t cnt = cnt0 + (int32_t)(now & 0xffffffffu);
              const int32_t done = base + (int32_t)(now >> 32);
              const uint8_t verdict = cnt >= need ? 2 : (cnt + (du - done) < need) ? 3 : 0;
              if (verdict) {
                q_st[k] = verdict;  // the same value from every lane of the group
                break;
              }
              if (q_st[k] != 1) break;
            }
          }
          if (exact) atomicAdd(&q_acc[k], ((unsigned long long)my_seen << 32) | my_hits);
        }
        };
        if (bitmap) chunk_loop(KindTag<1>{});
        else if (sparse) chunk_loop(KindTag<2>{});
        else chunk_loop(KindTag<0>{});
        __syncthreads();
        if (tid < nbatch && q_st[tid] != 0 && q_next[tid] < hi) {
          // window finished for this survivor (or it was decided on the way)
          const unsigned long long a = q_acc[tid];
          const int32_t cnt = q_cnt[tid] + (int32_t)(a & 0xffffffffu);
          const int32_t pos = q_pos[tid] + (int32_t)(a >> 32);
          q_cnt[tid] = cnt;
          q_pos[tid] = pos;
          if (q_st[tid] == 1) {
            q_next[tid] = (pos < q_du[tid]) ? A.hci[q_bu[tid] + pos] : INT_MAX;
            if (!exact) {
              if (cnt >= q_need[tid]) q_st[tid] = 2;
              else if (cnt + (q_du[tid] - pos) < q_need[tid]) q_st[tid] = 3;
            }
          }
        }
        __syncthreads();
      }
      __syncthreads();
      if (tid < nbatch && q_st[tid] != 0) {
        const int32_t st = q_st[tid], cnt = q_cnt[tid];
        ++n_eval;
        n_probe += (unsigned long long)q_pos[tid];
        const bool sim = st == 2 ? true : st == 3 ? false : (cnt + 2 >= ev.need);
        if (MODE == MODE_CORES) {
          int32_t cu, cv;
          cores_count(A, ev, sim, ev.open_u, false, cu, cv);
          A.state[e] = sim ? SIM_YES : SIM_NO;
          cores_roles(A, ev, sim, ev.open_u, false, cu, cv);
          if (ev.open_v && sim) atomicAdd(&s_vsim, 1);
        } else {
          apply<MODE>(A, e, ev, MODE == MODE_COUNTS ? false : sim, cnt + 2);
        }
      }
      __syncthreads();
    }
    if (MODE == MODE_CORES && tid == 0 && s_vsim) {
      uint64_t gp, gq;
      int32_t vmu;
      graph_params(A, J.v, gp, gq, vmu);
      if (atomicAdd(A.lower + J.v, s_vsim) + s_vsim >= vmu) st_u8(A.role + J.v, ROLE_CORE);
    }
    __syncthreads();  // every thread is done with this job's shared values
  }
  const unsigned long long splits = wave_sum(n_split);
  if ((tid & 63) == 0 && splits) atomicAdd(A.stats + ST_GROUP_SPLIT, splits);
  flush_stats(A, MODE, n_eval, n_bound, n_probe);
}

__global__ void k_line_samples(int64_t nlines, const int32_t* rows, int32_t* samp) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; k < nlines; k += stride) samp[k] = rows[k << 5];
}

__global__ void k_edge_degrees(int64_t m, const int64_t* rp, const int2* edges, int2* deg) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < m; e += stride) {
    const int2 uv = edges[e];
    deg[e] = make_int2((int32_t)(rp[uv.x + 1] - rp[uv.x]), (int32_t)(rp[uv.y + 1] - rp[uv.y]));
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Plain streaming copy, 16 bytes per lane per step: the reference kernel against which hardware
// byte counters are scaled (every byte is read once and written once).
__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Plain streaming read, 16 bytes per lane per load and four independent loads
// per lane in flight, folded into one word per thread (written so that the
// reads are not removed): the achievable rate of a read-only stream, the
// ceiling for kernels that mostly read.
__global__ void k_read16(const uint4* __restrict__ src, int64_t n16, uint32_t* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n16; i += stride) {
    const uint4 v = src[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void k_init(int32_t n, const int64_t* rp, int32_t mu, const int32_t* gid, const int32_t* gmu,
                       int32_t* lower, int32_t* upper, uint8_t* role, int32_t* parent) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  if (gid) mu = gmu[gid[u]];
  const int64_t d = rp[u + 1] - rp[u];
  lower[u] = 1;                       // u itself is in N_eps[u]
  upper[u] = (int32_t)(d + 1);        // |N[u]|
  role[u] = (d + 1 < mu) ? ROLE_NONCORE : ROLE_UNK;  // Lemma 4.1 with no edge seen yet
  parent[u] = (int32_t)u;
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 16;
  for (; i < n; i += stride) {
    if (i + 16 <= n && ((uintptr_t)(p + i) & 15) == 0) {
      *(uint4*)(p + i) = make_uint4(v * 0x01010101u, v * 0x01010101u, v * 0x01010101u, v * 0x01010101u);
    } else {
      for (int64_t k = i; k < n && k < i + 16; ++k) p[k] = v;
    }
  }
}

__global__ void k_finalize(int32_t n, int32_t mu, const int32_t* gid, const int32_t* gmu, const int32_t* lower,
                           uint8_t* role, unsigned long long* ncores) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool core = false;
  if (u < n) {
    if (gid) mu = gmu[gid[u]];
    // A role still unknown here had every incident edge evaluated (an edge is
    // only deferred when both roles are known), so lower is |N_eps[u]| exactly.
    uint8_t r = role[u];
    if (r == ROLE_UNK) {
      r = lower[u] >= mu ? ROLE_CORE : ROLE_NONCORE;
      role[u] = r;
    }
    core = r == ROLE_CORE;
  }
  // cores counted so that the merge and attach passes can stop at once when there are none
  const unsigned long long c = __popcll(__ballot(core));
  if (ncores && (threadIdx.x & 63) == 0 && c) atomicAdd(ncores, c);
}

__global__ void k_hook(int64_t m, const int2* edges, const uint8_t* state, const uint8_t* role,
                       int32_t* parent) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < m; e += stride) {
    if (state[e] != SIM_YES) continue;
    const int2 uv = edges[e];
    if (role[uv.x] == ROLE_CORE && role[uv.y] == ROLE_CORE) uf_union(parent, uv.x, uv.y);
  }
}

__global__ void k_flatten(int32_t n, const uint8_t* role, int32_t* parent, int32_t* label) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  label[u] = role[u] == ROLE_CORE ? uf_find(parent, (int32_t)u) : INT_MAX;
}

// Def 2.7 (the classification step, Alg. 4, done per edge): an edge with one
// endpoint x in no cluster and the other in the cluster labelled L lets x
// record the first L it meets in first[x]; meeting a different L makes x a hub.
// A border's cluster is the label it was given.  first[] starts at -1.
__global__ void k_hub_outlier(int64_t m, const int2* edges, const int32_t* label, int32_t* first,
                              uint8_t* role) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < m; e += stride) {
    const int2 uv = edges[e];
    const int32_t lu = label[uv.x], lv = label[uv.y];
    if ((lu == INT_MAX) == (lv == INT_MAX)) continue;
    const int32_t x = (lu == INT_MAX) ? uv.x : uv.y;
    const int32_t L = (lu == INT_MAX) ? lv : lu;
    const int32_t seen = first[x];
    if (seen == L) continue;
    const int32_t old = (seen == -1) ? atomicCAS(first + x, -1, L) : seen;
    if (old != -1 && old != L) role[x] = ROLE_HUB;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Output roles: 1 core, 2 border, and for vertices in no cluster 0, or with
// split set 3 (hub) / 4 (outlier).
__global__ void k_output(int32_t n, const uint8_t* role, const int32_t* label, const int32_t* gid,
                         const int32_t* gbase, int32_t* out_labels, uint8_t* out_roles, int32_t split) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t l = label[u] - ((gid && label[u] != INT_MAX) ? gbase[gid[u]] : 0);  // batch: local ids
  if (role[u] == ROLE_CORE) {
    out_roles[u] = 1;
    out_labels[u] = l;
  } else if (l != INT_MAX) {
    out_roles[u] = 2;
    out_labels[u] = l;
  } else {
    out_roles[u] = split ? (role[u] == ROLE_HUB ? 3 : 4) : 0;
    out_labels[u] = -1;
  }
}


// ---------------------------------------------------------------------------
// Re-thresholding from cached closed counts (serving).  With c_e known for
// every edge, a query (eps, mu) needs no intersection: each edge is tested
// with (c q)^2 >= p^2 a b directly (c <= min(a, b) and q max(a, b) < 2^32 keep
// both sides below 2^64), cores come from exact counts, then the same hook /
// flatten / attach steps as the full run.
__global__ void k_rt_init(int32_t n, int32_t* lower, int32_t* parent) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  lower[u] = 1;
  parent[u] = (int32_t)u;
}

// |N[u]| |N[v]| of every oriented edge, computed once when a graph is added,
// so that a query streams it with the count instead of gathering row offsets.
__global__ void k_closed_products(int64_t m, const int2* edges, const int64_t* rp, uint64_t* ab) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < m; e += stride) {
    const int2 uv = edges[e];
    const uint64_t a = (uint64_t)(rp[uv.x + 1] - rp[uv.x]) + 1;
    const uint64_t b = (uint64_t)(rp[uv.y + 1] - rp[uv.y]) + 1;
    ab[e] = a * b;
  }
}

__global__ void k_rt_edges(int64_t m, const int2* edges, const int32_t* ecount, const uint64_t* ab,
                           uint64_t p, uint64_t q, uint8_t* state, int32_t* lower) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < m; e += stride) {
    const int2 uv = edges[e];
    const uint64_t cq = (uint64_t)ecount[e] * q;
    const bool sim = cq * cq >= (p * p) * ab[e];
    state[e] = sim ? SIM_YES : SIM_NO;
    if (sim) {
      atomicAdd(lower + uv.x, 1);
      atomicAdd(lower + uv.y, 1);
    }
  }
}

__global__ void k_rt_roles(int32_t n, int32_t mu, const int32_t* lower, uint8_t* role) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) role[u] = lower[u] >= mu ? ROLE_CORE : ROLE_NONCORE;
}

__global__ void k_rt_attach(int64_t m, const int2* edges, const uint8_t* state, const uint8_t* role,
                            int32_t* label) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; e < m; e += stride) {
    if (state[e] != SIM_YES) continue;
    const int2 uv = edges[e];
    const bool cu = role[uv.x] == ROLE_CORE, cv = role[uv.y] == ROLE_CORE;
    if (cu == cv) continue;
    if (cu) atomicMin(label + uv.y, label[uv.x]);
    else atomicMin(label + uv.x, label[uv.y]);
  }
}

// ---------------------------------------------------------------------------
// Batched clustering in one persistent launch.  Blocks take (graph, phase,
// tile) items: item slot k < init_items is the BP_INIT tile that init_prefix
// assigns to it; later slots are read from the queue, where the block that
// finished the last tile of a graph's phase wrote that graph's next phase.
// remaining[g] counts the unfinished tiles of graph g's current phase.
//
// Visibility between blocks (each XCD has its own L2): a finished tile's
// writes are released (agent-scope fence in every wave) before its count is
// taken off remaining[g]; the block taking the last count acquires them, and
// releases again before it writes the next phase's items; a block acquires
// after reading an item.  A block waits for an item only while it holds a
// claimed slot, every slot below the final fill level is eventually written by
// a block that is running, and a slot at or above it is recognised (skipped
// phases are counted in ctl[3]); a wall-clock watchdog nevertheless ends the
// wait with the error flag ctl[2] set, which makes every block return.
constexpr unsigned long long kBatchEmpty = ~0ull;

__device__ __forceinline__ unsigned long long batch_item(int32_t g, int ph, int64_t t) {
  return ((unsigned long long)(uint32_t)g << 32) | ((unsigned long long)ph << 28) | (unsigned long long)t;
}

// Edges of graph g in bucket k (ek[k]) and their first edge (lo[k]).
__device__ __forceinline__ void batch_graph_edges(const BatchArgs& B, int32_t g, int64_t* lo, int64_t* ek) {
#pragma unroll
  for (int k = 0; k < kNumBuckets; ++k) {
    const int64_t* row = B.eoff + (int64_t)k * (B.G + 1);
    lo[k] = row[g];
    ek[k] = row[g + 1] - row[g];
  }
}

__device__ __forceinline__ int64_t batch_tiles(const BatchArgs& B, int32_t g, int ph) {
  int64_t lo[kNumBuckets], ek[kNumBuckets];
  batch_graph_edges(B, g, lo, ek);
  return batch_phase_tiles(ph, B.vtx_off[g + 1] - B.vtx_off[g], ek, B.tile_edges, B.tile_vertices, B.split);
}

// Thread 0: claims the next slot and returns its item, or kBatchEmpty when
// the run is over (or was abandoned).
__device__ __forceinline__ unsigned long long batch_take(const BatchArgs& B) {
  const unsigned long long slot = atomicAdd(B.ctl + 0, 1ull);
  if ((int64_t)slot >= B.total) return kBatchEmpty;
  if ((int64_t)slot < B.init_items) {
    int32_t lo = 0, hi = B.G;  // graph g: init_prefix[g] <= slot < init_prefix[g + 1]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (B.init_prefix[mid] <= (int64_t)slot) lo = mid;
      else hi = mid;
    }
    return batch_item(lo, BP_INIT, (int64_t)slot - B.init_prefix[lo]);
  }
  const int64_t idx = (int64_t)slot - B.init_items;
  const uint64_t t0 = wall_clock64();
  while (true) {
    const unsigned long long v = __hip_atomic_load(B.queue + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v != kBatchEmpty) return v;
    // phases skipped so far lower the fill level; a slot at or above it is never written
    const unsigned long long skipped = __hip_atomic_load(B.ctl + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int64_t)slot >= B.total - (int64_t)skipped) return kBatchEmpty;
    if (__hip_atomic_load(B.ctl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return kBatchEmpty;
    if (wall_clock64() - t0 > B.watchdog_ticks) {
      atomicOr(B.ctl + 2, 1ull);
      return kBatchEmpty;
    }
    __builtin_amdgcn_s_sleep(8);
  }
}

template <int MODE>
__device__ __forceinline__ void batch_group(const BatchArgs& B, int k, int64_t lo, int64_t hi, int32_t* T,
                                            PassCounts& pc) {
  const int64_t wave = threadIdx.x >> 6;
  constexpr int64_t nw = kBlock / 64;
  switch (4 << ((B.lanes_code >> (3 * k)) & 7u)) {
    case 4: group_edges<MODE, 4, false>(B.A, lo, hi, wave, nw, T, pc); break;
    case 8: group_edges<MODE, 8, false>(B.A, lo, hi, wave, nw, T, pc); break;
    case 16: group_edges<MODE, 16, false>(B.A, lo, hi, wave, nw, T, pc); break;
    case 32: group_edges<MODE, 32, false>(B.A, lo, hi, wave, nw, T, pc); break;
    default:
      if (k == 4 || k == 5) group_edges<MODE, 64, true>(B.A, lo, hi, wave, nw, T, pc);
      else group_edges<MODE, 64, false>(B.A, lo, hi, wave, nw, T, pc);
      break;
  }
}

// Adds a wave's pass counters to the block's statistics.
__device__ __forceinline__ void batch_count(unsigned long long* sh, int mode, int k, PassCounts pc) {
  const unsigned long long ev = wave_sum(pc.eval), bd = wave_sum(pc.bound), pr = wave_sum(pc.probe);
  if ((threadIdx.x & 63) == 0) {
    if (ev) atomicAdd(sh + ST_EVAL + mode, ev);
    if (bd) atomicAdd(sh + ST_BOUND + mode, bd);
    if (pr) atomicAdd(sh + ST_PROBES + mode, pr);
    if (mode == MODE_CORES) {
      if (ev) atomicAdd(sh + ST_BUCKET_EVAL + k, ev);
      if (pr) atomicAdd(sh + ST_BUCKET_PROBES + k, pr);
    }
  }
}

// Six waves per SIMD: the intersections of the small buckets wait on global
// memory, so occupancy pays for the few registers spilled.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_batch(BatchArgs B) {
  __shared__ __align__(16) int32_t stage[(kBlock / 64) * kWaveSlots];
  __shared__ unsigned long long sh_stats[ST_COUNT];
  __shared__ unsigned long long s_item, s_cores;
  __shared__ int64_t s_base, s_cnt;
  __shared__ int32_t s_next;
  const int tid = threadIdx.x;
  int32_t* T = stage + (tid >> 6) * kWaveSlots;
  for (int i = tid; i < ST_COUNT; i += kBlock) sh_stats[i] = 0;
  const EdgeArgs& A = B.A;
  while (true) {
    if (tid == 0) {
      s_item = batch_take(B);
      s_cores = 0;
    }
    __syncthreads();
    const unsigned long long item = s_item;
    if (item == kBatchEmpty) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the graph's earlier phases
    // uniform over the block: kept in scalar registers
    const int32_t g = __builtin_amdgcn_readfirstlane((int32_t)(item >> 32));
    const int ph = __builtin_amdgcn_readfirstlane((int)((item >> 28) & 15u));
    const int64_t t = __builtin_amdgcn_readfirstlane((int32_t)(item & 0x0FFFFFFFull));
    const int64_t v0 = B.vtx_off[g], v1 = B.vtx_off[g + 1];
    if (batch_vertex_phase(ph)) {
      const int64_t b = v0 + t * B.tile_vertices;
      const int64_t e = min(v1, b + (int64_t)B.tile_vertices);
      bool core = false;
      for (int64_t u = b + tid; u < e; u += kBlock) {
        if (ph == BP_INIT) {
          const int32_t mu = A.gmu[g];
          const int64_t d = A.rp[u + 1] - A.rp[u];
          A.lower[u] = 1;
          A.upper[u] = (int32_t)(d + 1);
          A.role[u] = (d + 1 < mu) ? ROLE_NONCORE : ROLE_UNK;
          A.parent[u] = (int32_t)u;
        } else if (ph == BP_FINAL) {
          uint8_t r = ld_u8(A.role + u);
          if (r == ROLE_UNK) {  // every edge of u was evaluated: lower is exact
            r = A.lower[u] >= A.gmu[g] ? ROLE_CORE : ROLE_NONCORE;
            st_u8(A.role + u, r);
          }
          core = core || r == ROLE_CORE;
          if (r == ROLE_CORE) atomicAdd(&s_cores, 1ull);
        } else if (ph == BP_FLAT) {
          A.label[u] = ld_u8(A.role + u) == ROLE_CORE ? uf_find(A.parent, (int32_t)u) : INT_MAX;
          if (B.split) A.upper[u] = -1;  // first cluster label seen (hub / outlier)
        } else {  // BP_OUTPUT: graph-local labels
          const int32_t lab = A.label[u];
          const int32_t l = lab == INT_MAX ? INT_MAX : lab - (int32_t)v0;
          const uint8_t r = A.role[u];
          if (r == ROLE_CORE) {
            B.out_roles[u] = 1;
            B.out_labels[u] = l;
          } else if (lab != INT_MAX) {
            B.out_roles[u] = 2;
            B.out_labels[u] = l;
          } else {
            B.out_roles[u] = B.split ? (r == ROLE_HUB ? 3 : 4) : 0;
            B.out_labels[u] = -1;
          }
        }
      }
      (void)core;
    } else {
      // edge tile t: edges t * tile_edges .. of the graph's bucket ranges
      // taken one after the other; each bucket's part with its own lanes
      const int64_t tb = t * B.tile_edges, te = tb + B.tile_edges;
      int64_t pos = 0;  // position of bucket k's first edge in the concatenation
      for (int k = 0; k < kNumBuckets; ++k) {
        const int64_t* row = B.eoff + (int64_t)k * (B.G + 1);
        const int64_t lo = row[g], ek = row[g + 1] - lo;
        const int64_t at = pos;
        pos += ek;
        if (at + ek <= tb || at >= te) continue;
        const int64_t eb = lo + max(tb - at, (int64_t)0);
        const int64_t ee = lo + min(te - at, ek);
        PassCounts pc;
        if (ph == BP_CORES) {
          for (int64_t e = eb + tid; e < ee; e += kBlock) A.state[e] = SIM_UNK;
          __syncthreads();
          batch_group<MODE_CORES>(B, k, eb, ee, T, pc);
          batch_count(sh_stats, MODE_CORES, k, pc);
        } else if (ph == BP_HOOK) {
          for (int64_t e = eb + tid; e < ee; e += kBlock) {
            if (A.state[e] != SIM_YES) continue;
            const int2 uv = A.edges[e];
            if (ld_u8(A.role + uv.x) == ROLE_CORE && ld_u8(A.role + uv.y) == ROLE_CORE) uf_union(A.parent, uv.x, uv.y);
          }
        } else if (ph == BP_MERGE) {
          batch_group<MODE_MERGE>(B, k, eb, ee, T, pc);
          batch_count(sh_stats, MODE_MERGE, k, pc);
        } else if (ph == BP_ATTACH) {
          batch_group<MODE_ATTACH>(B, k, eb, ee, T, pc);
          batch_count(sh_stats, MODE_ATTACH, k, pc);
        } else {  // BP_HUBOUT
          for (int64_t e = eb + tid; e < ee; e += kBlock) {
            const int2 uv = A.edges[e];
            const int32_t lu = A.label[uv.x], lv = A.label[uv.y];
            if ((lu == INT_MAX) == (lv == INT_MAX)) continue;
            const int32_t x = (lu == INT_MAX) ? uv.x : uv.y;
            const int32_t L = (lu == INT_MAX) ? lv : lu;
            const int32_t seen = ld_i32(A.upper + x);
            if (seen == L) continue;
            const int32_t old = (seen == -1) ? atomicCAS(A.upper + x, -1, L) : seen;
            if (old != -1 && old != L) st_u8(A.role + x, ROLE_HUB);
          }
        }
      }
    }
    // release this tile's writes, then take it off the graph's phase count
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      s_cnt = 0;
      if (ph == BP_FINAL && s_cores) atomicAdd(B.ncores + g, s_cores);
      if (atomicSub(B.remaining + g, 1) == 1) {
        // last tile of this phase: every other tile's writes are visible from here on
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const bool cores = __hip_atomic_load(B.ncores + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        int next = ph + 1;
        int64_t cnt = 0, skipped = 0;
        for (; next < BP_DONE; ++next) {
          cnt = batch_tiles(B, g, next);
          if (cnt > 0 && !cores && batch_phase_needs_cores(next)) {
            skipped += cnt;
            cnt = 0;
          }
          if (cnt > 0) break;
        }
        if (skipped) atomicAdd(B.ctl + 3, (unsigned long long)skipped);
        if (next < BP_DONE) {
          __hip_atomic_store(B.remaining + g, (int32_t)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_base = (int64_t)atomicAdd(B.ctl + 1, (unsigned long long)cnt);
          s_cnt = cnt;
          s_next = next;
        }
      }
    }
    __syncthreads();
    if (s_cnt > 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the phase's writes and remaining[g] before the items
      const int64_t base = s_base, cnt = s_cnt;
      const int next = s_next;
      for (int64_t i = tid; i < cnt; i += kBlock)
        if (base + i < B.queue_cap)
          __hip_atomic_store(B.queue + base + i, batch_item(g, next, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  for (int i = tid; i < ST_COUNT; i += kBlock)
    if (sh_stats[i]) atomicAdd(A.stats + i, sh_stats[i]);
}

__global__ void k_batch_reset(BatchArgs B) {
  const int64_t n = max(max(B.queue_cap, (int64_t)B.G), (int64_t)ST_COUNT);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    if (i < B.queue_cap) B.queue[i] = kBatchEmpty;
    if (i < B.G) {
      B.remaining[i] = (int32_t)(B.init_prefix[i + 1] - B.init_prefix[i]);
      B.ncores[i] = 0;
    }
    if (i < 4) B.ctl[i] = 0;
    if (i < ST_COUNT) B.A.stats[i] = 0;
  }
}

// eoff[k * (G + 1) + g] = first edge of bucket k whose larger side is at or
// after vtx_off[g] (edges of a bucket are in increasing order of their larger
// side, and graph g's vertices are vtx_off[g] .. vtx_off[g + 1] - 1).
__global__ void k_batch_edge_offsets(int32_t G, const int64_t* vtx_off, const int2* edges, int64_t b0, int64_t b1,
                                     int64_t* eoff) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g > G) return;
  const int64_t v = vtx_off[g];
  int64_t lo = b0, hi = b1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)edges[mid].y < v) lo = mid + 1;
    else hi = mid;
  }
  eoff[g] = (g == G) ? b1 : lo;
}

inline unsigned blocks_for(int64_t items, int64_t per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

// Grid-size caps of the group buckets (blocks of kBlock threads; a smaller
// grid makes each wave loop over several 64-edge chunks).  The buckets of the
// shortest lists are latency-bound on per-vertex state, where fewer, longer-
// lived waves do better; the wider groups keep more waves in flight.
constexpr int64_t kGroupGridCap[kNumBuckets] = {2048, 2048, 4096, 8192, 8192, 8192, 8192};

template <int MODE>
void launch_edges_mode(hipStream_t s, int bucket, const EdgeArgs& a) {
  const int64_t m = a.e_end - a.e_begin;
  if (m <= 0) return;
  const unsigned grid = blocks_for(m, kBlock, kGroupGridCap[bucket >= 0 && bucket < kNumBuckets ? bucket : kNumBuckets - 1]);
  switch (bucket) {
    case 0: k_group<MODE, 4><<<grid, kBlock, 0, s>>>(a); break;
    case 1: k_group<MODE, 8><<<grid, kBlock, 0, s>>>(a); break;
    case 2: k_group<MODE, 16><<<grid, kBlock, 0, s>>>(a); break;
    case 3: k_group<MODE, 32><<<grid, kBlock, 0, s>>>(a); break;
    case 4:
    case 5: k_group<MODE, 64, true><<<grid, kBlock, 0, s>>>(a); break;
    default: k_group<MODE, 64><<<grid, kBlock, 0, s>>>(a); break;
  }
}

}  // namespace

void launch_init(hipStream_t s, int32_t n, const int64_t* rp, int32_t mu, int32_t* lower,
                 int32_t* upper, uint8_t* role, int32_t* parent, const int32_t* gid, const int32_t* gmu) {
  if (n > 0) k_init<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, rp, mu, gid, gmu, lower, upper, role, parent);
}

void launch_fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v) {
  if (n > 0) k_fill_u8<<<blocks_for(n, 256 * 16, 8192), 256, 0, s>>>(p, n, v);
}

template <int MODE>
void launch_edges_width(hipStream_t s, int lanes, const EdgeArgs& a) {
  const int64_t m = a.e_end - a.e_begin;
  if (m <= 0) return;
  const unsigned grid = blocks_for(m, kBlock, 8192);
  switch (lanes) {
    case 4: k_group<MODE, 4><<<grid, kBlock, 0, s>>>(a); break;
    case 8: k_group<MODE, 8><<<grid, kBlock, 0, s>>>(a); break;
    case 16: k_group<MODE, 16><<<grid, kBlock, 0, s>>>(a); break;
    case 32: k_group<MODE, 32><<<grid, kBlock, 0, s>>>(a); break;
    default:
      if (a.bucket == 4 || a.bucket == 5) k_group<MODE, 64, true><<<grid, kBlock, 0, s>>>(a);
      else k_group<MODE, 64><<<grid, kBlock, 0, s>>>(a);
      break;
  }
}

void launch_edges_lanes(hipStream_t s, int mode, int lanes, const EdgeArgs& a) {
  switch (mode) {
    case MODE_CORES: launch_edges_width<MODE_CORES>(s, lanes, a); break;
    case MODE_MERGE: launch_edges_width<MODE_MERGE>(s, lanes, a); break;
    case MODE_ATTACH: launch_edges_width<MODE_ATTACH>(s, lanes, a); break;
    default: launch_edges_width<MODE_COUNTS>(s, lanes, a); break;
  }
}

void launch_edges(hipStream_t s, int mode, int bucket, const EdgeArgs& a) {
  switch (mode) {
    case MODE_CORES: launch_edges_mode<MODE_CORES>(s, bucket, a); break;
    case MODE_MERGE: launch_edges_mode<MODE_MERGE>(s, bucket, a); break;
    case MODE_ATTACH: launch_edges_mode<MODE_ATTACH>(s, bucket, a); break;
    default: launch_edges_mode<MODE_COUNTS>(s, bucket, a); break;
  }
}

int hub_grid_blocks() {
  static int n_cu = 0;  // compute units of the current device (the library drives one GPU)
  if (n_cu == 0) {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      n_cu = cu;
    else
      n_cu = 256;
  }
  return n_cu;
}

void launch_hub(hipStream_t s, int mode, const EdgeArgs& a, const HubJob* jobs, int64_t njobs,
                unsigned long long* counter, int32_t* worklist) {
  if (njobs <= 0) return;
  // kHubBlocksPerCU resident blocks per compute unit (their tables fill most
  // of its LDS; while one block waits at a barrier the other computes);
  // blocks take jobs from the counter until none are left
  const unsigned grid = blocks_for(njobs, 1, (int64_t)kHubBlocksPerCU * hub_grid_blocks());
  switch (mode) {
    case MODE_CORES: k_hub<MODE_CORES><<<grid, kHubBlock, 0, s>>>(a, jobs, njobs, counter, worklist); break;
    case MODE_MERGE: k_hub<MODE_MERGE><<<grid, kHubBlock, 0, s>>>(a, jobs, njobs, counter, worklist); break;
    case MODE_ATTACH: k_hub<MODE_ATTACH><<<grid, kHubBlock, 0, s>>>(a, jobs, njobs, counter, worklist); break;
    default: k_hub<MODE_COUNTS><<<grid, kHubBlock, 0, s>>>(a, jobs, njobs, counter, worklist); break;
  }
}

void launch_copy16(hipStream_t s, const void* src, void* dst, int64_t n16) {
  if (n16 > 0) k_copy16<<<blocks_for(n16, 256, 16384), 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
}

int read16_sink_words() { return 16384 * 256; }

void launch_read16(hipStream_t s, const void* src, int64_t n16, uint32_t* sink) {
  if (n16 > 0) k_read16<<<blocks_for(n16, 256, 16384), 256, 0, s>>>((const uint4*)src, n16, sink);
}

void launch_line_samples(hipStream_t s, int64_t nlines, const int32_t* rows, int32_t* samp) {
  if (nlines > 0) k_line_samples<<<blocks_for(nlines, 256, 16384), 256, 0, s>>>(nlines, rows, samp);
}

void launch_edge_degrees(hipStream_t s, int64_t m, const int64_t* rp, const int2* edges, int2* deg) {
  if (m > 0) k_edge_degrees<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, rp, edges, deg);
}

void launch_zero_u64(hipStream_t s, unsigned long long* p, int n) {
  if (n > 0) k_zero_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
}

void launch_finalize_roles(hipStream_t s, int32_t n, int32_t mu, const int32_t* lower, uint8_t* role,
                           const int32_t* gid, const int32_t* gmu, unsigned long long* ncores) {
  if (n > 0) k_finalize<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, mu, gid, gmu, lower, role, ncores);
}

void launch_hook(hipStream_t s, int64_t m, const int2* edges, const uint8_t* state,
                 const uint8_t* role, int32_t* parent) {
  if (m > 0) k_hook<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, state, role, parent);
}

void launch_flatten(hipStream_t s, int32_t n, const uint8_t* role, int32_t* parent, int32_t* label) {
  if (n > 0) k_flatten<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, role, parent, label);
}

void launch_output(hipStream_t s, int32_t n, const uint8_t* role, const int32_t* label,
                   int32_t* out_labels, uint8_t* out_roles, int32_t split, const int32_t* gid,
                   const int32_t* gbase) {
  if (n > 0)
    k_output<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, role, label, gid, gbase, out_labels, out_roles, split);
}

void launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n > 0) k_fill_i32<<<blocks_for(n, 256, 8192), 256, 0, s>>>(p, n, v);
}

void launch_hub_outlier_edges(hipStream_t s, int64_t m, const int2* edges, const int32_t* label, int32_t* first,
                              uint8_t* role) {
  if (m > 0) k_hub_outlier<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, label, first, role);
}


void launch_closed_products(hipStream_t s, int64_t m, const int64_t* rp, const int2* edges, uint64_t* ab) {
  if (m > 0) k_closed_products<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, rp, ab);
}

void launch_rethreshold(hipStream_t s, int32_t n, int64_t m, const int2* edges, const int32_t* ecount,
                        const uint64_t* ab, uint64_t p, uint64_t q, int32_t mu, int32_t* lower,
                        uint8_t* role, int32_t* parent, int32_t* label, uint8_t* state,
                        int32_t* out_labels, uint8_t* out_roles, int32_t split) {
  if (n <= 0) return;
  k_rt_init<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, lower, parent);
  if (m > 0) k_rt_edges<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, ecount, ab, p, q, state, lower);
  k_rt_roles<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, mu, lower, role);
  if (m > 0) k_hook<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, state, role, parent);
  k_flatten<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, role, parent, label);
  if (m > 0) k_rt_attach<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, state, role, label);
  if (split) {
    k_fill_i32<<<blocks_for(n, 256, 8192), 256, 0, s>>>(lower, n, -1);  // counts are no longer needed
    if (m > 0) k_hub_outlier<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, label, lower, role);
  }
  k_output<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, role, label, nullptr, nullptr, out_labels, out_roles,
                                                       split);
}

void launch_batch(hipStream_t s, const BatchArgs& B, int grid) {
  const int64_t n = std::max<int64_t>(std::max<int64_t>(B.queue_cap, B.G), ST_COUNT);
  k_batch_reset<<<blocks_for(n, 256, 16384), 256, 0, s>>>(B);
  if (B.total > 0) k_batch<<<grid, kBlock, 0, s>>>(B);
}

void launch_batch_edge_offsets(hipStream_t s, int32_t G, const int64_t* vtx_off, const int2* edges,
                               const int64_t* bucket_off_host, int64_t* eoff) {
  for (int k = 0; k < kNumBuckets; ++k)
    k_batch_edge_offsets<<<blocks_for((int64_t)G + 1, 256, 1 << 30), 256, 0, s>>>(
        G, vtx_off, edges, bucket_off_host[k], bucket_off_host[k + 1], eoff + (int64_t)k * (G + 1));
}

int batch_grid_blocks() {
  static int blocks = 0;  // the library drives one GPU
  if (blocks == 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_batch), kBlock, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    blocks = per_cu * hub_grid_blocks();
  }
  return blocks;
}

}  // namespace scan
