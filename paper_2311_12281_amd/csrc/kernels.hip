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
//   d_s <= 64 : a group of G in {4, 8, 16, 32, 64} lanes per edge, one lane
//               per element of the smaller list, each binary-searching the
//               larger list; the group's count is a ballot popcount.
//   d_s  > 64 : one wave per edge; the smaller list in tiles of 64, each lane
//               binary-searching the unread remainder of the larger list; the
//               remainder shrinks tile by tile because both lists are sorted.
//               The loop stops as soon as the verdict is known (count reached
//               or unreachable), except when exact counts are requested.
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

// Per-edge decision taken before any intersection.
struct EdgeView {
  int32_t u, v;       // u = smaller side
  int64_t bu, bv;     // row starts
  int64_t du, dv;     // degrees
  int32_t need;       // closed count needed for similarity
  int32_t core_side;  // ATTACH: endpoint that is the core (u or v)
  int32_t other;      // ATTACH: the non-core endpoint
  int32_t core_label; // ATTACH
  uint8_t work;       // 1: run the intersection
};

template <int MODE>
__device__ __forceinline__ void classify(const EdgeArgs& A, int64_t e, bool active, EdgeView& ev,
                                         unsigned long long& n_bound) {
  ev.work = 0;
  if (!active) return;
  const int2 uv = A.edges[e];
  ev.u = uv.x;
  ev.v = uv.y;
  ev.bu = A.rp[ev.u];
  ev.du = A.rp[ev.u + 1] - ev.bu;
  ev.bv = A.rp[ev.v];
  ev.dv = A.rp[ev.v + 1] - ev.bv;
  const uint64_t a = (uint64_t)ev.du + 1, b = (uint64_t)ev.dv + 1;
  if (MODE == MODE_COUNTS) {
    ev.work = 1;
    return;
  }
  if (MODE == MODE_CORES) {
    if (A.pruning) {
      const uint8_t ru = ld_u8(A.role + ev.u), rv = ld_u8(A.role + ev.v);
      if (ru != ROLE_UNK && rv != ROLE_UNK) return;  // Alg. 2: both roles known, defer
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
  if (A.pruning && a * A.q * A.q < A.p * A.p * b) {
    ev.work = 3;
    ++n_bound;
    return;
  }
  ev.need = (int32_t)closed_needed(A.p, A.q, a, b);
  ev.work = 1;
}

// Effect of a decided edge; executed by one lane.
template <int MODE>
__device__ __forceinline__ void apply(const EdgeArgs& A, int64_t e, const EdgeView& ev, bool sim,
                                      int32_t closed) {
  if (MODE == MODE_COUNTS) {
    const int64_t pu = lower_bound(A.ci, ev.bu, ev.bu + ev.du, ev.v);
    const int64_t pv = lower_bound(A.ci, ev.bv, ev.bv + ev.dv, ev.u);
    if (pu < ev.bu + ev.du && A.ci[pu] == ev.v) A.counts[pu] = closed;
    if (pv < ev.bv + ev.dv && A.ci[pv] == ev.u) A.counts[pv] = closed;
    return;
  }
  if (MODE == MODE_CORES) {
    A.state[e] = sim ? SIM_YES : SIM_NO;
    if (sim) {
      if (atomicAdd(A.lower + ev.u, 1) + 1 >= A.mu) st_u8(A.role + ev.u, ROLE_CORE);
      if (atomicAdd(A.lower + ev.v, 1) + 1 >= A.mu) st_u8(A.role + ev.v, ROLE_CORE);
    } else {
      if (atomicSub(A.upper + ev.u, 1) - 1 < A.mu) st_u8(A.role + ev.u, ROLE_NONCORE);
      if (atomicSub(A.upper + ev.v, 1) - 1 < A.mu) st_u8(A.role + ev.v, ROLE_NONCORE);
    }
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

// Buckets 0-4: G lanes per edge, d_s <= G.
template <int MODE, int G>
__global__ __launch_bounds__(kBlock) void k_edges_group(EdgeArgs A) {
  constexpr int kPerWave = 64 / G;
  const int lane = threadIdx.x & 63;
  const int sub = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  unsigned long long n_eval = 0, n_bound = 0, n_probe = 0;
  for (int64_t t = A.e_begin + wave * kPerWave; t < A.e_end; t += nwaves * kPerWave) {
    const int64_t e = t + lane / G;
    EdgeView ev;
    unsigned long long nb = 0;
    classify<MODE>(A, e, e < A.e_end, ev, nb);
    bool found = false;
    if (ev.work == 1 && sub < ev.du) {
      const int32_t x = A.ci[ev.bu + sub];
      const int64_t pos = lower_bound(A.ci, ev.bv, ev.bv + ev.dv, x);
      found = pos < ev.bv + ev.dv && A.ci[pos] == x;
    }
    const int32_t cnt = __popcll(__ballot(found) & gmask);
    if (sub == 0) {
      n_bound += nb;
      if (ev.work == 1) {
        ++n_eval;
        n_probe += (unsigned long long)ev.du;
        const int32_t closed = cnt + 2;
        apply<MODE>(A, e, ev, MODE == MODE_COUNTS ? false : closed >= ev.need, closed);
      } else if (ev.work == 2) {
        apply<MODE>(A, e, ev, true, 0);
      } else if (ev.work == 3 && MODE != MODE_ATTACH) {
        apply<MODE>(A, e, ev, false, 0);
      }
    }
  }
  flush_stats(A, MODE, n_eval, n_bound, n_probe);
}

// Bucket 5: one wave per edge, d_s > 64.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_edges_wave(EdgeArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const bool exact = (MODE == MODE_COUNTS) || !A.pruning;
  unsigned long long n_eval = 0, n_bound = 0, n_probe = 0;
  for (int64_t e = A.e_begin + wave; e < A.e_end; e += nwaves) {
    EdgeView ev;
    unsigned long long nb = 0;
    classify<MODE>(A, e, true, ev, nb);
    n_bound += (lane == 0) ? nb : 0;
    if (ev.work == 2 || ev.work == 3) {
      if (lane == 0 && (ev.work == 2 || MODE != MODE_ATTACH)) apply<MODE>(A, e, ev, ev.work == 2, 0);
      continue;
    }
    if (ev.work != 1) continue;
    const int32_t* B = A.ci + ev.bv;
    const int32_t* Arow = A.ci + ev.bu;
    const int32_t need_open = ev.need - 2;
    int32_t cnt = 0;
    int64_t lo = 0, consumed = 0;
    bool decided = false, sim = false;
    if (!exact && need_open <= 0) { decided = true; sim = true; }
    for (int64_t t = 0; t < ev.du && !decided; t += 64) {
      const int64_t i = t + lane;
      const bool valid = i < ev.du;
      int64_t pos = ev.dv;
      bool f = false;
      if (valid) {
        const int32_t x = Arow[i];
        pos = lower_bound(B, lo, ev.dv, x);
        f = pos < ev.dv && B[pos] == x;
      }
      cnt += __popcll(__ballot(f));
      const int64_t take = ev.du - t < 64 ? ev.du - t : 64;
      consumed += take;
      lo = __shfl(pos, (int)(take - 1), 64);
      if (!exact) {
        if (cnt >= need_open) { decided = true; sim = true; }
        else {
          int64_t rem = ev.du - (t + take);
          if (ev.dv - lo < rem) rem = ev.dv - lo;
          if (cnt + rem < need_open) { decided = true; sim = false; }
        }
      }
      if (lo >= ev.dv && !decided) break;  // larger list exhausted
    }
    if (!decided) sim = (cnt + 2) >= ev.need;
    if (lane == 0) {
      ++n_eval;
      n_probe += (unsigned long long)consumed;
      apply<MODE>(A, e, ev, MODE == MODE_COUNTS ? false : sim, cnt + 2);
    }
  }
  flush_stats(A, MODE, n_eval, n_bound, n_probe);
}

__global__ void k_init(int32_t n, const int64_t* rp, int32_t mu, int32_t* lower, int32_t* upper,
                       uint8_t* role, int32_t* parent) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
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

__global__ void k_finalize(int32_t n, int32_t mu, const int32_t* lower, uint8_t* role) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  // A role still unknown here had every incident edge evaluated (an edge is
  // only deferred when both roles are known), so lower is |N_eps[u]| exactly.
  if (role[u] == ROLE_UNK) role[u] = lower[u] >= mu ? ROLE_CORE : ROLE_NONCORE;
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

__global__ void k_output(int32_t n, const uint8_t* role, const int32_t* label, int32_t* out_labels,
                         uint8_t* out_roles) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t l = label[u];
  if (role[u] == ROLE_CORE) {
    out_roles[u] = 1;
    out_labels[u] = l;
  } else if (l != INT_MAX) {
    out_roles[u] = 2;
    out_labels[u] = l;
  } else {
    out_roles[u] = 0;
    out_labels[u] = -1;
  }
}

inline unsigned blocks_for(int64_t items, int64_t per_block, int64_t cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <int MODE>
void launch_edges_mode(hipStream_t s, int bucket, const EdgeArgs& a) {
  const int64_t m = a.e_end - a.e_begin;
  if (m <= 0) return;
  constexpr int64_t kCap = 16384;
  switch (bucket) {
    case 0: k_edges_group<MODE, 4><<<blocks_for(m, 64, kCap), kBlock, 0, s>>>(a); break;
    case 1: k_edges_group<MODE, 8><<<blocks_for(m, 32, kCap), kBlock, 0, s>>>(a); break;
    case 2: k_edges_group<MODE, 16><<<blocks_for(m, 16, kCap), kBlock, 0, s>>>(a); break;
    case 3: k_edges_group<MODE, 32><<<blocks_for(m, 8, kCap), kBlock, 0, s>>>(a); break;
    case 4: k_edges_group<MODE, 64><<<blocks_for(m, 4, kCap), kBlock, 0, s>>>(a); break;
    default: k_edges_wave<MODE><<<blocks_for(m, 4, kCap), kBlock, 0, s>>>(a); break;
  }
}

}  // namespace

void launch_init(hipStream_t s, int32_t n, const int64_t* rp, int32_t mu, int32_t* lower,
                 int32_t* upper, uint8_t* role, int32_t* parent) {
  if (n > 0) k_init<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, rp, mu, lower, upper, role, parent);
}

void launch_fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v) {
  if (n > 0) k_fill_u8<<<blocks_for(n, 256 * 16, 8192), 256, 0, s>>>(p, n, v);
}

void launch_edges(hipStream_t s, int mode, int bucket, const EdgeArgs& a) {
  switch (mode) {
    case MODE_CORES: launch_edges_mode<MODE_CORES>(s, bucket, a); break;
    case MODE_MERGE: launch_edges_mode<MODE_MERGE>(s, bucket, a); break;
    case MODE_ATTACH: launch_edges_mode<MODE_ATTACH>(s, bucket, a); break;
    default: launch_edges_mode<MODE_COUNTS>(s, bucket, a); break;
  }
}

void launch_finalize_roles(hipStream_t s, int32_t n, int32_t mu, const int32_t* lower, uint8_t* role) {
  if (n > 0) k_finalize<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, mu, lower, role);
}

void launch_hook(hipStream_t s, int64_t m, const int2* edges, const uint8_t* state,
                 const uint8_t* role, int32_t* parent) {
  if (m > 0) k_hook<<<blocks_for(m, 256, 16384), 256, 0, s>>>(m, edges, state, role, parent);
}

void launch_flatten(hipStream_t s, int32_t n, const uint8_t* role, int32_t* parent, int32_t* label) {
  if (n > 0) k_flatten<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, role, parent, label);
}

void launch_output(hipStream_t s, int32_t n, const uint8_t* role, const int32_t* label,
                   int32_t* out_labels, uint8_t* out_roles) {
  if (n > 0) k_output<<<blocks_for(n, 256, 1 << 30), 256, 0, s>>>(n, role, label, out_labels, out_roles);
}

}  // namespace scan
