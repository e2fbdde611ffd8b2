// Seeded synthetic graph generators (host C++, OpenMP).
//
// This file produces input graphs only: it holds none of the structural
// clustering arithmetic, and both the CPU oracle and the GPU path consume
// its output through the same Python module.  Every generator is
// deterministic for a given seed, independent of the thread count.
//
// Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), used both as a counter-based
// hash (R-MAT: one output per (sample, level)) and as a sequential stream
// (planted partition and Chung-Lu: one stream per pair region / per row).
//
// Output format: undirected simple graph as a symmetric CSR with int64 row
// offsets and strictly increasing int32 neighbour ids per row.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t splitmix64_next(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter-based use: the value at position `ctr` of the stream seeded by `key`.
inline uint64_t splitmix64_at(uint64_t key, uint64_t ctr) {
  uint64_t s = key + ctr * 0x9E3779B97F4A7C15ull;
  return splitmix64_next(s);
}

// Uniform double in [0, 1) from the top 53 bits.
inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

inline uint64_t mix_key(uint64_t seed, uint64_t a, uint64_t b) {
  uint64_t s = seed ^ 0x6A09E667F3BCC909ull;
  uint64_t k = splitmix64_next(s);
  s = k ^ (a * 0xD1B54A32D192ED03ull);
  k = splitmix64_next(s);
  s = k ^ (b * 0x8CB92BA72F3D8DD7ull);
  return splitmix64_next(s);
}

// Geometric skip for Bernoulli(p) trials (Batagelj & Brandes 2005): number of
// failures before the next success.
inline double geo_skip(uint64_t& st, double log1mp) {
  double u = u01(splitmix64_next(st));
  // 1-u in (0,1]; log(1-u) <= 0.
  return std::floor(std::log1p(-u) / log1mp);
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): for every sample pick, at
// each of `scale` bit levels, one of four quadrants with probabilities
// (a, b, c, 1-a-b-c).  Sample i uses hash outputs (seed, i, level).
// Writes raw (possibly self-loop / duplicate) directed pairs.
int gg_rmat_pairs(int scale, int64_t nsamples, double a, double b, double c,
                  uint64_t seed, int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30 || nsamples < 0) return -1;
  const double ab = a + b, abc = a + b + c;
  const uint64_t key = mix_key(seed, 0x524D4154ull, (uint64_t)scale);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nsamples; ++i) {
    uint32_t u = 0, v = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      double r = u01(splitmix64_at(key, (uint64_t)i * 64u + (uint64_t)lvl));
      uint32_t bu, bv;
      if (r < a) { bu = 0; bv = 0; }
      else if (r < ab) { bu = 0; bv = 1; }
      else if (r < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Planted partition: vertices 0..n-1 in `nblocks` contiguous blocks
// (block k = [floor(k*n/B), floor((k+1)*n/B)) ), every unordered pair an
// independent Bernoulli trial with p_in inside a block and p_out across.
// Pairs are drawn region by region with geometric skipping, one SplitMix64
// stream per (seed, region).  Two calls: with src == NULL the function
// returns the number of pairs it would write; otherwise it writes them.
int64_t gg_planted_pairs(int32_t n, int32_t nblocks, double p_in, double p_out,
                         uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 0 || nblocks < 1 || nblocks > n + 1 || p_in < 0 || p_in > 1 ||
      p_out < 0 || p_out > 1)
    return -1;
  if (n == 0) return 0;
  const int64_t B = nblocks;
  std::vector<int32_t> bstart(B + 1);
  for (int64_t k = 0; k <= B; ++k) bstart[k] = (int32_t)((k * (int64_t)n) / B);
  const int64_t nreg = B + B * (B - 1) / 2;
  std::vector<std::vector<int32_t>> out((size_t)nreg);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nreg; ++r) {
    std::vector<int32_t>& o = out[(size_t)r];
    uint64_t st = mix_key(seed, 0x504C414Eull, (uint64_t)r);
    if (r < B) {
      // within block r: pairs (i<j), enumerated row by row
      const int64_t lo = bstart[r], s = bstart[r + 1] - bstart[r];
      const int64_t total = s * (s - 1) / 2;
      if (total <= 0 || p_in <= 0) continue;
      int64_t i = 0, row_end = s - 1;  // pairs with first index i: [row_begin, row_end)
      int64_t row_begin = 0;
      if (p_in >= 1) {
        for (int64_t a = 0; a < s; ++a)
          for (int64_t b = a + 1; b < s; ++b) { o.push_back((int32_t)(lo + a)); o.push_back((int32_t)(lo + b)); }
        continue;
      }
      const double l1p = std::log1p(-p_in);
      double t = -1;
      for (;;) {
        t += 1 + geo_skip(st, l1p);
        if (t >= (double)total) break;
        int64_t ti = (int64_t)t;
        while (ti >= row_end) {
          ++i;
          row_begin = row_end;
          row_end += s - 1 - i;
        }
        int64_t j = i + 1 + (ti - row_begin);
        o.push_back((int32_t)(lo + i));
        o.push_back((int32_t)(lo + j));
      }
    } else {
      // across blocks k1 < k2 (region index r - B in row-major upper triangle)
      int64_t q = r - B, k1 = 0;
      while (q >= B - 1 - k1) { q -= B - 1 - k1; ++k1; }
      const int64_t k2 = k1 + 1 + q;
      const int64_t lo1 = bstart[k1], s1 = bstart[k1 + 1] - bstart[k1];
      const int64_t lo2 = bstart[k2], s2 = bstart[k2 + 1] - bstart[k2];
      const int64_t total = s1 * s2;
      if (total <= 0 || p_out <= 0) continue;
      if (p_out >= 1) {
        for (int64_t a = 0; a < s1; ++a)
          for (int64_t b = 0; b < s2; ++b) { o.push_back((int32_t)(lo1 + a)); o.push_back((int32_t)(lo2 + b)); }
        continue;
      }
      const double l1p = std::log1p(-p_out);
      double t = -1;
      for (;;) {
        t += 1 + geo_skip(st, l1p);
        if (t >= (double)total) break;
        int64_t ti = (int64_t)t;
        o.push_back((int32_t)(lo1 + ti / s2));
        o.push_back((int32_t)(lo2 + ti % s2));
      }
    }
  }
  int64_t cnt = 0;
  for (auto& o : out) cnt += (int64_t)o.size() / 2;
  if (!src) return cnt;
  int64_t pos = 0;
  for (auto& o : out) {
    for (size_t k = 0; k < o.size(); k += 2) { src[pos] = o[k]; dst[pos] = o[k + 1]; ++pos; }
  }
  return cnt;
}

// ---------------------------------------------------------------------------
// Chung-Lu (Chung & Lu 2002) with expected degrees w (non-increasing), edge
// probability p_ij = min(1, w_i w_j / S), S = sum w, drawn in O(n + m) by the
// skipping method of Miller & Hagberg (WAW 2011): row i uses its own
// SplitMix64 stream, so rows can be generated in parallel.  With src == NULL
// returns the pair count only.
int64_t gg_chunglu_pairs(int32_t n, const double* w, uint64_t seed,
                         int32_t* src, int32_t* dst, int64_t* row_counts) {
  if (n < 0) return -1;
  double S = 0;
  for (int32_t i = 0; i < n; ++i) S += w[i];
  if (S <= 0) return 0;
  const uint64_t key = mix_key(seed, 0x43484C55ull, (uint64_t)n);
  // pass 1 (counting) or pass 2 (writing at row_counts prefix)
  const bool write = src != nullptr;
#pragma omp parallel for schedule(dynamic, 256)
  for (int32_t u = 0; u < n; ++u) {
    uint64_t st = splitmix64_at(key, (uint64_t)u);
    int64_t pos = write ? row_counts[u] : 0;
    int64_t cnt = 0;
    int64_t v = (int64_t)u + 1;
    double p = std::min(1.0, w[u] * (v < n ? w[v] : 0.0) / S);
    while (v < n && p > 0) {
      if (p != 1.0) {
        double r = u01(splitmix64_next(st));
        v += (int64_t)std::floor(std::log1p(-r) / std::log1p(-p));
      }
      if (v < n) {
        double q = std::min(1.0, w[u] * w[v] / S);
        double r = u01(splitmix64_next(st));
        if (r < q / p) {
          if (write) { src[pos] = u; dst[pos] = (int32_t)v; ++pos; }
          ++cnt;
        }
        p = q;
        ++v;
      }
    }
    if (!write) row_counts[u] = cnt;
  }
  if (write) return row_counts[n];
  // exclusive prefix over row_counts (size n+1)
  int64_t acc = 0;
  for (int32_t u = 0; u < n; ++u) { int64_t c = row_counts[u]; row_counts[u] = acc; acc += c; }
  row_counts[n] = acc;
  return acc;
}

// ---------------------------------------------------------------------------
// Raw directed pairs -> symmetric simple CSR, step 1: drop self-loops, insert
// both directions, sort each row, drop duplicates.  raw_rp must hold n+1
// entries and raw_ci 2*npairs entries.  deg receives the deduplicated row
// lengths.  Returns the final number of arcs.
int64_t gg_symmetrize(int32_t n, int64_t npairs, const int32_t* src, const int32_t* dst,
                      int64_t* raw_rp, int32_t* raw_ci, int64_t* deg) {
  if (n < 0 || npairs < 0) return -1;
  std::memset(raw_rp, 0, sizeof(int64_t) * ((size_t)n + 1));
  int bad = 0;
  // counts and scatter in parallel with atomic cursors: the order inside a
  // raw row depends on the threads, but every row is sorted and deduplicated
  // below, so the result does not
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < npairs; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (u < 0 || v < 0 || u >= n || v >= n) { bad = 1; continue; }
    if (u == v) continue;
    __atomic_fetch_add(raw_rp + u + 1, 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(raw_rp + v + 1, 1, __ATOMIC_RELAXED);
  }
  if (bad) return -2;
  for (int32_t u = 0; u < n; ++u) raw_rp[u + 1] += raw_rp[u];
  std::vector<int64_t> cur(raw_rp, raw_rp + n);
  int64_t* cp = cur.data();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (u == v) continue;
    raw_ci[__atomic_fetch_add(cp + u, 1, __ATOMIC_RELAXED)] = v;
    raw_ci[__atomic_fetch_add(cp + v, 1, __ATOMIC_RELAXED)] = u;
  }
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : total)
  for (int32_t u = 0; u < n; ++u) {
    int32_t* b = raw_ci + raw_rp[u];
    int32_t* e = raw_ci + raw_rp[u + 1];
    std::sort(b, e);
    int64_t k = std::unique(b, e) - b;
    deg[u] = k;
    total += k;
  }
  return total;
}

// Step 2: compact the deduplicated rows into the final CSR.
int gg_compact(int32_t n, const int64_t* raw_rp, const int32_t* raw_ci, const int64_t* deg,
               int64_t* rp, int32_t* ci) {
  rp[0] = 0;
  for (int32_t u = 0; u < n; ++u) rp[u + 1] = rp[u] + deg[u];
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; ++u)
    std::memcpy(ci + rp[u], raw_ci + raw_rp[u], sizeof(int32_t) * (size_t)deg[u]);
  return 0;
}

// Relabel a CSR by a permutation perm (new id of old vertex v = perm[v]).
// out arrays are preallocated with the same sizes.
int gg_permute(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* perm,
               int64_t* rp_out, int32_t* ci_out) {
  std::vector<int32_t> inv((size_t)n);
  for (int32_t v = 0; v < n; ++v) inv[perm[v]] = v;
  rp_out[0] = 0;
  for (int32_t x = 0; x < n; ++x) rp_out[x + 1] = rp_out[x] + (rp[inv[x] + 1] - rp[inv[x]]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t x = 0; x < n; ++x) {
    int32_t v = inv[x];
    int32_t* o = ci_out + rp_out[x];
    int64_t d = rp[v + 1] - rp[v];
    for (int64_t k = 0; k < d; ++k) o[k] = perm[ci[rp[v] + k]];
    std::sort(o, o + d);
  }
  return 0;
}

int gg_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
