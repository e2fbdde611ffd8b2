/*
 * CPU oracle for exact structural graph clustering (SCAN) over closed
 * neighbourhoods, as defined in GPUSCAN++ (Yuan et al., arXiv 2311.12281),
 * Section 2.1, Definitions 2.1-2.6 and the problem statement after them.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against a plain
 * implementation of the definitions.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * What is computed (all integer, exact):
 *   N[x]        = nbr(x) + {x}                                  (Def 2.1)
 *   c(u,v)      = |N[u] intersect N[v]|                         (Def 2.2 numerator)
 *   similar     : sigma(u,v) = c / sqrt(|N[u]| |N[v]|) >= eps = p/q.  All
 *                 quantities are non-negative, so this holds exactly when
 *                 (c q)^2 >= p^2 |N[u]| |N[v]|; evaluated in 128-bit
 *                 integers, so it is exact (Def 2.3; equality is similar).
 *   core        : |N_eps[u]| >= mu, where N_eps[u] counts u itself
 *                 (sigma(u,u) = 1) plus every similar neighbour (Def 2.4).
 *   clusters    : cores joined by similar core-core edges (structural
 *                 reachability, Def 2.5, and the cluster of Def 2.6); a
 *                 cluster is labelled by its minimum core id, found by a
 *                 breadth-first search started from every unlabelled core in
 *                 ascending id order.
 *   borders     : a non-core vertex similar to at least one core belongs to
 *                 the cluster(s) of those cores; it receives the minimum of
 *                 their labels.  Every other vertex is unclassified (-1).
 *
 * Readings where the paper leaves a choice (each is also listed in the
 * design notes): the exact integer test replaces the floating-point test of
 * checkSim (Alg. 2); "<= mu" of Lemma 4.1 is not used here at all (the
 * oracle counts N_eps exactly); a border in several clusters takes the
 * minimum label (Alg. 3 leaves the last writer); a cluster must hold a core.
 *
 * Two ways of counting c(u,v) are provided:
 *   oracle_closed_count  - one pair at a time, merging the two closed sorted
 *                          lists (the definition of |A intersect B| for
 *                          sorted sets);
 *   oracle_counts_all    - every edge, as sum over w in the smaller closed
 *                          set of [w in the larger set], the membership test
 *                          read from an indicator array of the larger set.
 * Both give the same integer; the tests pin each against brute force.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_INVAL (-1)
#define OR_GRAPH (-2)
#define OR_NOMEM (-4)

#define ROLE_UNCLASSIFIED 0
#define ROLE_CORE 1
#define ROLE_BORDER 2
#define ROLE_HUB 3     /* Def 2.7 */
#define ROLE_OUTLIER 4

/* Position of x in the sorted row, or -1. */
static int64_t row_find(const int32_t* row, int64_t len, int32_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (row[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return (lo < len && row[lo] == x) ? lo : -1;
}

/* Input checks: offsets monotone from 0 to nnz, ids in range, rows strictly
 * increasing (simple graph), no self-loops, every arc has its reverse. */
int oracle_validate(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci) {
  if (n < 0 || nnz < 0 || !rp || (nnz > 0 && !ci)) return OR_INVAL;
  if (rp[0] != 0 || rp[n] != nnz) return OR_GRAPH;
  for (int32_t u = 0; u < n; ++u) {
    if (rp[u + 1] < rp[u]) return OR_GRAPH;
    for (int64_t i = rp[u]; i < rp[u + 1]; ++i) {
      int32_t v = ci[i];
      if (v < 0 || v >= n || v == u) return OR_GRAPH;
      if (i > rp[u] && ci[i - 1] >= v) return OR_GRAPH;
    }
  }
  for (int32_t u = 0; u < n; ++u)
    for (int64_t i = rp[u]; i < rp[u + 1]; ++i) {
      int32_t v = ci[i];
      if (row_find(ci + rp[v], rp[v + 1] - rp[v], u) < 0) return OR_GRAPH;
    }
  return OR_OK;
}

/* k-th element (0-based) of the closed neighbourhood N[x] in ascending
 * order: the open row with x inserted at its sorted position `at`. */
static int32_t closed_elem(const int32_t* row, int64_t at, int32_t x, int64_t k) {
  if (k < at) return row[k];
  if (k == at) return x;
  return row[k - 1];
}

static int64_t insert_pos(const int32_t* row, int64_t len, int32_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (row[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* |N[u] intersect N[v]| by a two-pointer merge of the two closed sorted
 * lists (Def 2.1 for N[.], Def 2.2 for the numerator of sigma). */
int64_t oracle_closed_count(const int64_t* rp, const int32_t* ci, int32_t u, int32_t v) {
  const int32_t* ru = ci + rp[u];
  const int32_t* rv = ci + rp[v];
  const int64_t du = rp[u + 1] - rp[u], dv = rp[v + 1] - rp[v];
  const int64_t au = insert_pos(ru, du, u), av = insert_pos(rv, dv, v);
  int64_t i = 0, j = 0, c = 0;
  while (i < du + 1 && j < dv + 1) {
    int32_t x = closed_elem(ru, au, u, i), y = closed_elem(rv, av, v, j);
    if (x == y) { ++c; ++i; ++j; }
    else if (x < y) ++i;
    else ++j;
  }
  return c;
}

/* sigma >= p/q  <=>  (c q)^2 >= p^2 a b, with a = |N[u]|, b = |N[v]|
 * (Def 2.2, Def 2.3; ">=" so equality counts as similar). */
int oracle_similar(int64_t c, int64_t a, int64_t b, int64_t p, int64_t q) {
  unsigned __int128 lhs = (unsigned __int128)(uint64_t)(c * q) * (uint64_t)(c * q);
  unsigned __int128 rhs = (unsigned __int128)((uint64_t)p * (uint64_t)p) * (uint64_t)a * (uint64_t)b;
  return lhs >= rhs;
}

/* Closed counts for every arc (CSR order); both arcs of an edge receive the
 * same value.  For each vertex u, the indicator array holds N[u]; each
 * neighbour v whose closed set is not larger than N[u] (ties broken by id)
 * sums the indicator over N[v].  Each edge is therefore counted exactly once,
 * from its endpoint with the larger closed set. */
int oracle_counts_all(int32_t n, const int64_t* rp, const int32_t* ci, int32_t* counts,
                      int threads) {
  if (threads < 1) threads = 1;
  int err = 0;
#pragma omp parallel num_threads(threads)
  {
    unsigned char* mark = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!mark) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int32_t u = 0; u < n; ++u) {
      if (!mark) continue;
      const int64_t du = rp[u + 1] - rp[u];
      mark[u] = 1;
      for (int64_t i = rp[u]; i < rp[u + 1]; ++i) mark[ci[i]] = 1;
      for (int64_t i = rp[u]; i < rp[u + 1]; ++i) {
        const int32_t v = ci[i];
        const int64_t dv = rp[v + 1] - rp[v];
        if (dv > du || (dv == du && v > u)) continue; /* counted from v's side */
        int64_t c = mark[v];
        for (int64_t k = rp[v]; k < rp[v + 1]; ++k) c += mark[ci[k]];
        counts[i] = (int32_t)c;
        counts[rp[v] + row_find(ci + rp[v], dv, u)] = (int32_t)c;
      }
      mark[u] = 0;
      for (int64_t i = rp[u]; i < rp[u + 1]; ++i) mark[ci[i]] = 0;
    }
    free(mark);
  }
  return err ? OR_NOMEM : OR_OK;
}

/* Clustering from given per-arc closed counts (as produced by
 * oracle_counts_all): Defs 2.3-2.6 and the border rule.  labels[n] and
 * roles[n] are outputs. */
int oracle_cluster(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* cnt, int64_t p,
                   int64_t q, int32_t mu, int32_t* labels, uint8_t* roles) {
  if (n < 0 || p < 1 || q < p || q > 0x7fffffffLL || mu < 2 || !labels || !roles)
    return OR_INVAL;
  const int64_t nnz = rp[n];
  uint8_t* sim = (uint8_t*)malloc((size_t)(nnz > 0 ? nnz : 1));
  uint8_t* core = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!sim || !core || !queue) {
    free(sim); free(core); free(queue);
    return OR_NOMEM;
  }
  /* Def 2.3: similarity of every arc. */
  for (int32_t u = 0; u < n; ++u)
    for (int64_t i = rp[u]; i < rp[u + 1]; ++i) {
      const int32_t v = ci[i];
      sim[i] = (uint8_t)oracle_similar(cnt[i], rp[u + 1] - rp[u] + 1, rp[v + 1] - rp[v] + 1, p, q);
    }
  /* Def 2.4: |N_eps[u]| = 1 (u itself) + number of similar neighbours. */
  for (int32_t u = 0; u < n; ++u) {
    int64_t ne = 1;
    for (int64_t i = rp[u]; i < rp[u + 1]; ++i) ne += sim[i];
    core[u] = (uint8_t)(ne >= mu);
  }
  /* Defs 2.5-2.6: breadth-first search over similar core-core edges,
   * seeds in ascending order, so each cluster's label is its smallest core. */
  for (int32_t u = 0; u < n; ++u) labels[u] = -1;
  for (int32_t s = 0; s < n; ++s) {
    if (!core[s] || labels[s] != -1) continue;
    int64_t head = 0, tail = 0;
    labels[s] = s;
    queue[tail++] = s;
    while (head < tail) {
      const int32_t x = queue[head++];
      for (int64_t i = rp[x]; i < rp[x + 1]; ++i) {
        const int32_t v = ci[i];
        if (sim[i] && core[v] && labels[v] == -1) {
          labels[v] = s;
          queue[tail++] = v;
        }
      }
    }
  }
  /* Borders: the minimum label among similar core neighbours. */
  for (int32_t v = 0; v < n; ++v) {
    if (core[v]) { roles[v] = ROLE_CORE; continue; }
    int32_t best = -1;
    for (int64_t i = rp[v]; i < rp[v + 1]; ++i) {
      const int32_t u = ci[i];
      if (core[u] && sim[i] && (best < 0 || labels[u] < best)) best = labels[u];
    }
    roles[v] = best >= 0 ? ROLE_BORDER : ROLE_UNCLASSIFIED;
    labels[v] = best;
  }
  free(sim); free(core); free(queue);
  return OR_OK;
}

/* Def 2.7: a vertex in no cluster is a hub when its neighbours lie in two or
 * more clusters, and an outlier otherwise.  A neighbour's cluster is the label
 * it was given (its own cluster for a core, the minimum label for a border),
 * which is how the classification step of the paper (Alg. 4) reads it.  roles
 * are updated in place: every ROLE_UNCLASSIFIED vertex becomes ROLE_HUB or
 * ROLE_OUTLIER; labels stay -1 for both. */
int oracle_hub_outlier(int32_t n, const int64_t* rp, const int32_t* ci, const int32_t* labels,
                       uint8_t* roles) {
  if (n < 0 || !labels || !roles) return OR_INVAL;
  for (int32_t u = 0; u < n; ++u) {
    if (roles[u] != ROLE_UNCLASSIFIED) continue;
    int32_t first = -1, distinct = 0;
    for (int64_t i = rp[u]; i < rp[u + 1] && distinct < 2; ++i) {
      const int32_t c = labels[ci[i]];
      if (c < 0) continue;
      if (first < 0) { first = c; distinct = 1; }
      else if (c != first) distinct = 2;
    }
    roles[u] = distinct >= 2 ? ROLE_HUB : ROLE_OUTLIER;
  }
  return OR_OK;
}

/* Full clustering: closed counts of every arc, then oracle_cluster.
 * counts (nnz) is an optional output of the per-arc counts (NULL to skip). */
int oracle_scan(int32_t n, const int64_t* rp, const int32_t* ci, int64_t p, int64_t q,
                int32_t mu, int threads, int32_t* labels, uint8_t* roles, int32_t* counts) {
  if (n < 0 || p < 1 || q < p || q > 0x7fffffffLL || mu < 2 || !labels || !roles)
    return OR_INVAL;
  const int64_t nnz = rp[n];
  int32_t* cnt = counts;
  if (!cnt) {
    cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!cnt) return OR_NOMEM;
  }
  int rc = oracle_counts_all(n, rp, ci, cnt, threads);
  if (rc == OR_OK) rc = oracle_cluster(n, rp, ci, cnt, p, q, mu, labels, roles);
  if (!counts) free(cnt);
  return rc;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
