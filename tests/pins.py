"""Checks that pin the CPU oracle to facts outside itself.

Each check takes an ``oracle.Oracle`` instance so that the same checks can be
run against deliberately broken copies of the oracle (see
``test_oracle_mutants.py``): a plausible mistake anywhere in the oracle must
make at least one of them fail.

Sources of truth used here, none of which is the oracle's own code:
* the paper's worked examples (``tests/golden/paper_example_graph.json``);
* closed forms of sigma on cycles, complete bipartite graphs, stars and
  cliques, including exact-equality cases sigma == eps;
* the brute force of ``bruteforce.py`` (definitions, decimal square roots);
* an independent pipeline from library routines: closed counts from the sparse
  product A*A (scipy), connected components (scipy.sparse.csgraph);
* invariants: triangle identity, monotonicity in eps and mu, relabelling.
"""
from __future__ import annotations

import json
import os
from decimal import Decimal, localcontext
from itertools import combinations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen as gg
from bruteforce import brute_scan, closed_count as bf_closed_count, closed_sets as bf_closed_sets

HUB, OUTLIER = 3, 4

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS_GRID = [(1, 10), (1, 5), (1, 3), (1, 2), (2, 3), (3, 4), (4, 5), (1, 1)]
MU_GRID = [2, 3, 4, 5]


def load_paper_example():
    with open(os.path.join(GOLDEN, "paper_example_graph.json")) as f:
        return json.load(f)


def check_paper_example(orc):
    fx = load_paper_example()
    g = gg.from_edges(fx["n"], fx["edges"])
    ex = fx["sigma_example"]
    u, v = ex["u"], ex["v"]
    deg = g.degrees()
    # Example 3.1 / 4.2: d(v0)=7, d(v1)=4, three common neighbours, c = 2 + 3
    assert deg[u] == 7 and deg[v] == 4
    assert orc.closed_count(g, u, v) == ex["closed_count"] == 5
    cnt = orc.counts(g)
    arc = g.row_ptr[u] + int(np.searchsorted(g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]], v))
    assert cnt[arc] == 5
    a, b = ex["closed_sizes"]
    assert orc.similar(5, a, b, 3, 5)          # 5/sqrt(40) = 0.79 >= 0.6
    assert not orc.similar(5, a, b, 4, 5)      # 0.79 < 0.8
    p, q = fx["eps"]
    labels, roles = orc.scan(g, p, q, fx["mu"])
    assert roles.tolist() == fx["expected_roles"]
    assert labels.tolist() == fx["expected_labels"]
    # N_eps[v0] = {v0, v1, v4, v7} (Example 3.1)
    row = g.col_idx[g.row_ptr[0]:g.row_ptr[1]]
    sims = [int(w) for w, c in zip(row, cnt[g.row_ptr[0]:g.row_ptr[1]])
            if orc.similar(int(c), deg[0] + 1, deg[w] + 1, p, q)]
    assert sorted([0] + sims) == fx["expected_eps_neighbourhood_v0"]
    # Example 2.1 / Def 2.7: v8 is a hub (neighbours v2 and v9 in two clusters), v3 v5 v6 outliers
    ho = orc.hub_outlier(g, labels, roles)
    assert sorted(np.flatnonzero(ho == HUB).tolist()) == fx["expected_hubs"]
    assert sorted(np.flatnonzero(ho == OUTLIER).tolist()) == fx["expected_outliers"]
    keep = roles != 0
    assert np.array_equal(ho[keep], roles[keep])


def cycle(n):
    return gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def complete(n):
    return gg.from_edges(n, list(combinations(range(n), 2)))


def complete_bipartite(s, t):
    return gg.from_edges(s + t, [(i, s + j) for i in range(s) for j in range(t)])


def star(k):
    return gg.from_edges(k + 1, [(0, i) for i in range(1, k + 1)])


def check_closed_forms(orc):
    # Cycle C_n, n >= 4: N[u] and N[u+1] share exactly {u, u+1}: sigma = 2/3.
    for n in range(4, 10):
        g = cycle(n)
        assert set(orc.counts(g).tolist()) == {2}
        lab, rol = orc.scan(g, 2, 3, 3)          # equality: similar; |N_eps| = 3
        assert rol.tolist() == [1] * n and lab.tolist() == [0] * n
        lab, rol = orc.scan(g, 2, 3, 4)          # |N_eps| = 3 < 4
        assert rol.tolist() == [0] * n and lab.tolist() == [-1] * n
        lab, rol = orc.scan(g, 67, 100, 2)       # 0.667 < 0.67
        assert rol.tolist() == [0] * n
    # Triangle C_3 = K_3: sigma = 1.
    assert set(orc.counts(cycle(3)).tolist()) == {3}
    # K_{3,3}: c = 2, |N| = 4 each: sigma = 1/2.
    g = complete_bipartite(3, 3)
    assert set(orc.counts(g).tolist()) == {2}
    lab, rol = orc.scan(g, 1, 2, 4)
    assert rol.tolist() == [1] * 6 and lab.tolist() == [0] * 6
    lab, rol = orc.scan(g, 51, 100, 2)
    assert rol.tolist() == [0] * 6
    # K_{2,5}: sides of closed size 6 and 3: sigma = 2/sqrt(18) = 0.4714
    g = complete_bipartite(2, 5)
    assert set(orc.counts(g).tolist()) == {2}
    lab, rol = orc.scan(g, 47, 100, 2)
    assert rol.tolist() == [1] * 7
    lab, rol = orc.scan(g, 48, 100, 2)
    assert rol.tolist() == [0] * 7
    # Star K_{1,7}: sigma(centre, leaf) = 2/sqrt(2*8) = 1/2 exactly.
    g = star(7)
    assert set(orc.counts(g).tolist()) == {2}
    lab, rol = orc.scan(g, 1, 2, 2)          # leaves: N_eps = {leaf, centre}
    assert rol.tolist() == [1] * 8 and lab.tolist() == [0] * 8
    lab, rol = orc.scan(g, 1, 2, 3)          # only the centre reaches 3
    assert rol.tolist() == [1] + [2] * 7 and lab.tolist() == [0] * 8
    lab, rol = orc.scan(g, 1, 2, 9)
    assert rol.tolist() == [0] * 8
    # K_n: every closed set is the whole vertex set, sigma = 1.
    for n in range(2, 8):
        g = complete(n)
        assert set(orc.counts(g).tolist()) == {n}
        lab, rol = orc.scan(g, 1, 1, n)
        assert rol.tolist() == [1] * n and lab.tolist() == [0] * n
        lab, rol = orc.scan(g, 1, 1, n + 1)
        assert rol.tolist() == [0] * n
    # Path 0-1-2 plus isolated vertex 3: sigma(0,1) = 2/sqrt(6) = 0.816.
    g = gg.from_edges(4, [(0, 1), (1, 2)])
    lab, rol = orc.scan(g, 4, 5, 2)
    assert rol.tolist() == [1, 1, 1, 0] and lab.tolist() == [0, 0, 0, -1]
    lab, rol = orc.scan(g, 82, 100, 2)
    assert rol.tolist() == [0, 0, 0, 0]
    # Two triangles {0,1,2} and {4,5,6}, vertex 3 joined to 2 and 4.  At
    # eps = 1/2: sigma within a triangle side 3/sqrt(12), sigma(2,3) =
    # sigma(3,4) = 2/sqrt(12).  mu = 3 makes 3 a core that joins everything;
    # mu = 4 leaves cores 2 and 4 only, and 3 is a border of both clusters
    # (minimum label 2 wins).
    g = gg.from_edges(7, [(0, 1), (0, 2), (1, 2), (4, 5), (4, 6), (5, 6), (2, 3), (3, 4)])
    check_hub_outlier_closed_form(orc)
    lab, rol = orc.scan(g, 1, 2, 3)
    assert rol.tolist() == [1] * 7 and lab.tolist() == [0] * 7
    lab, rol = orc.scan(g, 1, 2, 4)
    assert rol.tolist() == [2, 2, 1, 2, 1, 2, 2] and lab.tolist() == [2, 2, 2, 2, 4, 4, 4]


def check_hub_outlier_closed_form(orc):
    """Two triangles {0,1,2} and {4,5,6} bridged by 3 (edges 2-3, 3-4), a pendant 7 on 0 and an
    isolated 8.  At eps = 3/4, mu = 3: sigma(0,2) = 3/sqrt(16) = 3/4 exactly (similar), the other
    triangle edges are 3/sqrt(12) or 1, sigma(2,3) = sigma(3,4) = 2/sqrt(12) < 3/4 and sigma(0,7)
    = 2/sqrt(8) < 3/4.  So the triangles are clusters 0 and 4, vertex 3 touches both (hub), the
    pendant touches one (outlier) and the isolated vertex none (outlier), Def 2.7."""
    g = gg.from_edges(9, [(0, 1), (0, 2), (1, 2), (4, 5), (4, 6), (5, 6), (2, 3), (3, 4), (0, 7)])
    lab, rol = orc.scan(g, 3, 4, 3)
    assert rol.tolist() == [1, 1, 1, 0, 1, 1, 1, 0, 0]
    assert lab.tolist() == [0, 0, 0, -1, 4, 4, 4, -1, -1]
    ho = orc.hub_outlier(g, lab, rol)
    assert ho.tolist() == [1, 1, 1, HUB, 1, 1, 1, OUTLIER, OUTLIER]
    # at mu = 4 nothing is a core: no clusters, every vertex an outlier
    lab, rol = orc.scan(g, 3, 4, 4)
    assert orc.hub_outlier(g, lab, rol).tolist() == [OUTLIER] * 9


def expected_hub_outlier(n, edges, labels, roles, clusters):
    """Def 2.7 from the brute force's clusters, two ways: (assigned) a neighbour's cluster is the
    label it was given; (literal) a neighbour counts in every cluster that holds it.  They differ
    only next to a border that lies in several clusters."""
    _, nbr = bf_closed_sets(n, edges)
    member = [{min(w for w in C if roles[w] == 1) for C in clusters if v in C} for v in range(n)]
    assigned, literal = list(roles), list(roles)
    for u in range(n):
        if roles[u] != 0:
            continue
        a = {labels[w] for w in nbr[u] if labels[w] >= 0}
        lit = set().union(*[member[w] for w in nbr[u]]) if nbr[u] else set()
        assigned[u] = HUB if len(a) >= 2 else OUTLIER
        literal[u] = HUB if len(lit) >= 2 else OUTLIER
        if all(len(member[w]) <= 1 for w in nbr[u]):
            assert assigned[u] == literal[u]
    return assigned, literal


def _edges_of(n, mask):
    pairs = list(combinations(range(n), 2))
    return [pairs[k] for k in range(len(pairs)) if (mask >> k) & 1]


def check_against_bruteforce(orc, n, edges, grid=None, literal=False):
    g = gg.from_edges(n, edges)
    cnt = orc.counts(g)
    for u in range(n):
        for k in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col_idx[k])
            want = bf_closed_count(n, edges, u, v)
            assert cnt[k] == want, (n, edges, u, v)
            assert orc.closed_count(g, u, v) == want
    for (p, q), mu in (grid or [(e, m) for e in EPS_GRID for m in MU_GRID]):
        labels, roles, clusters, hub = brute_scan(n, edges, p, q, mu, literal_subsets=literal)
        ol, orr = orc.scan(g, p, q, mu)
        assert orr.tolist() == roles, (n, edges, p, q, mu, orr.tolist(), roles)
        assert ol.tolist() == labels, (n, edges, p, q, mu, ol.tolist(), labels)
        assigned, lit = expected_hub_outlier(n, edges, labels, roles, clusters)
        assert [HUB if h else (OUTLIER if r == 0 else r) for h, r in zip(hub, roles)] == lit
        assert orc.hub_outlier(g, ol, orr).tolist() == assigned, (n, edges, p, q, mu)


def check_bruteforce_exhaustive(orc, nmax=5, literal_upto=4):
    for n in range(1, nmax + 1):
        npairs = n * (n - 1) // 2
        for mask in range(1 << npairs):
            check_against_bruteforce(orc, n, _edges_of(n, mask), literal=(n <= literal_upto))


def check_bruteforce_random(orc, count=60, nmin=6, nmax=12, seed=7):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        dens = float(rng.uniform(0.15, 0.8))
        edges = [(i, j) for i, j in combinations(range(n), 2) if rng.random() < dens]
        grid = [(EPS_GRID[int(rng.integers(len(EPS_GRID)))], int(rng.integers(2, 6)))
                for _ in range(6)]
        check_against_bruteforce(orc, n, edges, grid=grid)


# ---------------------------------------------------------------------------
# Independent pipeline from library routines.

def adjacency(g):
    data = np.ones(g.nnz, dtype=np.int64)
    return sp.csr_matrix((data, g.col_idx.astype(np.int64), g.row_ptr), shape=(g.n, g.n))


def arc_rows(g):
    return np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))


def library_closed_counts(g):
    """c(u,v) = (A^2)_{uv} + 2 for adjacent u != v (common open neighbours
    plus u and v themselves)."""
    A = adjacency(g)
    A2 = (A @ A).tocsr()
    rows, cols = arc_rows(g), g.col_idx.astype(np.int64)
    vals = np.asarray(A2[rows, cols]).ravel() if g.nnz else np.zeros(0, np.int64)
    return vals + 2


def library_similar(c, a, b, p, q):
    """sigma >= p/q from float64 sigma; the few arcs within 1e-9 of eps are
    decided with 60-digit decimals."""
    c = np.asarray(c, dtype=np.float64)
    s = c / np.sqrt(np.asarray(a, np.float64) * np.asarray(b, np.float64))
    e = p / q
    out = s >= e
    close = np.nonzero(np.abs(s - e) < 1e-9)[0]
    with localcontext() as ctx:
        ctx.prec = 60
        for k in close:
            sk = Decimal(int(c[k])) / (Decimal(int(a[k])) * Decimal(int(b[k]))).sqrt()
            out[k] = sk >= Decimal(p) / Decimal(q)
    return out


def library_scan(g, p, q, mu):
    n = g.n
    deg = np.diff(g.row_ptr)
    rows, cols = arc_rows(g), g.col_idx.astype(np.int64)
    c = library_closed_counts(g)
    sim = library_similar(c, deg[rows] + 1, deg[cols] + 1, p, q)
    ne = 1 + np.bincount(rows[sim], minlength=n)
    core = ne >= mu
    keep = sim & core[rows] & core[cols]
    M = sp.csr_matrix((np.ones(int(keep.sum())), (rows[keep], cols[keep])), shape=(n, n))
    ncomp, comp = connected_components(M, directed=False)
    big = np.iinfo(np.int64).max
    comp_min = np.full(ncomp, big, dtype=np.int64)
    np.minimum.at(comp_min, comp[core], np.nonzero(core)[0])
    labels = np.full(n, -1, dtype=np.int64)
    labels[core] = comp_min[comp[core]]
    att = sim & core[cols] & ~core[rows]
    best = np.full(n, big, dtype=np.int64)
    np.minimum.at(best, rows[att], labels[cols[att]])
    border = (~core) & (best != big)
    labels[border] = best[border]
    roles = np.zeros(n, dtype=np.uint8)
    roles[core] = 1
    roles[border] = 2
    return labels.astype(np.int32), roles, c


def check_library_pipeline(orc, g, params):
    lc = library_closed_counts(g)
    oc = orc.counts(g)
    assert np.array_equal(lc, oc)
    for (p, q), mu in params:
        ll, lr, _ = library_scan(g, p, q, mu)
        ol, orr = orc.scan(g, p, q, mu)
        assert np.array_equal(lr, orr), (p, q, mu)
        assert np.array_equal(ll, ol), (p, q, mu)


def check_triangles(orc, g):
    """sum over edges of open common neighbours = 3 * #triangles, and
    #triangles = trace(A^3) / 6."""
    A = adjacency(g).toarray().astype(np.float64)   # exact: entries < 2^53
    trace3 = int(round(np.trace(A @ A @ A)))        # = 6 * #triangles
    oc = orc.counts(g).astype(np.int64)
    # per arc c - 2 open common neighbours; every triangle is seen from 6 arcs
    assert int(oc.sum()) - 2 * g.nnz == trace3


def check_monotone(orc, g):
    """Raising eps or mu never adds a core."""
    prev = None
    for p, q in [(1, 10), (1, 5), (1, 3), (1, 2), (2, 3), (4, 5), (1, 1)]:
        _, r = orc.scan(g, p, q, 3)
        cores = r == 1
        if prev is not None:
            assert not np.any(cores & ~prev)
        prev = cores
    prev = None
    for mu in [2, 3, 4, 6, 10, 20]:
        _, r = orc.scan(g, 1, 5, mu)
        cores = r == 1
        if prev is not None:
            assert not np.any(cores & ~prev)
        prev = cores


def check_relabel(orc, g, seed=11):
    """Roles move with the vertices; the core partition is unchanged."""
    h, perm = gg.permute(g, seed)
    for (p, q), mu in [((1, 5), 3), ((1, 2), 2), ((1, 10), 4)]:
        l0, r0 = orc.scan(g, p, q, mu)
        l1, r1 = orc.scan(h, p, q, mu)
        assert np.array_equal(r1[perm], r0)
        core = r0 == 1
        a, b = l0[core], l1[perm][core]
        # same partition: the label maps are bijective on cores
        pairs = set(zip(a.tolist(), b.tolist()))
        assert len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


def check_components_case(orc, g):
    """eps no larger than every edge's sigma and mu = 2: every non-isolated
    vertex is a core and the clusters are the connected components of G."""
    c = library_closed_counts(g).astype(np.float64)
    deg = np.diff(g.row_ptr)
    rows = arc_rows(g)
    smin = float(np.min(c / np.sqrt((deg[rows] + 1.0) * (deg[g.col_idx] + 1.0))))
    q = 1000
    p = max(1, int(np.floor(smin * q)) - 1)
    labels, roles = orc.scan(g, p, q, 2)
    A = adjacency(g)
    _, comp = connected_components(A, directed=False)
    iso = deg == 0
    assert np.all(roles[~iso] == 1) and np.all(roles[iso] == 0)
    cmin = np.full(comp.max() + 1, g.n, dtype=np.int64)
    np.minimum.at(cmin, comp, np.arange(g.n))
    assert np.array_equal(labels[~iso], cmin[comp][~iso])


def check_validation(orc):
    good = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    assert orc.validate(good) == 0

    class G:
        def __init__(self, n, rp, ci):
            self.n, self.row_ptr, self.col_idx = n, np.array(rp, np.int64), np.array(ci, np.int32)

    assert orc.validate(G(3, [0, 1, 2, 2], [1, 0])) == 0
    assert orc.validate(G(2, [0, 1, 2], [0, 1])) == -2          # self-loops
    assert orc.validate(G(3, [0, 2, 3, 4], [2, 1, 0, 0])) == -2  # unsorted row
    assert orc.validate(G(3, [0, 2, 3, 4], [1, 1, 0, 0])) == -2  # duplicate
    assert orc.validate(G(3, [0, 1, 1, 1], [1])) == -2           # missing reverse arc
    assert orc.validate(G(2, [0, 1, 2], [1, 5])) == -2           # out of range
    assert orc.validate(G(2, [0, 1, 3], [1, 0])) == -2           # offsets past the end


QUICK_CHECKS = [
    check_paper_example,
    check_closed_forms,
    lambda o: check_bruteforce_exhaustive(o, nmax=4, literal_upto=4),
    lambda o: check_bruteforce_random(o, count=25, seed=3),
    lambda o: check_library_pipeline(o, gg.planted(600, 6, 0.3, 0.01, 5),
                                     [((1, 5), 3), ((1, 3), 4), ((1, 2), 2)]),
    lambda o: check_triangles(o, gg.rmat(9, 8, seed=9)),
    check_validation,
]
