"""Parity of the HIP path (through the C-ABI) with the CPU oracle: bit-exact
labels, roles and per-arc closed counts."""
import os
from itertools import combinations

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
import pins
from gpu_helpers import assert_groups_whole, assert_same, gpu_counts, gpu_run, note

pytestmark = pytest.mark.gpu

EPS_ALL = [(1, 10), (1, 5), (1, 3), (1, 2), (2, 3), (3, 4), (4, 5), (1, 1)]


def check_graph(g, params, name, counts=True, **opts):
    note(name, f"n={g.n} m={g.m}", opts)
    if counts:
        oc = oracle.counts(g, threads=oracle.max_threads())
        gc = gpu_counts(g, **opts)
        assert np.array_equal(gc, oc), f"{name}: closed counts differ at {np.count_nonzero(gc != oc)} arcs"
    else:
        oc = None
    with S.Graph.from_csr(g, **opts) as G:
        for (p, q), mu in params:
            note(name, f"eps={p}/{q} mu={mu}")
            gl, gr = G.run(p, q, mu)
            assert_groups_whole(G, f"{name} eps={p}/{q} mu={mu}")
            if oc is not None:
                ol, orr = oracle.cluster(g, oc, p, q, mu)
            else:
                ol, orr = oracle.scan(g, p, q, mu, threads=oracle.max_threads())
            assert_same(gl, gr, ol, orr, f"{name} eps={p}/{q} mu={mu}")


def test_paper_example():
    fx = pins.load_paper_example()
    g = gg.from_edges(fx["n"], fx["edges"])
    note("paper example")
    gl, gr = gpu_run(g, *fx["eps"], fx["mu"])
    assert gr.tolist() == fx["expected_roles"]
    assert gl.tolist() == fx["expected_labels"]
    c = gpu_counts(g)
    k = int(np.searchsorted(g.col_idx[g.row_ptr[0]:g.row_ptr[1]], 1))
    assert c[g.row_ptr[0] + k] == 5  # (2 + 3) of Example 3.1


def test_closed_forms():
    for n in range(4, 9):
        note("cycle", n)
        gl, gr = gpu_run(pins.cycle(n), 2, 3, 3)
        assert gr.tolist() == [1] * n and gl.tolist() == [0] * n
        gl, gr = gpu_run(pins.cycle(n), 67, 100, 2)
        assert gr.tolist() == [0] * n
    note("K33")
    gl, gr = gpu_run(pins.complete_bipartite(3, 3), 1, 2, 4)
    assert gr.tolist() == [1] * 6
    note("star7")
    gl, gr = gpu_run(pins.star(7), 1, 2, 3)
    assert gr.tolist() == [1] + [2] * 7 and gl.tolist() == [0] * 8
    for n in (2, 5, 70, 130):   # K_70 and K_130 use the one-wave-per-edge kernel
        note("clique", n)
        g = pins.complete(n)
        gl, gr = gpu_run(g, 1, 1, n)
        assert gr.tolist() == [1] * n and gl.tolist() == [0] * n
        gl, gr = gpu_run(g, 1, 1, n + 1)
        assert gr.tolist() == [0] * n
        assert set(gpu_counts(g).tolist()) == {n}


def test_small_graphs_against_oracle():
    rng = np.random.default_rng(12)
    cases = []
    for n in range(1, 6):
        npairs = n * (n - 1) // 2
        masks = range(1 << npairs) if npairs <= 6 else rng.choice(1 << npairs, 40, replace=False)
        for mask in masks:
            cases.append((n, pins._edges_of(n, int(mask))))
    for _ in range(60):
        n = int(rng.integers(6, 13))
        dens = float(rng.uniform(0.2, 0.8))
        cases.append((n, [(i, j) for i, j in combinations(range(n), 2) if rng.random() < dens]))
    note(f"{len(cases)} small graphs")
    for n, edges in cases:
        g = gg.from_edges(n, edges)
        oc = oracle.counts(g)
        with S.Graph.from_csr(g) as G:
            assert np.array_equal(G.similarity(), oc), (n, edges)
            for (p, q) in EPS_ALL[::2]:
                for mu in (2, 3, 5):
                    gl, gr = G.run(p, q, mu)
                    ol, orr = oracle.cluster(g, oc, p, q, mu)
                    assert_same(gl, gr, ol, orr, f"n={n} edges={edges} eps={p}/{q} mu={mu}")


def test_planted_config_A():
    """Planted partition, n = 10,000 in 50 blocks, p_in 0.15, p_out 0.0005; eps 1/2
    is degenerate (no similar edge), so 1/5 and 1/10 are added."""
    g = gg.planted(10000, 50, 0.15, 0.0005, 1)
    check_graph(g, [((1, 2), 5), ((1, 5), 5), ((1, 10), 5), ((1, 5), 2), ((1, 5), 12)], "planted-A")


def test_planted_pruning_off_is_identical():
    g = gg.planted(10000, 50, 0.15, 0.0005, 1)
    note("planted pruning on/off")
    with S.Graph.from_csr(g, pruning=True) as A, S.Graph.from_csr(g, pruning=False) as B:
        for (p, q), mu in [((1, 5), 5), ((1, 10), 5), ((1, 5), 3)]:
            la, ra = A.run(p, q, mu)
            lb, rb = B.run(p, q, mu)
            assert np.array_equal(ra, rb) and np.array_equal(la, lb)


@pytest.mark.parametrize("scale", [14, 16, 18])
def test_rmat(scale):
    g = gg.rmat(scale, 16, seed=2)
    check_graph(g, [((1, 10), 5), ((1, 5), 5), ((1, 2), 5), ((4, 5), 5), ((1, 5), 2), ((1, 10), 3)],
                f"rmat{scale}")


def test_rmat_relabelled():
    g, _ = gg.permute(gg.rmat(16, 16, seed=2), 3)
    check_graph(g, [((1, 5), 5), ((1, 10), 3)], "rmat16-permuted")


def test_chung_lu():
    g = gg.chung_lu(200000, 30.0, 2.1, 4000.0, seed=3)
    check_graph(g, [((1, 10), 3), ((1, 5), 5), ((1, 2), 10)], "chung-lu-200k")


def test_repeated_runs_identical():
    g = gg.rmat(16, 16, seed=5)
    note("determinism rmat16")
    with S.Graph.from_csr(g) as G:
        ref = G.run(1, 10, 3)
        for _ in range(5):
            l, r = G.run(1, 10, 3)
            assert np.array_equal(l, ref[0]) and np.array_equal(r, ref[1])


def test_edge_cases():
    note("empty graph")
    g0 = gg.from_edges(0, [])
    with S.Graph.from_csr(g0) as G:
        l, r = G.run(1, 2, 2)
        assert l.size == 0 and r.size == 0
        assert G.similarity().size == 0
    note("isolated vertices")
    g1 = gg.from_edges(7, [])
    l, r = gpu_run(g1, 1, 2, 2)
    assert l.tolist() == [-1] * 7 and r.tolist() == [0] * 7
    note("single edge")
    l, r = gpu_run(gg.from_edges(3, [(0, 2)]), 1, 1, 2)
    assert l.tolist() == [0, -1, 0] and r.tolist() == [1, 0, 1]
    note("big star")   # one hub of degree 100,000: skewed pairs in the smallest bucket
    k = 100000
    star = gg.from_edges(k + 1, [(0, i) for i in range(1, k + 1)])
    check_graph(star, [((1, 2), 2), ((1, 500), 2), ((1, 1000), 3)], "star100k")
    note("two hubs sharing leaves")  # hub-hub edge in the one-wave bucket
    e = [(0, 1)] + [(0, i) for i in range(2, 3000)] + [(1, i) for i in range(1000, 5000)]
    check_graph(gg.from_edges(5000, e), [((1, 2), 2), ((1, 10), 3), ((1, 5), 1000)], "two-hubs")


def test_invalid_inputs():
    note("invalid inputs")
    bad = [
        (2, np.array([0, 1, 2]), np.array([0, 1])),          # self-loops
        (3, np.array([0, 2, 3, 4]), np.array([2, 1, 0, 0])),  # unsorted row
        (3, np.array([0, 2, 3, 4]), np.array([1, 1, 0, 0])),  # duplicate
        (3, np.array([0, 1, 1, 2]), np.array([1, 0])),        # missing reverse arc
        (2, np.array([0, 1, 2]), np.array([1, 5])),           # id out of range
    ]
    for n, rp, ci in bad:
        with pytest.raises(S.ScanError) as ei:
            S.scan_graph_create(n, int(rp[-1]), rp, ci)
        assert ei.value.code == S.SCAN_E_GRAPH
    with pytest.raises(S.ScanError) as ei:
        S.scan_graph_create(2, 2, np.array([0, 1, 3]), np.array([1, 0, 0]))
    assert ei.value.code == S.SCAN_E_GRAPH
    g = gg.from_edges(4, [(0, 1), (1, 2)])
    with S.Graph.from_csr(g) as G:
        for p, q, mu in [(0, 2, 2), (3, 2, 2), (1, 2, 1)]:
            with pytest.raises(S.ScanError) as ei:
                G.run(p, q, mu)
            assert ei.value.code == S.SCAN_E_INVAL
        with pytest.raises(S.ScanError) as ei:
            G.run(1, 2_000_000_000, 2)
        assert ei.value.code == S.SCAN_E_RANGE
        l, r = G.run(2, 4, 2)           # eps given unreduced is reduced by gcd
        l2, r2 = G.run(1, 2, 2)
        assert np.array_equal(l, l2) and np.array_equal(r, r2)


def test_device_entry_points():
    g = gg.planted(5000, 25, 0.2, 0.001, 7)
    note("device entry points")
    with S.Graph.from_csr(g) as G:
        dl = S.scan_device_alloc(4 * g.n)
        dr = S.scan_device_alloc(g.n)
        dc = S.scan_device_alloc(4 * g.nnz)
        try:
            G.run_device(1, 5, 4, dl, dr)
            l = np.empty(g.n, np.int32)
            r = np.empty(g.n, np.uint8)
            S.scan_memcpy_d2h(l, dl, 4 * g.n)
            S.scan_memcpy_d2h(r, dr, g.n)
            hl, hr = G.run(1, 5, 4)
            assert np.array_equal(l, hl) and np.array_equal(r, hr)
            S.scan_similarity_device(G.handle, dc)
            c = np.empty(g.nnz, np.int32)
            S.scan_memcpy_d2h(c, dc, 4 * g.nnz)
            assert np.array_equal(c, G.similarity())
        finally:
            for p in (dl, dr, dc):
                S.scan_device_free(p)


def test_device_copy_calibration_kernel():
    note("scan_device_copy")
    nbytes = (3 << 20) + 48
    src = np.random.default_rng(5).integers(0, 256, nbytes, dtype=np.uint8)
    ds = S.scan_device_alloc(nbytes)
    dd = S.scan_device_alloc(nbytes)
    try:
        S.scan_memcpy_h2d(ds, src, nbytes)
        ms = S.scan_device_copy(dd, ds, nbytes, iters=2)
        out = np.empty(nbytes, np.uint8)
        S.scan_memcpy_d2h(out, dd, nbytes)
        assert np.array_equal(out, src) and ms > 0
        with pytest.raises(S.ScanError):
            S.scan_device_copy(dd, ds, nbytes - 8)
        with pytest.raises(S.ScanError):
            S.scan_device_copy(dd, ds, nbytes, iters=0)
        assert S.scan_h2d_rate(1 << 22, 2) > 0
        with pytest.raises(S.ScanError):
            S.scan_h2d_rate(0, 1)
    finally:
        S.scan_device_free(ds)
        S.scan_device_free(dd)


def test_stats_are_consistent():
    g = gg.rmat(16, 16, seed=2)
    note("stats rmat16")
    with S.Graph.from_csr(g, timing=True) as G:
        G.run(1, 5, 5)
        st = G.stats()
        assert st["edges"] == g.m
        assert sum(st["bucket_edges"]) == g.m
        assert st["ms_total"] > 0
        assert sum(st["cores_bucket_evaluated"]) == st["evaluated"]["cores"]
        assert st["evaluated"]["cores"] + st["bounded"]["cores"] <= g.m


@pytest.mark.parametrize("ranked", [False, True])
def test_rmat20_permuted(ranked):
    """R-MAT scale 20 with shuffled ids (no correlation between id and degree),
    above the size at which the LDS-hash kernel reads degree-ranked rows: the
    same counts and clusterings with and without them."""
    g, _ = gg.permute(gg.rmat(20, 16, seed=4), 7)
    check_graph(g, [((1, 5), 5), ((1, 2), 3), ((4, 5), 2)], f"rmat20-permuted-ranked{int(ranked)}", hub_ranked=ranked)


@pytest.mark.skipif(os.environ.get("SCAN_SKIP_FULL") == "1", reason="full-size case disabled")
def test_rmat22_full_size():
    """R-MAT scale 22, edge factor 16: every arc count and every label/role at
    eps 1/5, 1/2, 4/5 (and 1/10), mu 5, in the launch configuration the
    benchmark times."""
    note("rmat22 generate")
    g = gg.rmat(22, 16, seed=2)
    check_graph(g, [((1, 5), 5), ((1, 2), 5), ((4, 5), 5), ((1, 10), 5)], "rmat22", timing=True)


def windowed_hub_graph(seed=5, hub_deg=20000, heavy=300, extra=150):
    """Vertex 0 is adjacent to 1..hub_deg (several LDS windows); vertices
    1..heavy get `extra` more neighbours inside 1..hub_deg, so their edges to
    the hub have a smaller side of degree > 64 and share many neighbours with
    it across every window."""
    rng = np.random.default_rng(seed)
    edges = [(0, i) for i in range(1, hub_deg + 1)]
    for u in range(1, heavy + 1):
        for w in rng.choice(np.arange(1, hub_deg + 1), size=extra, replace=False):
            if int(w) != u:
                edges.append((u, int(w)))
    return gg.from_edges(hub_deg + 1, edges)


def test_windowed_hub():
    g = windowed_hub_graph()
    check_graph(g, [((1, 10), 2), ((1, 5), 3), ((1, 20), 5), ((1, 100), 2)], "windowed-hub")


def test_full_survivor_batch():
    """More heavy in-edges of one hub than a table fill takes (every one of them
    intersected, all in one window), so a fill holds a full batch of active
    survivors."""
    g = windowed_hub_graph(seed=9, hub_deg=3000, heavy=1400, extra=120)
    check_graph(g, [((1, 10), 2), ((1, 5), 3), ((1, 4), 5), ((1, 1), 2)], "full-survivor-batch")
    check_graph(g, [((1, 5), 3)], "full-survivor-batch-exhaustive", counts=False, pruning=False)


def spread_hub_graph(seed=11, heavy=400):
    """Vertex 0 has a neighbourhood whose ids are dense in some ranges and
    sparse in others, so the LDS-hash kernel takes it as a bitmap window
    (ids 1 .. 9000), hash windows (2^20, 2^20 + 1 and 33000 ids spread over
    2^24 ids from 2^21 on, a few hundred per bitmap's worth of ids) and a
    bitmap window again (the last spread ids with 6000 consecutive ids just
    after them).  Heavy neighbours of vertex 0 get
    100 .. 300 more neighbours inside its neighbourhood and 0 .. 200 private
    leaves, so their edges to the hub have a smaller side of degree > 64,
    span every window and range from similar to dissimilar."""
    rng = np.random.default_rng(seed)
    spread = 2 ** 21 + rng.choice(2 ** 24, size=33000, replace=False)
    dense = 2 ** 21 + 2 ** 24 + 1000 + np.arange(6000)
    hub_nbrs = np.unique(np.concatenate([np.arange(1, 9001), [2 ** 20, 2 ** 20 + 1], spread, dense]))
    leaf = int(dense[-1]) + 1
    edges = [(0, int(w)) for w in hub_nbrs]
    for u in rng.choice(hub_nbrs, size=heavy, replace=False):
        n_in, n_out = int(rng.integers(100, 301)), int(rng.integers(0, 201))
        for w in rng.choice(hub_nbrs, size=n_in, replace=False):
            if int(w) != int(u):
                edges.append((int(u), int(w)))
        for _ in range(n_out):
            edges.append((int(u), leaf))
            leaf += 1
    return gg.from_edges(leaf, edges)


def crowded_bucket_graph(seed=13, n=1 << 19, crowd=48, spread=700, heavy=300):
    """Vertex 0 has a few hundred neighbours (one sparse hash window of the
    LDS-hash kernel) of which `crowd` share the first bucket of the set's
    multiplicative hash, so all but four of them are placed in their second
    bucket (or beyond), and probes of ids hashing to the crowded bucket read
    further than the first bucket.  Heavy neighbours link to many of these ids,
    crowded ones included, so their edges to vertex 0 need the lookups."""
    rng = np.random.default_rng(seed)
    x = np.arange(1, n, dtype=np.uint64)
    b1 = ((x * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(19)
    target = int(b1[rng.integers(len(b1))])
    crowded = x[b1 == target][:crowd].astype(np.int64)
    others = rng.choice(np.setdiff1d(np.arange(1, n), crowded), size=spread, replace=False)
    hub_nbrs = np.unique(np.concatenate([crowded, others]))
    edges = [(0, int(w)) for w in hub_nbrs]
    for u in rng.choice(hub_nbrs, size=heavy, replace=False):
        picks = np.unique(np.concatenate([rng.choice(crowded, size=crowd // 2, replace=False),
                                          rng.choice(hub_nbrs, size=int(rng.integers(60, 200)), replace=False)]))
        for w in picks:
            if int(w) != int(u):
                edges.append((int(u), int(w)))
        # ids that hash to the crowded bucket but are not neighbours of vertex 0
        for w in x[b1 == target][crowd:crowd + 8]:
            edges.append((int(u), int(w)))
    return gg.from_edges(n, edges)


def test_crowded_hash_bucket():
    g = crowded_bucket_graph()
    check_graph(g, [((1, 4), 2), ((1, 3), 3), ((1, 6), 5), ((1, 10), 2)], "crowded-bucket")
    check_graph(g, [((1, 4), 3)], "crowded-bucket-exhaustive", counts=False, pruning=False)


def bitmap_edge_graph(seed=17, bits=1 << 19, heavy=200):
    """Vertex 0's row is 6000 consecutive ids from 1 on plus the ids 1 + bits - 1
    (the last id a bitmap window starting at id 1 covers) and 1 + bits (the
    first it does not), so the row is a bitmap window followed by a short hash
    window.  Heavy neighbours link to both boundary ids, to ids just past them
    that are not in the row, and to many row ids, so probes hit every edge of
    the bitmap's id range."""
    rng = np.random.default_rng(seed)
    last, first_out = 1 + bits - 1, 1 + bits
    hub_nbrs = np.concatenate([np.arange(1, 6001), [last, first_out]])
    n = first_out + 8
    edges = [(0, int(w)) for w in hub_nbrs]
    for u in rng.choice(np.arange(1, 6001), size=heavy, replace=False):
        picks = set(int(w) for w in rng.choice(hub_nbrs, size=int(rng.integers(80, 200)), replace=False))
        picks |= {last, first_out, first_out + 1, first_out + 2, 6001}
        picks.discard(int(u))
        edges += [(int(u), w) for w in sorted(picks)]
    return gg.from_edges(n, edges)


@pytest.mark.parametrize("ranked", [False, True])
def test_bitmap_window_edges(ranked):
    g = bitmap_edge_graph()
    check_graph(g, [((1, 8), 2), ((1, 5), 3), ((1, 12), 4)], f"bitmap-edge-ranked{int(ranked)}", hub_ranked=ranked)
    check_graph(g, [((1, 8), 3)], f"bitmap-edge-ranked{int(ranked)}-exhaustive", counts=False, pruning=False,
                hub_ranked=ranked)


@pytest.mark.parametrize("ranked", [False, True])
def test_bitmap_and_hash_windows(ranked):
    """With the rows as given the hub's row is taken as bitmap, hash and
    bitmap windows; with the rows renamed by degree rank (the graph is large
    enough for the renaming) its neighbours move into a narrow id range."""
    g = spread_hub_graph()
    check_graph(g, [((1, 12), 2), ((1, 16), 3), ((1, 25), 5), ((1, 40), 2)], f"spread-hub-ranked{int(ranked)}",
                hub_ranked=ranked)
    check_graph(g, [((1, 16), 3)], f"spread-hub-ranked{int(ranked)}-exhaustive", counts=False, pruning=False,
                hub_ranked=ranked)


@pytest.mark.parametrize("name,gen", [
    ("rmat16", lambda: gg.rmat(16, 16, seed=2)),
    ("spread-hub", spread_hub_graph),
    ("windowed-hub", windowed_hub_graph),
    ("planted-A", lambda: gg.planted(10000, 50, 0.15, 0.0005, 1)),
])
def test_strategies_identical(name, gen):
    """The LDS-hash kernel and the binary-search kernel give the same counts
    and the same clustering."""
    g = gen()
    note("strategies", name)
    with S.Graph.from_csr(g, strategy=0) as A, S.Graph.from_csr(g, strategy=1) as B:
        assert np.array_equal(A.similarity(), B.similarity())
        for (p, q), mu in [((1, 10), 3), ((1, 5), 5), ((1, 2), 2)]:
            la, ra = A.run(p, q, mu)
            lb, rb = B.run(p, q, mu)
            assert np.array_equal(ra, rb) and np.array_equal(la, lb), (name, p, q, mu)
