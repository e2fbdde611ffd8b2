"""Serving (cached closed counts + re-thresholding, continuous batching):
every answer must equal the oracle's and a plain scan_run, alone and in a mix
of concurrent requests on several graphs."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import assert_same, note

pytestmark = pytest.mark.gpu


def test_serving_matches_oracle_alone_and_in_mix():
    graphs = [gg.rmat(14, 16, seed=11), gg.planted(10000, 50, 0.15, 0.0005, 1),
              gg.rmat(12, 8, seed=12), gg.chung_lu(30000, 20.0, 2.1, 1500.0, seed=13)]
    counts = [oracle.counts(g, threads=oracle.max_threads()) for g in graphs]
    rng = np.random.default_rng(5)
    queries = [(int(rng.integers(len(graphs))), int(rng.integers(1, 10)), 10, int(rng.integers(2, 21)))
               for _ in range(120)]
    note("serving: 4 graphs, 120 queries, 4 slots")
    with S.Server(num_slots=4) as srv:
        gids = [srv.add(g) for g in graphs]
        # alone: one request at a time
        alone = {}
        for gi, p, q, mu in queries[:20]:
            r = srv.submit(gids[gi], p, q, mu)
            alone[(gi, p, q, mu)] = srv.wait(r, gids[gi])[:2]
        # in the mix: everything submitted at once
        reqs = [(srv.submit(gids[gi], p, q, mu), gi, p, q, mu) for gi, p, q, mu in queries]
        for r, gi, p, q, mu in reqs:
            l, ro, lat = srv.wait(r, gids[gi])
            assert lat >= 0
            ol, orr = oracle.cluster(graphs[gi], counts[gi], p, q, mu)
            assert_same(l, ro, ol, orr, f"served graph {gi} eps={p}/{q} mu={mu}")
            if (gi, p, q, mu) in alone:
                al, ar = alone[(gi, p, q, mu)]
                assert np.array_equal(al, l) and np.array_equal(ar, ro)
        info = srv.info()
        assert info["graphs"] == 4 and info["resident_graphs"] == 4
        assert info["completed"] == len(queries) + 20


def test_serving_equals_scan_run():
    g = gg.rmat(16, 16, seed=2)
    note("serving vs scan_run rmat16")
    with S.Server(num_slots=2) as srv, S.Graph.from_csr(g) as G:
        gid = srv.add(g)
        for p, q, mu in [(1, 5, 5), (1, 2, 5), (4, 5, 5), (1, 10, 3), (1, 10, 2)]:
            l, r, _ = srv.wait(srv.submit(gid, p, q, mu), gid)
            gl, gr = G.run(p, q, mu)
            assert np.array_equal(l, gl) and np.array_equal(r, gr)


def test_serving_add_remove_and_errors():
    note("serving add/remove/errors")
    g1 = gg.planted(3000, 10, 0.2, 0.002, 3)
    g2 = gg.rmat(15, 16, seed=4)  # larger: grows the slots' scratch
    with S.Server(num_slots=3) as srv:
        a = srv.add(g1)
        ra = [srv.submit(a, 1, 5, 4) for _ in range(6)]
        b = srv.add(g2)
        rb = [srv.submit(b, 1, 10, 3) for _ in range(6)]
        la = [srv.wait(r, a)[:2] for r in ra]
        lb = [srv.wait(r, b)[:2] for r in rb]
        ol, orr = oracle.scan(g1, 1, 5, 4)
        for l, r in la:
            assert_same(l, r, ol, orr, "g1")
        ol, orr = oracle.scan(g2, 1, 10, 3, threads=oracle.max_threads())
        for l, r in lb:
            assert_same(l, r, ol, orr, "g2")
        srv.remove(a)
        with pytest.raises(S.ScanError) as ei:
            srv.submit(a, 1, 5, 4)
        assert ei.value.code == S.SCAN_E_INVAL
        with pytest.raises(S.ScanError):
            srv.submit(b, 0, 5, 4)
        with pytest.raises(S.ScanError):
            srv.submit(b, 1, 5, 1)
        assert srv.info()["graphs"] == 1


def test_serving_admission_falls_back_to_partitioned_path():
    """A graph that does not fit the server's device budget stays on the host;
    its queries run through the budgeted (partition-based) path with the same
    results."""
    small = gg.rmat(12, 8, seed=21)
    big = gg.rmat(15, 16, seed=22)
    g_small = 8 * (small.n + 1) + 4 * small.nnz + 17 * (small.nnz // 2) + 22 * small.n
    slots = 2 * (18 * big.n + big.nnz // 2)
    budget = g_small + slots + 30 * big.n + (6 << 20)
    note("serving admission budget", budget)
    with S.Server(num_slots=2, budget=budget) as srv:
        a = srv.add(small)
        b = srv.add(big)
        info = srv.info()
        assert info["graphs"] == 2 and info["resident_graphs"] == 1
        for gid, g in ((a, small), (b, big)):
            for p, q, mu in [(1, 5, 4), (1, 10, 3)]:
                l, r, _ = srv.wait(srv.submit(gid, p, q, mu), gid)
                ol, orr = oracle.scan(g, p, q, mu, threads=oracle.max_threads())
                assert_same(l, r, ol, orr, f"admission gid={gid} eps={p}/{q} mu={mu}")


def _served_bytes(g, **opts):
    """Peak device bytes the server reserves for adding g (its admission rule)."""
    return S.scan_graph_footprint(g.n, g.nnz, S.make_opts(**opts)) + 12 * g.m


def test_serving_admission_counts_the_ranked_rows():
    """A graph of more than 2^19 vertices gets a degree-ranked copy of its rows
    when it is created; admission must count it.  A budget that holds the graph
    without that copy (but not with it) keeps the graph on the host."""
    g = gg.rmat(20, 4, seed=23)
    assert g.n > (1 << 19)
    slots = 18 * g.n + g.m  # one slot
    without = _served_bytes(g, hub_ranked=False) + slots
    with_ranked = _served_bytes(g) + slots
    assert with_ranked - without >= 4 * g.nnz
    oc = oracle.counts(g, threads=oracle.max_threads())
    for budget, resident in ((without + (1 << 20), 0), (with_ranked + (1 << 20), 1)):
        note("serving ranked-row admission", budget, resident)
        with S.Server(num_slots=1, budget=budget) as srv:
            gid = srv.add(g)
            assert srv.info()["resident_graphs"] == resident
            assert srv.info()["resident_bytes"] <= budget
            for p, q, mu in [(1, 5, 3), (1, 2, 2)]:
                l, r, _ = srv.wait(srv.submit(gid, p, q, mu), gid)
                ol, orr = oracle.cluster(g, oc, p, q, mu)
                assert_same(l, r, ol, orr, f"ranked admission resident={resident} eps={p}/{q} mu={mu}")


def test_serving_resident_queries_complete_while_fallback_runs():
    """A query on a graph kept on the host runs on the fallback worker; queries
    on resident graphs submitted after it are admitted and completed while it
    runs (no head-of-line blocking), and every answer equals the oracle's."""
    import time

    smalls = [gg.rmat(11, 8, seed=31 + k) for k in range(3)]
    big = gg.rmat(18, 16, seed=34)
    nslots = 4
    resident_need = sum(_served_bytes(g) for g in smalls) + nslots * max(18 * g.n + g.m for g in smalls)
    budget = resident_need + (24 << 20)
    assert _served_bytes(big) > budget - resident_need  # the big graph cannot be resident
    with S.Server(num_slots=nslots, budget=budget) as srv:
        gids = [srv.add(g) for g in smalls]
        b = srv.add(big)
        info = srv.info()
        assert info["resident_graphs"] == len(smalls) and info["graphs"] == len(smalls) + 1
        note("fallback query + resident queries")
        t_fb = time.perf_counter()
        rf = srv.submit(b, 1, 5, 4)
        sub = []
        for k in range(30):
            gi = k % len(smalls)
            sub.append((time.perf_counter(), srv.submit(gids[gi], 1 + k % 9, 10, 2 + k % 7), gi, 1 + k % 9, 2 + k % 7))
        done_res = []
        for t0, r, gi, p, mu in sub:
            l, ro, lat = srv.wait(r, gids[gi])
            done_res.append(t0 + lat * 1e-3)
            ol, orr = oracle.scan(smalls[gi], p, 10, mu)
            assert_same(l, ro, ol, orr, f"resident graph {gi} eps={p}/10 mu={mu}")
        l, ro, lat = srv.wait(rf, b)
        done_fb = t_fb + lat * 1e-3
        ol, orr = oracle.scan(big, 1, 5, 4, threads=oracle.max_threads())
        assert_same(l, ro, ol, orr, "fallback graph")
        assert max(done_res) < done_fb, (max(done_res) - t_fb, done_fb - t_fb)
        # the partitioned graph is kept: a second query of it needs no new build
        l2, ro2, lat2 = srv.wait(srv.submit(b, 1, 5, 4), b)
        assert np.array_equal(l2, l) and np.array_equal(ro2, ro)
        assert srv.info()["resident_bytes"] <= budget
