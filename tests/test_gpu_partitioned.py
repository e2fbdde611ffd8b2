"""Partition-based path (device budget smaller than the graph): identical
results to the oracle and to the in-memory path, for clustering and for the
per-arc closed counts."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import assert_groups_whole, assert_same, note

pytestmark = pytest.mark.gpu


def _budget_for(g, frac):
    """A device budget that holds the per-vertex state but only `frac` of the
    in-memory layout, so the run must stream blocks."""
    n, nnz = g.n, g.nnz
    resident = 8 * (n + 1) + 22 * n + (1 << 20)
    layout = 8 * (n + 1) + 4 * nnz + 13 * (nnz // 2) + 22 * n + (1 << 20)
    return int(resident + frac * (layout - resident))


@pytest.mark.parametrize("name,gen,frac", [
    ("chunglu-200k", lambda: gg.chung_lu(200000, 30.0, 2.1, 4000.0, seed=3), 0.08),
    ("rmat16", lambda: gg.rmat(16, 16, seed=2), 0.15),
    ("planted-A", lambda: gg.planted(10000, 50, 0.15, 0.0005, 1), 0.3),
])
def test_partitioned_matches_oracle(name, gen, frac):
    g = gen()
    budget = _budget_for(g, frac)
    note("partitioned", name, f"budget={budget}")
    oc = oracle.counts(g, threads=oracle.max_threads())
    with S.Graph.from_csr(g, budget=budget, timing=True) as P:
        assert np.array_equal(P.similarity(), oc)
        for (p, q), mu in [((1, 10), 3), ((1, 5), 5), ((1, 2), 2), ((1, 5), 2)]:
            note(name, f"eps={p}/{q} mu={mu}")
            gl, gr = P.run(p, q, mu)
            ol, orr = oracle.cluster(g, oc, p, q, mu)
            assert_same(gl, gr, ol, orr, f"partitioned {name} eps={p}/{q} mu={mu}")
            st = P.stats()
            assert st["h2d_bytes"] > 0


def test_partitioned_equals_in_memory_and_pruning_off():
    g = gg.rmat(15, 16, seed=7)
    budget = _budget_for(g, 0.1)
    note("partitioned vs in-memory rmat15")
    with S.Graph.from_csr(g) as M, S.Graph.from_csr(g, budget=budget) as P, \
            S.Graph.from_csr(g, budget=budget, pruning=False) as Q:
        for (p, q), mu in [((1, 10), 4), ((1, 5), 5), ((3, 10), 3)]:
            ml, mr = M.run(p, q, mu)
            pl, pr = P.run(p, q, mu)
            ql, qr = Q.run(p, q, mu)
            assert np.array_equal(ml, pl) and np.array_equal(mr, pr)
            assert np.array_equal(ml, ql) and np.array_equal(mr, qr)


def test_partitioned_budget_errors():
    g = gg.rmat(12, 16, seed=1)
    note("partitioned budget errors")
    with pytest.raises(S.ScanError) as ei:
        S.Graph.from_csr(g, budget=1024)
    assert ei.value.code == S.SCAN_E_NOMEM
    bad_rp = np.array([0, 1, 1, 2], np.int64)
    bad_ci = np.array([1, 0], np.int32)  # 0->1 without 1->0 is fine, 2->0 has no reverse
    with pytest.raises(S.ScanError) as ei:
        S.scan_graph_create(3, 2, bad_rp, bad_ci, S.make_opts(budget=64))
    assert ei.value.code in (S.SCAN_E_GRAPH, S.SCAN_E_NOMEM)


def _hub_graph_budget(g, blocks):
    """A budget whose row buffer holds the largest row but about 1/blocks of
    the arcs per block, so the rows are streamed in several blocks."""
    n, nnz = g.n, g.nnz
    resident = 8 * (n + 1) + 22 * n + (1 << 20)
    maxdeg = int(g.degrees().max())
    blk = max(maxdeg + 1, nnz // blocks)
    # part of the budget after the resident state: a quarter for the chunk
    # buffers, the rest for a row buffer of two blocks (8 bytes per block arc)
    rest = int(blk * 8 / 0.75) + 4096
    return resident + rest


@pytest.mark.parametrize("name", ["windowed-hub", "spread-hub", "bitmap-edge"])
def test_partitioned_hub_windows_in_a_later_block(name):
    """Hub rows that the LDS-hash kernel takes as several hash and bitmap
    windows, streamed as block rows: the graphs of the in-memory window tests
    with their ids reversed, so that the hub is the last vertex and its row
    sits in the last block, shifted in the device row buffer."""
    import test_gpu_parity as tp

    gen = {"windowed-hub": tp.windowed_hub_graph, "spread-hub": tp.spread_hub_graph,
           "bitmap-edge": tp.bitmap_edge_graph}[name]
    g = gg.reverse_ids(gen())
    budget = _hub_graph_budget(g, 4)
    note("partitioned hub windows", name, f"n={g.n} m={g.m} budget={budget}")
    oc = oracle.counts(g, threads=oracle.max_threads())
    params = [((1, 10), 2), ((1, 5), 3), ((1, 16), 3), ((1, 40), 2)]
    for ranked in (True, False):
        with S.Graph.from_csr(g, budget=budget, hub_ranked=ranked) as P:
            assert np.array_equal(P.similarity(), oc), f"{name}: partitioned counts differ"
            assert P.stats()["h2d_bytes"] > g.nnz * 4  # rows were streamed
            for (p, q), mu in params:
                gl, gr = P.run(p, q, mu)
                assert_groups_whole(P, f"partitioned {name} eps={p}/{q} mu={mu}")
                ol, orr = oracle.cluster(g, oc, p, q, mu)
                assert_same(gl, gr, ol, orr, f"partitioned {name} eps={p}/{q} mu={mu}")


def test_partitioned_chung_lu_with_large_hubs():
    """Chung-Lu with degrees up to 20,000 (hub rows of several LDS windows)
    under a budget of a few blocks."""
    g = gg.chung_lu(400000, 30.0, 2.1, 20000.0, seed=8)
    assert int(g.degrees().max()) > 2 * 4096
    budget = _budget_for(g, 0.12)
    note("partitioned chung-lu large hubs", f"m={g.m} budget={budget}")
    oc = oracle.counts(g, threads=oracle.max_threads())
    with S.Graph.from_csr(g, budget=budget) as P:
        assert np.array_equal(P.similarity(), oc)
        for (p, q), mu in [((1, 10), 3), ((1, 5), 4), ((1, 2), 2)]:
            gl, gr = P.run(p, q, mu)
            ol, orr = oracle.cluster(g, oc, p, q, mu)
            assert_same(gl, gr, ol, orr, f"partitioned chung-lu-400k eps={p}/{q} mu={mu}")
