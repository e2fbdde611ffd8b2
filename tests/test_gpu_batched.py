"""Batched clustering of many small graphs with per-graph eps and mu: every
graph's result equals the oracle's and scan_run's; the captured HIP graph,
replayed several times with eager work in between, matches the eager run
every time; the autotuner's choice does not change results."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import assert_same, note

pytestmark = pytest.mark.gpu


def _batch(count, seed, n_hi=3000):
    graphs, specs = gg.planted_batch(count, seed=seed, n_hi=n_hi)
    return graphs, [s.eps for s in specs], [s.mu for s in specs]


def test_batch_matches_oracle_per_graph():
    graphs, eps, mus = _batch(150, seed=4)
    # a few extra shapes: empty graph, isolated vertices, a clique, an R-MAT
    graphs += [gg.from_edges(0, []), gg.from_edges(5, []),
               gg.from_edges(70, [(i, j) for i in range(70) for j in range(i + 1, 70)]), gg.rmat(11, 16, seed=9)]
    eps += [(1, 2), (1, 2), (1, 1), (1, 5)]
    mus += [2, 2, 70, 4]
    note(f"batch of {len(graphs)} graphs")
    with S.Batch(graphs, eps, mus) as B:
        labels, roles = B.run(replay=True)
        for k, (g, (p, q), mu, l, r) in enumerate(zip(graphs, eps, mus, B.split(labels), B.split(roles))):
            ol, orr = oracle.scan(g, p, q, mu)
            assert_same(l, r, ol, orr, f"graph {k} eps={p}/{q} mu={mu}")


def test_batch_large_enough_for_ranked_rows():
    """A batch of 70 R-MAT scale-13 graphs: the disjoint union has more than
    2^19 vertices, so the LDS-hash kernel reads the degree-ranked copy of the
    rows of the union, and the graphs have hubs for it to work on."""
    graphs = [gg.rmat(13, 16, seed=100 + k) for k in range(70)]
    assert sum(g.n for g in graphs) > (1 << 19)
    eps = [(1, 2 + k % 9) for k in range(70)]
    mus = [2 + k % 7 for k in range(70)]
    note("batch above 2^19 vertices")
    with S.Batch(graphs, eps, mus) as B:
        labels, roles = B.run(replay=True)
        for k, (g, (p, q), mu, l, r) in enumerate(zip(graphs, eps, mus, B.split(labels), B.split(roles))):
            ol, orr = oracle.scan(g, p, q, mu)
            assert_same(l, r, ol, orr, f"graph {k} eps={p}/{q} mu={mu}")


def test_batch_replays_match_eager():
    graphs, eps, mus = _batch(80, seed=5)
    note("batch replay vs eager")
    with S.Batch(graphs, eps, mus) as B:
        el, er = B.run(replay=False)
        for _ in range(4):
            rl, rr = B.run(replay=True)
            assert np.array_equal(rl, el) and np.array_equal(rr, er)
            el2, er2 = B.run(replay=False)   # eager work between replays
            assert np.array_equal(el2, el) and np.array_equal(er2, er)


def test_batch_equals_scan_run_and_autotune():
    graphs, eps, mus = _batch(40, seed=6, n_hi=8000)
    graphs.append(gg.rmat(14, 16, seed=3))   # gives the last buckets work
    eps.append((1, 10))
    mus.append(3)
    note("batch autotune")
    with S.Batch(graphs, eps, mus, autotune=True) as B:
        lanes, hub = B.config()
        assert all(l in (4, 8, 16, 32, 64) for l in lanes)
        labels, roles = B.run()
        for g, (p, q), mu, l, r in zip(graphs, eps, mus, B.split(labels), B.split(roles)):
            with S.Graph.from_csr(g) as G:
                gl, gr = G.run(p, q, mu)
            assert np.array_equal(gl, l) and np.array_equal(gr, r)
    l1, r1 = S.scan_run_batch(graphs, eps, mus)
    assert np.array_equal(l1, labels) and np.array_equal(r1, roles)


def test_batch_errors():
    g = gg.planted(100, 5, 0.3, 0.02, 1)
    with pytest.raises(S.ScanError):
        S.Batch([g], [(0, 2)], [3])
    with pytest.raises(S.ScanError):
        S.Batch([g], [(1, 2)], [1])
