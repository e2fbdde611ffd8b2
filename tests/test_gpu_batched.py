"""Batched clustering of many small graphs with per-graph eps and mu in one
persistent kernel: every graph's result equals the oracle's and scan_run's;
the captured HIP graph, replayed several times with eager work in between,
matches the eager run every time; new per-graph parameters take effect
without a new capture; the autotuner's choice does not change results; a
run whose blocks wait too long for work items is reported, not hung."""
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


def test_batch_of_skewed_graphs():
    """A batch of 70 R-MAT scale-13 graphs (more than 2^19 vertices in the
    union): hubs with degrees in the hundreds and thousands put edges in every
    degree bucket, including the last two."""
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
        lanes, tile = B.config()
        assert all(l in (4, 8, 16, 32, 64) for l in lanes)
        assert tile in (1024, 2048, 4096, 8192, 16384)
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


def test_batch_new_params_without_recapture():
    graphs, eps, mus = _batch(60, seed=7)
    note("batch set_params")
    rng = np.random.default_rng(3)
    with S.Batch(graphs, eps, mus) as B:
        for rnd in range(3):
            if rnd:
                eps = [(int(rng.integers(1, 5)), 5) for _ in graphs]
                mus = [int(rng.integers(2, 11)) for _ in graphs]
                B.set_params(eps, mus)
            labels, roles = B.run(replay=True)
            for k, (g, (p, q), mu, l, r) in enumerate(zip(graphs, eps, mus, B.split(labels), B.split(roles))):
                ol, orr = oracle.scan(g, p, q, mu)
                assert_same(l, r, ol, orr, f"round {rnd} graph {k} eps={p}/{q} mu={mu}")
        with pytest.raises(S.ScanError):
            B.set_params([(0, 5)] * len(graphs), mus)


def test_batch_hub_outlier_roles():
    graphs, eps, mus = _batch(40, seed=8)
    note("batch hub/outlier")
    with S.Batch(graphs, eps, mus, hub_outlier=True) as B:
        labels, roles = B.run(replay=True)
        for k, (g, (p, q), mu, l, r) in enumerate(zip(graphs, eps, mus, B.split(labels), B.split(roles))):
            ol, orr = oracle.scan(g, p, q, mu)
            orr = oracle.hub_outlier(g, ol, orr)
            assert_same(l, r, ol, orr, f"hub/outlier graph {k}")


def test_batch_watchdog_reports_an_abandoned_run(monkeypatch):
    """With the kernel's wait for a work item limited to nothing, blocks that
    find their item not yet written give up at once: every block returns, and
    the run is reported as SCAN_E_DEVICE instead of hanging."""
    graphs, eps, mus = _batch(200, seed=9)
    monkeypatch.setenv("SCAN_BATCH_WATCHDOG_US", "0")
    note("batch watchdog")
    with S.Batch(graphs, eps, mus) as B:
        with pytest.raises(S.ScanError) as ei:
            for _ in range(20):  # some run has a block arrive before its item
                B.run(replay=True)
        assert ei.value.code == S.SCAN_E_DEVICE
    monkeypatch.delenv("SCAN_BATCH_WATCHDOG_US")
    with S.Batch(graphs, eps, mus) as B:  # the default wait
        labels, roles = B.run(replay=True)
        for k in (0, 57, 199):
            ol, orr = oracle.scan(graphs[k], *eps[k], mus[k])
            assert_same(B.split(labels)[k], B.split(roles)[k], ol, orr, f"graph {k} after watchdog test")
