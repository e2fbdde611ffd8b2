"""Partition-based path (device budget smaller than the graph): identical
results to the oracle and to the in-memory path, for clustering and for the
per-arc closed counts."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import assert_same, note

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
