"""Overlapping calls on one graph: scan_run and scan_run_device from several
threads at once on the same in-memory graph, every result against the
oracle.  A call that finds the graph's per-run buffers in use runs on a buffer
set of its own (scan_graph_device_bytes grows by whole sets); under a device
budget with no room for another set the calls wait for each other instead."""
import threading

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import assert_same, note

pytestmark = pytest.mark.gpu

PARAMS = [((1, 5), 5), ((1, 2), 3), ((3, 10), 4), ((7, 10), 2), ((1, 10), 6), ((2, 5), 5)]


def _expect(g):
    oc = oracle.counts(g, threads=oracle.max_threads())
    return {pm: oracle.cluster(g, oc, pm[0][0], pm[0][1], pm[1]) for pm in PARAMS}


def _in_threads(nt, fn):
    """fn(t) on nt threads released together; re-raises the first failure."""
    start = threading.Barrier(nt)
    errs = []

    def body(t):
        try:
            start.wait()
            fn(t)
        except BaseException as e:  # noqa: BLE001 - reported below
            errs.append(e)

    ts = [threading.Thread(target=body, args=(t,)) for t in range(nt)]
    for x in ts:
        x.start()
    for x in ts:
        x.join()
    if errs:
        raise errs[0]


def _set_bytes(G, g, host):
    """Device bytes of one buffer set of an overlapping call (as the header states them)."""
    b6 = G.stats()["bucket_edges"][6]
    return 17 * g.n + g.m + 4 * b6 + 256 + (5 * g.n if host else 0)


def test_overlapping_host_calls():
    g = gg.rmat(14, 16, seed=31)
    expect = _expect(g)
    with S.Graph.from_csr(g) as G:
        G.run(1, 2, 5)  # the graph's own staging exists from here on
        base = G.device_bytes()
        per_set = _set_bytes(G, g, host=True)
        out = {}

        def work(t):
            for k in range(4):
                (p, q), mu = pm = PARAMS[(t + k) % len(PARAMS)]
                out[(t, k)] = (pm, *G.run(p, q, mu))

        note("rmat14", "6 threads x 4 scan_run")
        _in_threads(6, work)
        for (t, k), (pm, lab, rol) in sorted(out.items()):
            ol, orr = expect[pm]
            assert_same(lab, rol, ol, orr, f"thread {t} call {k} eps={pm[0]} mu={pm[1]}")
        grown = G.device_bytes() - base
        assert grown > 0, "no call overlapped another"
        # one set per call that overlapped, at most one per thread
        assert grown % per_set == 0 and grown // per_set <= 6, (grown, per_set)
        # the sets are kept and taken again: a second round adds none beyond one per thread
        _in_threads(6, work)
        assert G.device_bytes() - base <= 6 * per_set


def test_overlapping_device_calls():
    g = gg.chung_lu(30000, 16.0, 2.2, 2500.0, seed=32)
    expect = _expect(g)
    nt = 5
    bufs = [(S.scan_device_alloc(4 * g.n), S.scan_device_alloc(g.n)) for _ in range(nt)]
    try:
        with S.Graph.from_csr(g) as G:
            base = G.device_bytes()
            out = {}

            def work(t):
                dl, dr = bufs[t]
                for k in range(3):
                    (p, q), mu = pm = PARAMS[(2 * t + k) % len(PARAMS)]
                    G.run_device(p, q, mu, dl, dr)  # returns with the outputs written
                    lab = np.empty(g.n, np.int32)
                    rol = np.empty(g.n, np.uint8)
                    S.scan_memcpy_d2h(lab, dl, 4 * g.n)
                    S.scan_memcpy_d2h(rol, dr, g.n)
                    out[(t, k)] = (pm, lab, rol)

            note("chunglu30k", f"{nt} threads x 3 scan_run_device")
            _in_threads(nt, work)
            for (t, k), (pm, lab, rol) in sorted(out.items()):
                ol, orr = expect[pm]
                assert_same(lab, rol, ol, orr, f"thread {t} call {k} eps={pm[0]} mu={pm[1]}")
            per_set = _set_bytes(G, g, host=False)
            grown = G.device_bytes() - base
            assert grown > 0 and grown % per_set == 0 and grown // per_set <= nt, (grown, per_set)
    finally:
        for dl, dr in bufs:
            S.scan_device_free(dl)
            S.scan_device_free(dr)


def test_calls_wait_when_the_budget_has_no_room():
    # many vertices, few edges: a buffer set (17 n + m + ...) is larger than
    # what a budget equal to the in-memory footprint leaves over
    g = gg.chung_lu(200000, 4.0, 2.2, 1500.0, seed=33)
    expect = _expect(g)
    fp = S.scan_graph_footprint(g.n, g.nnz)
    with S.Graph.from_csr(g, budget=fp) as G:
        G.run(1, 2, 5)
        assert G.stats()["h2d_bytes"] == 0  # the in-memory path
        base = G.device_bytes()
        assert base + _set_bytes(G, g, host=True) > fp, "the budget leaves room for a set: test graph too dense"
        out = {}

        def work(t):
            for k in range(2):
                (p, q), mu = pm = PARAMS[(t + k) % len(PARAMS)]
                out[(t, k)] = (pm, *G.run(p, q, mu))

        note("chunglu200k", "4 threads x 2 scan_run under a full budget")
        _in_threads(4, work)
        for (t, k), (pm, lab, rol) in sorted(out.items()):
            ol, orr = expect[pm]
            assert_same(lab, rol, ol, orr, f"thread {t} call {k} eps={pm[0]} mu={pm[1]}")
        assert G.device_bytes() == base


def test_similarity_and_runs_overlap():
    """scan_similarity holds the graph's own buffers; scan_run calls started
    beside it run on buffer sets of the pool, and both are exact."""
    g = gg.rmat(14, 16, seed=34)
    oc = oracle.counts(g, threads=oracle.max_threads())
    expect = _expect(g)
    with S.Graph.from_csr(g) as G:
        out = {}

        def work(t):
            if t == 0:
                out["counts"] = [G.similarity() for _ in range(3)]
            else:
                for k in range(3):
                    (p, q), mu = pm = PARAMS[(t + k) % len(PARAMS)]
                    out[(t, k)] = (pm, *G.run(p, q, mu))

        note("rmat14", "scan_similarity beside 3 threads of scan_run")
        _in_threads(4, work)
        for c in out.pop("counts"):
            np.testing.assert_array_equal(c, oc)
        for (t, k), (pm, lab, rol) in sorted(out.items()):
            ol, orr = expect[pm]
            assert_same(lab, rol, ol, orr, f"thread {t} call {k} eps={pm[0]} mu={pm[1]}")


def test_partitioned_graph_calls_wait():
    """A partitioned graph has one set of streaming buffers: overlapping calls
    wait for each other, hold no pool, and stay exact."""
    g = gg.rmat(13, 16, seed=35)
    expect = _expect(g)
    n, nnz = g.n, g.nnz
    resident = 8 * (n + 1) + 22 * n + (1 << 20)
    layout = 8 * (n + 1) + 4 * nnz + 13 * (nnz // 2) + 22 * n + (1 << 20)
    maxdeg = int(np.diff(g.row_ptr).max())
    budget = resident + max(int(0.2 * (layout - resident)), 12 * (maxdeg + 64), 1 << 17)
    with S.Graph.from_csr(g, budget=budget) as G:
        out = {}

        def work(t):
            for k in range(2):
                (p, q), mu = pm = PARAMS[(2 * t + k) % len(PARAMS)]
                out[(t, k)] = (pm, *G.run(p, q, mu), G.stats()["h2d_bytes"])

        note("rmat13", f"partitioned at budget {budget}: 3 threads x 2 scan_run")
        _in_threads(3, work)
        for (t, k), (pm, lab, rol, h2d) in sorted(out.items()):
            ol, orr = expect[pm]
            assert_same(lab, rol, ol, orr, f"thread {t} call {k} eps={pm[0]} mu={pm[1]}")
            assert h2d > 0, "the budget did not select the partition-based path"
        assert G.device_bytes() == 0
