"""scan_run_device_noalloc (per-run buffers in the library's static device
array, no allocation on the call) against scan_run_device on the same graph:
identical labels and roles, on two calls in a row, the second on a smaller
graph (the array keeps the first call's contents), and both equal to the
oracle.  A graph whose run needs more than the array is refused."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import assert_same, note

pytestmark = pytest.mark.gpu


def _device_result(G, n, run, p, q, mu):
    dl = S.scan_device_alloc(4 * max(n, 1))
    dr = S.scan_device_alloc(max(n, 1))
    try:
        run(p, q, mu, dl, dr)
        labels = np.empty(max(n, 1), np.int32)
        roles = np.empty(max(n, 1), np.uint8)
        S.scan_memcpy_d2h(labels, dl, 4 * n)
        S.scan_memcpy_d2h(roles, dr, n)
        return labels[:n], roles[:n]
    finally:
        S.scan_device_free(dl)
        S.scan_device_free(dr)


@pytest.mark.parametrize("hub_outlier", [False, True])
def test_noalloc_matches_scan_run_device(hub_outlier):
    big = gg.rmat(16, 16, seed=2)           # has LDS-hash jobs (worklist in the array)
    small = gg.planted(2000, 10, 0.2, 0.002, 1)
    cases = [(big, (1, 5), 5), (small, (1, 5), 4)]
    for g, (p, q), mu in cases:
        note("noalloc", f"n={g.n} m={g.m} eps={p}/{q} mu={mu} hub_outlier={hub_outlier}")
        with S.Graph.from_csr(g, hub_outlier=hub_outlier) as G:
            nl, nr = _device_result(G, g.n, G.run_device_noalloc, p, q, mu)
            dl, dr = _device_result(G, g.n, G.run_device, p, q, mu)
        assert_same(nl, nr, dl, dr, f"noalloc vs scan_run_device n={g.n}")
        ol, orr = oracle.scan(g, p, q, mu, threads=oracle.max_threads())
        if hub_outlier:
            orr = oracle.hub_outlier(g, ol, orr)
        assert_same(nl, nr, ol, orr, f"noalloc vs oracle n={g.n}")


def test_noalloc_refuses_oversize_run():
    g = gg.from_edges(5_000_000, [])  # 17 bytes per vertex alone exceed the 64 MiB array
    note("noalloc oversize")
    with S.Graph.from_csr(g) as G:
        with pytest.raises(S.ScanError) as ei:
            _device_result(G, g.n, G.run_device_noalloc, 1, 2, 2)
        assert ei.value.code == S.SCAN_E_NOMEM
        # the graph still runs through the allocating entry point
        dl, dr = _device_result(G, g.n, G.run_device, 1, 2, 2)
        assert (dr == 0).all() and (dl == -1).all()
