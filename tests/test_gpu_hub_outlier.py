"""Hub / outlier classification (Def 2.7) on the GPU against the oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2311_12281_amd as S
from gpu_helpers import note

pytestmark = pytest.mark.gpu


def _expect(g, p, q, mu):
    ol, orr = oracle.scan(g, p, q, mu)
    return ol, oracle.hub_outlier(g, ol, orr)


def _check(g, p, q, mu, **opts):
    el, er = _expect(g, p, q, mu)
    with S.Graph.from_csr(g, hub_outlier=True, **opts) as G:
        l, r = G.run(p, q, mu)
    assert np.array_equal(l, el)
    assert np.array_equal(r, er), np.flatnonzero(r != er)[:10]
    return er


def test_paper_example_hubs_and_outliers():
    import pins
    fx = pins.load_paper_example()
    g = gg.from_edges(fx["n"], fx["edges"])
    p, q = fx["eps"]
    note("hub/outlier paper example")
    r = _check(g, p, q, fx["mu"])
    assert sorted(np.flatnonzero(r == 3).tolist()) == fx["expected_hubs"]
    assert sorted(np.flatnonzero(r == 4).tolist()) == fx["expected_outliers"]


@pytest.mark.parametrize("name,gen,params", [
    ("planted", lambda: gg.planted(20000, 100, 0.2, 0.002, 11), [((1, 5), 5), ((1, 3), 4), ((1, 2), 3)]),
    ("rmat16", lambda: gg.rmat(16, 16, seed=2), [((1, 5), 5), ((1, 10), 3)]),
    ("chunglu", lambda: gg.chung_lu(100000, 20.0, 2.1, 2000.0, seed=3), [((1, 10), 3), ((1, 5), 5)]),
])
def test_hub_outlier_matches_oracle(name, gen, params):
    g = gen()
    for (p, q), mu in params:
        note(f"hub/outlier {name} eps={p}/{q} mu={mu}")
        r = _check(g, p, q, mu)
        if name == "planted" and (p, q) == (1, 5):
            assert (r == 3).any() and (r == 4).any()


def test_hub_outlier_off_keeps_three_roles():
    g = gg.planted(5000, 25, 0.2, 0.002, 4)
    with S.Graph.from_csr(g) as G:
        _, r = G.run(1, 5, 5)
    assert set(np.unique(r).tolist()) <= {0, 1, 2}


def test_hub_outlier_partitioned_batched_served():
    g = gg.chung_lu(60000, 20.0, 2.1, 1500.0, seed=8)
    el, er = _expect(g, 1, 10, 3)
    n, nnz = g.n, g.nnz
    resident = 8 * (n + 1) + 22 * n + (1 << 20)
    layout = 8 * (n + 1) + 4 * nnz + 13 * (nnz // 2) + 22 * n + (1 << 20)
    note("hub/outlier partitioned")
    with S.Graph.from_csr(g, budget=int(resident + 0.15 * (layout - resident)), hub_outlier=True,
                          timing=True) as P:
        l, r = P.run(1, 10, 3)
        assert P.stats()["h2d_bytes"] > 0
    assert np.array_equal(l, el) and np.array_equal(r, er)
    note("hub/outlier batched")
    gs = [g, gg.planted(3000, 20, 0.25, 0.003, 2), gg.from_edges(4, [])]
    eps, mus = [(1, 10), (1, 5), (1, 2)], [3, 4, 2]
    with S.Batch(gs, eps, mus, hub_outlier=True) as B:
        for replay in (True, False, True):
            bl, br = B.run(replay=replay)
            for gi, (p, q), mu, xl, xr in zip(gs, eps, mus, B.split(bl), B.split(br)):
                ol, orr = _expect(gi, p, q, mu)
                assert np.array_equal(xl, ol) and np.array_equal(xr, orr)
    note("hub/outlier served")
    with S.Server(num_slots=2, hub_outlier=True) as srv:
        gid = srv.add(g)
        l, r, _ = srv.wait(srv.submit(gid, 1, 10, 3), gid)
    assert np.array_equal(l, el) and np.array_equal(r, er)
