"""Pins of the CPU oracle (no GPU).  See pins.py for what each check rests on."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def test_paper_worked_example(orc):
    pins.check_paper_example(orc)


def test_closed_forms_and_exact_equality(orc):
    pins.check_closed_forms(orc)


def test_validation(orc):
    pins.check_validation(orc)


def test_bruteforce_all_graphs_up_to_5_vertices(orc):
    pins.check_bruteforce_exhaustive(orc, nmax=5, literal_upto=4)


def test_bruteforce_sampled_6_vertex_graphs(orc):
    rng = np.random.default_rng(6)
    masks = rng.choice(1 << 15, size=400, replace=False)
    grid = [((1, 5), 2), ((1, 3), 3), ((1, 2), 3), ((2, 3), 2), ((3, 4), 4), ((1, 1), 2)]
    for mask in masks:
        pins.check_against_bruteforce(orc, 6, pins._edges_of(6, int(mask)), grid=grid,
                                      literal=(int(mask) % 8 == 0))


def test_bruteforce_random_up_to_12_vertices(orc):
    pins.check_bruteforce_random(orc, count=150, nmin=6, nmax=12, seed=7)


@pytest.mark.parametrize("name,gen,params", [
    ("planted_A", lambda: gg.planted(10000, 50, 0.15, 0.0005, 1),
     [((1, 2), 5), ((1, 5), 5), ((1, 10), 5)]),
    ("rmat12", lambda: gg.rmat(12, 16, seed=2), [((1, 5), 5), ((1, 2), 5), ((1, 10), 3)]),
    ("chunglu", lambda: gg.chung_lu(8000, 20.0, 2.1, 400.0, seed=3), [((1, 10), 3), ((1, 2), 10)]),
])
def test_library_pipeline(orc, name, gen, params):
    pins.check_library_pipeline(orc, gen(), params)


def test_triangle_identity(orc):
    pins.check_triangles(orc, gg.rmat(10, 8, seed=5))
    pins.check_triangles(orc, gg.planted(800, 8, 0.2, 0.01, 2))


def test_monotone_in_eps_and_mu(orc):
    pins.check_monotone(orc, gg.planted(2000, 20, 0.2, 0.002, 3))


def test_relabel_invariance(orc):
    pins.check_relabel(orc, gg.planted(3000, 30, 0.2, 0.002, 4))
    pins.check_relabel(orc, gg.rmat(11, 8, seed=6))


def test_components_special_case(orc):
    pins.check_components_case(orc, gg.planted(1500, 15, 0.25, 0.001, 8))


def test_closed_count_pairwise_matches_counts_all(orc):
    g = gg.rmat(11, 16, seed=3)
    cnt = orc.counts(g)
    rng = np.random.default_rng(0)
    arcs = rng.integers(0, g.nnz, size=2000)
    rows = np.searchsorted(g.row_ptr, arcs, side="right") - 1
    for k, u in zip(arcs, rows):
        assert orc.closed_count(g, int(u), int(g.col_idx[k])) == cnt[k]


def test_threads_do_not_change_results(orc):
    g = gg.rmat(12, 16, seed=4)
    l1, r1, c1 = orc.scan(g, 1, 5, 5, threads=1, want_counts=True)
    l4, r4, c4 = orc.scan(g, 1, 5, 5, threads=4, want_counts=True)
    assert np.array_equal(c1, c4) and np.array_equal(l1, l4) and np.array_equal(r1, r4)


def test_isolated_and_empty(orc):
    g = gg.from_edges(5, [])
    l, r = orc.scan(g, 1, 2, 2)
    assert l.tolist() == [-1] * 5 and r.tolist() == [0] * 5
    g0 = gg.from_edges(0, [])
    l, r = orc.scan(g0, 1, 2, 2)
    assert l.size == 0 and r.size == 0


def test_invalid_parameters(orc):
    g = gg.from_edges(3, [(0, 1)])
    for p, q, mu in [(0, 2, 2), (3, 2, 2), (1, 2, 1)]:
        with pytest.raises(ValueError):
            orc.scan(g, p, q, mu)
