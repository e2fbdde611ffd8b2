"""Seeded input generators: determinism, simplicity and expected sizes."""
import numpy as np

import graphgen as gg


def _simple_symmetric(g):
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == ci.size
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(ci != rows)
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    fwd = rows.astype(np.int64) * g.n + ci
    rev = ci.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(fwd), np.sort(rev))


def test_planted_deterministic_and_sized():
    a = gg.planted(10000, 50, 0.15, 0.0005, 1)
    b = gg.planted(10000, 50, 0.15, 0.0005, 1)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
    _simple_symmetric(a)
    # E[m] = 50*C(200,2)*0.15 + (C(10000,2) - 50*C(200,2))*0.0005
    em = 50 * 19900 * 0.15 + (49995000 - 50 * 19900) * 0.0005
    assert abs(a.m - em) < 5 * np.sqrt(em)
    c = gg.planted(10000, 50, 0.15, 0.0005, 2)
    assert not np.array_equal(a.col_idx[:100], c.col_idx[:100])


def test_rmat_deterministic_and_sized():
    a = gg.rmat(14, 16, seed=2)
    b = gg.rmat(14, 16, seed=2)
    assert np.array_equal(a.col_idx, b.col_idx)
    _simple_symmetric(a)
    assert a.n == 1 << 14 and 0.4 * 16 * a.n < a.m < 16 * a.n
    # quadrant a = 0.57 dominates: vertex 0 has the largest degree
    assert a.degrees().argmax() == 0


def test_chung_lu_mean_degree():
    g = gg.chung_lu(50000, 30.0, 2.1, 5000.0, seed=3)
    _simple_symmetric(g)
    assert 25.0 < g.degrees().mean() < 31.0
    w = gg.chung_lu_weights(1000, 30.0, 2.1, 100.0)
    assert abs(w.mean() - 30.0) < 1e-6 and w.max() <= 100.0


def test_permute_is_relabelling():
    g = gg.rmat(10, 8, seed=1)
    h, perm = gg.permute(g, 5)
    _simple_symmetric(h)
    assert np.array_equal(np.sort(g.degrees()), np.sort(h.degrees()))
    assert np.array_equal(h.degrees()[perm], g.degrees())


def test_batch_specs_ranges():
    specs = gg.planted_batch_specs(500, seed=4)
    ns = np.array([s.n for s in specs])
    assert ns.min() >= 100 and ns.max() <= 20000
    assert all(2 <= s.mu <= 10 for s in specs)
    assert {s.eps for s in specs} <= {(1, 5), (2, 5), (3, 5), (4, 5)}
