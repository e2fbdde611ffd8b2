"""Seeded synthetic input graphs shared by the CPU oracle's tests and the GPU path.

This module only generates inputs: it contains none of the structural
clustering arithmetic.  Every generator is deterministic for its seed and
returns an undirected simple graph as a symmetric CSR
(``row_ptr`` int64[n+1], ``col_idx`` int32[nnz], rows strictly increasing).

Workload recipes (stand-ins for the paper's real datasets, which are not
available here):

* ``planted(n, blocks, p_in, p_out, seed)`` - planted partition; config
  "plain SCAN, n=10,000 in 50 blocks, p_in=0.15, p_out=0.0005".
* ``rmat(scale, edge_factor, a, b, c, seed)`` - R-MAT, symmetrised,
  deduplicated, self-loops removed; config "R-MAT scale 22, edge factor 16,
  (0.57, 0.19, 0.19, 0.05)".
* ``chung_lu(n, mean_deg, exponent, max_deg, seed)`` - power-law expected
  degrees for the partitioned (out-of-core) path.
* ``planted_batch(count, seed)`` - many small planted-partition graphs of
  uneven size for the batched path.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build(force: bool = True) -> str:
    """Compile the generator library with g++ (host code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.gg_rmat_pairs.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64, vp, vp]
        lib.gg_rmat_pairs.restype = ctypes.c_int
        lib.gg_planted_pairs.argtypes = [i32, i32, dbl, dbl, u64, vp, vp]
        lib.gg_planted_pairs.restype = i64
        lib.gg_chunglu_pairs.argtypes = [i32, vp, u64, vp, vp, vp]
        lib.gg_chunglu_pairs.restype = i64
        lib.gg_symmetrize.argtypes = [i32, i64, vp, vp, vp, vp, vp]
        lib.gg_symmetrize.restype = i64
        lib.gg_compact.argtypes = [i32, vp, vp, vp, vp, vp]
        lib.gg_compact.restype = ctypes.c_int
        lib.gg_permute.argtypes = [i32, vp, vp, vp, vp, vp]
        lib.gg_permute.restype = ctypes.c_int
        lib.gg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Undirected simple graph in symmetric CSR form."""

    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.n > 0 else 0

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def from_pairs(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    """Symmetrise, drop self-loops and duplicates, sort rows."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    npairs = int(src.shape[0])
    raw_rp = np.empty(n + 1, dtype=np.int64)
    raw_ci = np.empty(max(1, 2 * npairs), dtype=np.int32)
    deg = np.empty(max(1, n), dtype=np.int64)
    nnz = lib.gg_symmetrize(n, npairs, _ptr(src), _ptr(dst), _ptr(raw_rp), _ptr(raw_ci), _ptr(deg))
    if nnz < 0:
        raise ValueError("pair list has out-of-range vertex ids")
    rp = np.empty(n + 1, dtype=np.int64)
    ci = np.empty(max(1, nnz), dtype=np.int32)
    lib.gg_compact(n, _ptr(raw_rp), _ptr(raw_ci), _ptr(deg), _ptr(rp), _ptr(ci))
    return CSR(n, rp, ci[:nnz])


def from_edges(n: int, edges) -> CSR:
    """Build a CSR from an iterable of (u, v) pairs (small graphs, tests)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return from_pairs(n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 2) -> CSR:
    lib = _load()
    n = 1 << scale
    ns = edge_factor * n
    src = np.empty(ns, dtype=np.int32)
    dst = np.empty(ns, dtype=np.int32)
    rc = lib.gg_rmat_pairs(scale, ns, a, b, c, seed, _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("bad R-MAT parameters")
    g = from_pairs(n, src, dst)
    del src, dst
    return g


def planted(n: int, blocks: int, p_in: float, p_out: float, seed: int = 1) -> CSR:
    lib = _load()
    cnt = lib.gg_planted_pairs(n, blocks, p_in, p_out, seed, None, None)
    if cnt < 0:
        raise ValueError("bad planted-partition parameters")
    src = np.empty(max(1, cnt), dtype=np.int32)
    dst = np.empty(max(1, cnt), dtype=np.int32)
    lib.gg_planted_pairs(n, blocks, p_in, p_out, seed, _ptr(src), _ptr(dst))
    return from_pairs(n, src[:cnt], dst[:cnt])


def erdos_renyi(n: int, p: float, seed: int = 0) -> CSR:
    return planted(n, 1, p, 0.0, seed)


def chung_lu_weights(n: int, mean_deg: float = 30.0, exponent: float = 2.1,
                     max_deg: float = 1.0e6) -> np.ndarray:
    """Expected degrees w_i = s*(i+1)^(-1/(exponent-1)), capped at max_deg,
    with s fitted (bisection) so that the mean of w equals mean_deg."""
    i = np.arange(1, n + 1, dtype=np.float64)
    base = i ** (-1.0 / (exponent - 1.0))
    lo, hi = 0.0, float(mean_deg) * n
    for _ in range(200):
        s = 0.5 * (lo + hi)
        if s <= lo or s >= hi:
            break  # the interval cannot shrink any further: later rounds change nothing
        mean = np.minimum(s * base, max_deg).mean()
        if mean < mean_deg:
            lo = s
        else:
            hi = s
    return np.minimum(0.5 * (lo + hi) * base, max_deg)


def chung_lu(n: int, mean_deg: float = 30.0, exponent: float = 2.1,
             max_deg: float = 1.0e6, seed: int = 3) -> CSR:
    lib = _load()
    w = np.ascontiguousarray(chung_lu_weights(n, mean_deg, exponent, max_deg))
    counts = np.zeros(n + 1, dtype=np.int64)
    total = lib.gg_chunglu_pairs(n, _ptr(w), seed, None, None, _ptr(counts))
    src = np.empty(max(1, total), dtype=np.int32)
    dst = np.empty(max(1, total), dtype=np.int32)
    lib.gg_chunglu_pairs(n, _ptr(w), seed, _ptr(src), _ptr(dst), _ptr(counts))
    return from_pairs(n, src[:total], dst[:total])


def permute(g: CSR, seed: int) -> tuple[CSR, np.ndarray]:
    """Relabel vertices by a seeded random permutation; returns (graph, perm)
    with perm[old] = new."""
    perm = np.random.default_rng(seed).permutation(g.n).astype(np.int32)
    return relabel(g, perm), perm


def reverse_ids(g: CSR) -> CSR:
    """The same graph with vertex v renamed n - 1 - v."""
    return relabel(g, np.arange(g.n - 1, -1, -1, dtype=np.int32))


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """The same graph with vertex v renamed perm[v] (perm a permutation)."""
    lib = _load()
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    rp = np.empty_like(g.row_ptr)
    ci = np.empty(max(1, g.nnz), dtype=np.int32)
    lib.gg_permute(g.n, _ptr(g.row_ptr), _ptr(np.ascontiguousarray(g.col_idx)), _ptr(perm),
                   _ptr(rp), _ptr(ci))
    return CSR(g.n, rp, ci[: g.nnz])


# ---------------------------------------------------------------------------
# Batched workload: many planted-partition graphs of uneven size.

@dataclass
class BatchSpec:
    n: int
    blocks: int
    p_in: float
    p_out: float
    eps: tuple[int, int]
    mu: int
    seed: int


def planted_batch_specs(count: int, seed: int = 4, n_lo: int = 100, n_hi: int = 20000):
    """Per-graph parameters: n log-uniform in [n_lo, n_hi]; target mean degree
    D ~ U[8, 64]; blocks ~ U{5..200} (at most n/2); 86 % of the expected
    degree inside the block; eps from {1/5, 2/5, 3/5, 4/5}; mu ~ U{2..10}."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        D = float(rng.uniform(8, 64))
        B = int(min(rng.integers(5, 201), max(1, n // 2)))
        s = n / B
        p_in = min(1.0, 0.86 * D / max(1.0, s - 1))
        rest = D - p_in * (s - 1)
        p_out = min(1.0, max(0.0, rest / max(1.0, n - s)))
        k = int(rng.integers(1, 5))
        mu = int(rng.integers(2, 11))
        specs.append(BatchSpec(n, B, p_in, p_out, (k, 5), mu, seed * 1_000_003 + i))
    return specs


def planted_batch(count: int, seed: int = 4, n_lo: int = 100, n_hi: int = 20000):
    specs = planted_batch_specs(count, seed, n_lo, n_hi)
    return [planted(s.n, s.blocks, s.p_in, s.p_out, s.seed) for s in specs], specs


def num_threads() -> int:
    return int(_load().gg_num_threads())


# ---------------------------------------------------------------------------
# Serving workload: resident R-MAT graphs of mixed size plus later uploads,
# and a stream of (graph, eps = k/10, mu) queries.

@dataclass
class RmatSpec:
    scale: int
    edge_factor: int
    seed: int

    def make(self) -> CSR:
        return rmat(self.scale, self.edge_factor, seed=self.seed)


def serving_specs(count: int = 64, uploads: int = 8, seed: int = 5, scale_lo: int = 16,
                  scale_hi: int = 23, ef_lo: int = 8, ef_hi: int = 32):
    """R-MAT graphs (same a, b, c, d as the single-graph workload) with scale
    ~ U{scale_lo..scale_hi} and edge factor ~ U{ef_lo..ef_hi}: `count` resident
    from the start, then `uploads` added while queries run.  Graph k uses
    generator seed 100 + k."""
    rng = np.random.default_rng(seed)
    specs = [RmatSpec(int(rng.integers(scale_lo, scale_hi + 1)), int(rng.integers(ef_lo, ef_hi + 1)), 100 + k)
             for k in range(count + uploads)]
    return specs[:count], specs[count:]


def serving_queries(num: int, num_graphs: int, seed: int = 6):
    """Queries (graph index, p, q, mu) with graph uniform, eps = k/10 for
    k ~ U{1..9}, mu ~ U{2..20}."""
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(num_graphs)), int(rng.integers(1, 10)), 10, int(rng.integers(2, 21)))
            for _ in range(num)]

