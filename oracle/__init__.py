"""CPU oracle for exact structural graph clustering (SCAN), GPUSCAN++ Section 2.1.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the library package.
It shares no code with the GPU path.  The arithmetic lives in
``scan_oracle.c`` (plain C, built with gcc); this module only marshals arrays.

Functions follow the paper's definitions:

* ``closed_count(g, u, v)`` - |N[u] intersect N[v]| (Def 2.1, Def 2.2), one pair.
* ``counts(g)`` - the same for every arc, CSR order.
* ``similar(c, a, b, p, q)`` - sigma >= p/q evaluated as (c q)^2 >= p^2 a b
  (Def 2.3, exact).
* ``scan(g, p, q, mu)`` - labels (minimum core id of the cluster, -1 when
  unclassified) and roles (0 unclassified, 1 core, 2 border); Defs 2.4-2.6.
* ``cluster(g, counts, p, q, mu)`` - the same from counts already computed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "scan_oracle.c")
LIB = os.path.join(_HERE, "libscan_oracle.so")

ROLE_UNCLASSIFIED, ROLE_CORE, ROLE_BORDER = 0, 1, 2


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src],
                       check=True)
        os.replace(tmp, out)
    return out


def _vp(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """ctypes view of one build of the oracle library."""

    def __init__(self, path: str = LIB):
        if path == LIB and not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_validate.argtypes = [i32, i64, vp, vp]
        lib.oracle_validate.restype = ctypes.c_int
        lib.oracle_closed_count.argtypes = [vp, vp, i32, i32]
        lib.oracle_closed_count.restype = i64
        lib.oracle_similar.argtypes = [i64, i64, i64, i64, i64]
        lib.oracle_similar.restype = ctypes.c_int
        lib.oracle_counts_all.argtypes = [i32, vp, vp, vp, ctypes.c_int]
        lib.oracle_counts_all.restype = ctypes.c_int
        lib.oracle_scan.argtypes = [i32, vp, vp, i64, i64, i32, ctypes.c_int, vp, vp, vp]
        lib.oracle_scan.restype = ctypes.c_int
        lib.oracle_cluster.argtypes = [i32, vp, vp, vp, i64, i64, i32, vp, vp]
        lib.oracle_hub_outlier.argtypes = [i32, vp, vp, vp, vp]
        lib.oracle_cluster.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        self.lib = lib

    @staticmethod
    def _arrays(g):
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
        if ci.size == 0:
            ci = np.zeros(1, dtype=np.int32)
        return int(g.n), rp, ci

    def validate(self, g) -> int:
        n, rp, ci = self._arrays(g)
        return int(self.lib.oracle_validate(n, int(rp[-1]), _vp(rp), _vp(ci)))

    def closed_count(self, g, u: int, v: int) -> int:
        n, rp, ci = self._arrays(g)
        return int(self.lib.oracle_closed_count(_vp(rp), _vp(ci), int(u), int(v)))

    def similar(self, c: int, a: int, b: int, p: int, q: int) -> bool:
        return bool(self.lib.oracle_similar(int(c), int(a), int(b), int(p), int(q)))

    def counts(self, g, threads: int = 1) -> np.ndarray:
        n, rp, ci = self._arrays(g)
        out = np.zeros(max(1, int(rp[-1])), dtype=np.int32)
        rc = self.lib.oracle_counts_all(n, _vp(rp), _vp(ci), _vp(out), int(threads))
        if rc != 0:
            raise MemoryError("oracle_counts_all failed")
        return out[: int(rp[-1])]

    def scan(self, g, p: int, q: int, mu: int, threads: int = 1, want_counts: bool = False):
        n, rp, ci = self._arrays(g)
        labels = np.empty(max(1, n), dtype=np.int32)
        roles = np.empty(max(1, n), dtype=np.uint8)
        cnt = np.empty(max(1, int(rp[-1])), dtype=np.int32) if want_counts else None
        rc = self.lib.oracle_scan(n, _vp(rp), _vp(ci), int(p), int(q), int(mu), int(threads),
                                  _vp(labels), _vp(roles), _vp(cnt))
        if rc != 0:
            raise ValueError(f"oracle_scan failed with code {rc}")
        labels, roles = labels[:n], roles[:n]
        if want_counts:
            return labels, roles, cnt[: int(rp[-1])]
        return labels, roles

    def cluster(self, g, counts: np.ndarray, p: int, q: int, mu: int):
        """Clustering from per-arc closed counts previously returned by counts()."""
        n, rp, ci = self._arrays(g)
        cnt = np.ascontiguousarray(counts, dtype=np.int32)
        if cnt.size == 0:
            cnt = np.zeros(1, dtype=np.int32)
        labels = np.empty(max(1, n), dtype=np.int32)
        roles = np.empty(max(1, n), dtype=np.uint8)
        rc = self.lib.oracle_cluster(n, _vp(rp), _vp(ci), _vp(cnt), int(p), int(q), int(mu),
                                     _vp(labels), _vp(roles))
        if rc != 0:
            raise ValueError(f"oracle_cluster failed with code {rc}")
        return labels[:n], roles[:n]

    def hub_outlier(self, g, labels: np.ndarray, roles: np.ndarray) -> np.ndarray:
        """Roles with every unclassified vertex split into hub (3) or outlier (4), Def 2.7."""
        n, rp, ci = self._arrays(g)
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        out = np.array(roles, dtype=np.uint8, copy=True)
        if n == 0:
            return out
        rc = self.lib.oracle_hub_outlier(n, _vp(rp), _vp(ci), _vp(lab), _vp(out))
        if rc != 0:
            raise ValueError(f"oracle_hub_outlier failed with code {rc}")
        return out

    def max_threads(self) -> int:
        return int(self.lib.oracle_max_threads())


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def validate(g) -> int:
    return default().validate(g)


def closed_count(g, u, v) -> int:
    return default().closed_count(g, u, v)


def similar(c, a, b, p, q) -> bool:
    return default().similar(c, a, b, p, q)


def counts(g, threads: int = 1) -> np.ndarray:
    return default().counts(g, threads)


def scan(g, p, q, mu, threads: int = 1, want_counts: bool = False):
    return default().scan(g, p, q, mu, threads, want_counts)


def cluster(g, counts, p, q, mu):
    return default().cluster(g, counts, p, q, mu)


def hub_outlier(g, labels, roles):
    return default().hub_outlier(g, labels, roles)


def max_threads() -> int:
    return default().max_threads()
