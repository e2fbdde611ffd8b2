"""Python binding of the MI355X structural-clustering library.

Argument marshalling only: every function below forwards to the C-ABI of the
same name in ``libscan_mi355x.so`` (declared in ``include/scan.h``), and all
computation happens in the library's HIP kernels.  There is no CPU fallback:
if the library is not built, importing works but every call raises
``LibraryNotBuilt``.

Host arrays are numpy arrays; device buffers are raw addresses (int) obtained
from ``scan_device_alloc``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscan_mi355x.so")

SCAN_OK, SCAN_E_INVAL, SCAN_E_GRAPH, SCAN_E_RANGE, SCAN_E_NOMEM, SCAN_E_DEVICE = 0, -1, -2, -3, -4, -5
SCAN_UNCLASSIFIED, SCAN_CORE, SCAN_BORDER, SCAN_HUB, SCAN_OUTLIER = 0, 1, 2, 3, 4
PHASES = ["init", "cores", "finalize", "hook", "merge", "flatten", "attach", "output"]
NUM_PHASES = len(PHASES)
NUM_BUCKETS = 7
EXPORTED = [
    "scan_opts_default", "scan_graph_create", "scan_graph_destroy", "scan_graph_info", "scan_run",
    "scan_run_device", "scan_similarity", "scan_similarity_device", "scan_eps_threshold",
    "scan_last_stats", "scan_device_alloc", "scan_device_free", "scan_memcpy_d2h",
    "scan_memcpy_h2d", "scan_device_copy", "scan_h2d_rate", "scan_last_error", "scan_version",
    "scan_server_create", "scan_server_add_graph", "scan_server_remove_graph", "scan_server_submit",
    "scan_server_wait", "scan_server_info", "scan_server_destroy",
    "scan_batch_create", "scan_batch_run", "scan_batch_config", "scan_batch_stats", "scan_batch_destroy",
    "scan_run_batch", "scan_run_device_noalloc", "scan_graph_footprint", "scan_batch_set_params",
    "scan_server_set_budget", "scan_device_read", "scan_graph_device_bytes",
]


class LibraryNotBuilt(RuntimeError):
    pass


class ScanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class scan_opts(ctypes.Structure):
    _fields_ = [
        ("device_budget_bytes", ctypes.c_uint64),
        ("validate", ctypes.c_int32),
        ("pruning", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("strategy", ctypes.c_int32),
        ("hub_outlier", ctypes.c_int32),
        ("hub_ranked", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p),
    ]


class scan_batch(ctypes.Structure):
    _fields_ = [
        ("num_graphs", ctypes.c_int32),
        ("vtx_off", ctypes.c_void_p),
        ("arc_off", ctypes.c_void_p),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("eps_num", ctypes.c_void_p),
        ("eps_den", ctypes.c_void_p),
        ("mu", ctypes.c_void_p),
        ("autotune", ctypes.c_int32),
    ]


class scan_stats(ctypes.Structure):
    _fields_ = [
        ("ms_total", ctypes.c_double),
        ("ms_phase", ctypes.c_double * NUM_PHASES),
        ("ms_cores_bucket", ctypes.c_double * NUM_BUCKETS),
        ("edges", ctypes.c_int64),
        ("bucket_edges", ctypes.c_int64 * NUM_BUCKETS),
        ("evaluated", ctypes.c_int64 * NUM_PHASES),
        ("bounded", ctypes.c_int64 * NUM_PHASES),
        ("probes", ctypes.c_int64 * NUM_PHASES),
        ("cores_bucket_evaluated", ctypes.c_int64 * NUM_BUCKETS),
        ("cores_bucket_probes", ctypes.c_int64 * NUM_BUCKETS),
        ("h2d_bytes", ctypes.c_int64),
        ("group_split", ctypes.c_int64),
    ]


_lib = None


def lib():
    """The loaded library (raises LibraryNotBuilt if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryNotBuilt(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        P = ctypes.POINTER
        L.scan_opts_default.argtypes = [P(scan_opts)]
        L.scan_opts_default.restype = None
        L.scan_graph_create.argtypes = [i32, i64, vp, vp, P(scan_opts), P(vp)]
        L.scan_graph_destroy.argtypes = [vp]
        L.scan_graph_info.argtypes = [vp, P(i32), P(i64), P(i64), P(i32)]
        L.scan_graph_footprint.argtypes = [i32, i64, P(scan_opts), P(u64)]
        L.scan_graph_device_bytes.argtypes = [vp, P(u64)]
        L.scan_run.argtypes = [vp, i64, i64, i32, vp, vp]
        L.scan_run_device.argtypes = [vp, i64, i64, i32, vp, vp, vp]
        L.scan_run_device_noalloc.argtypes = [vp, i64, i64, i32, vp, vp, vp]
        L.scan_similarity.argtypes = [vp, vp]
        L.scan_similarity_device.argtypes = [vp, vp, vp]
        L.scan_eps_threshold.argtypes = [i64, i64, i64, i64]
        L.scan_eps_threshold.restype = i64
        L.scan_last_stats.argtypes = [vp, P(scan_stats)]
        L.scan_device_alloc.argtypes = [u64, P(vp)]
        L.scan_device_free.argtypes = [vp]
        L.scan_memcpy_d2h.argtypes = [vp, vp, u64]
        L.scan_memcpy_h2d.argtypes = [vp, vp, u64]
        L.scan_device_copy.argtypes = [vp, vp, u64, i32, P(ctypes.c_float)]
        L.scan_device_read.argtypes = [vp, u64, i32, P(ctypes.c_float)]
        L.scan_h2d_rate.argtypes = [u64, i32, P(ctypes.c_double)]
        L.scan_server_create.argtypes = [P(scan_opts), i32, P(vp)]
        L.scan_server_add_graph.argtypes = [vp, i32, i64, vp, vp, P(i32)]
        L.scan_server_remove_graph.argtypes = [vp, i32]
        L.scan_server_set_budget.argtypes = [vp, u64]
        L.scan_server_submit.argtypes = [vp, i32, i64, i64, i32, P(i64)]
        L.scan_server_wait.argtypes = [vp, i64, vp, vp, P(ctypes.c_double)]
        L.scan_server_info.argtypes = [vp, P(u64), P(i32), P(i32), P(i64)]
        L.scan_server_destroy.argtypes = [vp]
        L.scan_batch_create.argtypes = [P(scan_batch), P(scan_opts), P(vp)]
        L.scan_batch_run.argtypes = [vp, i32, vp, vp]
        L.scan_batch_set_params.argtypes = [vp, vp, vp, vp]
        L.scan_batch_config.argtypes = [vp, vp, P(i32)]
        L.scan_batch_stats.argtypes = [vp, P(scan_stats)]
        L.scan_batch_destroy.argtypes = [vp]
        L.scan_run_batch.argtypes = [P(scan_batch), P(scan_opts), vp, vp]
        L.scan_last_error.restype = ctypes.c_char_p
        L.scan_version.restype = ctypes.c_char_p
        for name in ("scan_graph_create", "scan_graph_destroy", "scan_graph_info", "scan_run",
                     "scan_run_device", "scan_similarity", "scan_similarity_device", "scan_last_stats",
                     "scan_device_alloc", "scan_device_free", "scan_memcpy_d2h", "scan_memcpy_h2d",
                     "scan_device_copy", "scan_h2d_rate", "scan_server_create", "scan_server_add_graph", "scan_server_remove_graph",
                     "scan_server_submit", "scan_server_wait", "scan_server_info", "scan_server_destroy",
                     "scan_batch_create", "scan_batch_run", "scan_batch_config", "scan_batch_stats",
                     "scan_batch_destroy", "scan_run_batch", "scan_run_device_noalloc",
                     "scan_graph_footprint", "scan_batch_set_params", "scan_server_set_budget",
                     "scan_device_read", "scan_graph_device_bytes"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SCAN_OK:
        raise ScanError(rc, lib().scan_last_error().decode(errors="replace"))


def _vp(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def scan_version() -> str:
    return lib().scan_version().decode()


def scan_last_error() -> str:
    return lib().scan_last_error().decode(errors="replace")


def scan_opts_default() -> scan_opts:
    o = scan_opts()
    lib().scan_opts_default(ctypes.byref(o))
    return o


def make_opts(budget: int = 0, validate: bool = True, pruning: bool = True, timing: bool = False,
              strategy: int = 0, hub_outlier: bool = False, hub_ranked: bool = True,
              stream: int | None = None) -> scan_opts:
    o = scan_opts_default()
    o.strategy = int(strategy)
    o.hub_outlier = int(bool(hub_outlier))
    o.hub_ranked = int(bool(hub_ranked))
    o.device_budget_bytes = int(budget)
    o.validate = int(bool(validate))
    o.pruning = int(bool(pruning))
    o.timing = int(bool(timing))
    o.hip_stream = stream
    return o


def scan_graph_create(n: int, nnz: int, row_ptr: np.ndarray, col_idx: np.ndarray,
                      opts: scan_opts | None = None) -> ctypes.c_void_p:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if rp.shape[0] != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    if ci.shape[0] < nnz:
        raise ValueError("col_idx shorter than nnz")
    h = ctypes.c_void_p()
    _check(lib().scan_graph_create(int(n), int(nnz), _vp(rp), _vp(ci) if nnz else None,
                                   ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
    return h


def scan_graph_destroy(g) -> None:
    _check(lib().scan_graph_destroy(g))


def scan_graph_footprint(n: int, nnz: int, opts: scan_opts | None = None) -> int:
    b = ctypes.c_uint64()
    _check(lib().scan_graph_footprint(int(n), int(nnz), ctypes.byref(opts) if opts is not None else None,
                                      ctypes.byref(b)))
    return int(b.value)


def scan_graph_device_bytes(g) -> int:
    b = ctypes.c_uint64()
    _check(lib().scan_graph_device_bytes(g, ctypes.byref(b)))
    return int(b.value)


def scan_graph_info(g) -> tuple[int, int, int, int]:
    n, nnz, m, dm = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(lib().scan_graph_info(g, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(m), ctypes.byref(dm)))
    return n.value, nnz.value, m.value, dm.value


def scan_run(g, eps_num: int, eps_den: int, mu: int, labels: np.ndarray | None = None,
             roles: np.ndarray | None = None):
    n = scan_graph_info(g)[0]
    labels = np.empty(max(n, 1), dtype=np.int32) if labels is None else labels
    roles = np.empty(max(n, 1), dtype=np.uint8) if roles is None else roles
    assert labels.dtype == np.int32 and roles.dtype == np.uint8 and labels.size >= n and roles.size >= n
    _check(lib().scan_run(g, int(eps_num), int(eps_den), int(mu), _vp(labels), _vp(roles)))
    return labels[:n], roles[:n]


def scan_run_device(g, eps_num: int, eps_den: int, mu: int, d_labels: int, d_roles: int,
                    stream: int | None = None) -> None:
    _check(lib().scan_run_device(g, int(eps_num), int(eps_den), int(mu), ctypes.c_void_p(d_labels),
                                 ctypes.c_void_p(d_roles), ctypes.c_void_p(stream) if stream else None))


def scan_run_device_noalloc(g, eps_num: int, eps_den: int, mu: int, d_labels: int, d_roles: int,
                            stream: int | None = None) -> None:
    _check(lib().scan_run_device_noalloc(g, int(eps_num), int(eps_den), int(mu), ctypes.c_void_p(d_labels),
                                         ctypes.c_void_p(d_roles), ctypes.c_void_p(stream) if stream else None))


def scan_similarity(g, counts: np.ndarray | None = None) -> np.ndarray:
    nnz = scan_graph_info(g)[1]
    counts = np.empty(max(nnz, 1), dtype=np.int32) if counts is None else counts
    _check(lib().scan_similarity(g, _vp(counts)))
    return counts[:nnz]


def scan_similarity_device(g, d_counts: int, stream: int | None = None) -> None:
    _check(lib().scan_similarity_device(g, ctypes.c_void_p(d_counts),
                                        ctypes.c_void_p(stream) if stream else None))


def scan_eps_threshold(p: int, q: int, a: int, b: int) -> int:
    return int(lib().scan_eps_threshold(int(p), int(q), int(a), int(b)))


def scan_last_stats(g) -> dict:
    s = scan_stats()
    _check(lib().scan_last_stats(g, ctypes.byref(s)))
    return {
        "ms_total": s.ms_total,
        "ms_phase": dict(zip(PHASES, list(s.ms_phase))),
        "ms_cores_bucket": list(s.ms_cores_bucket),
        "edges": s.edges,
        "bucket_edges": list(s.bucket_edges),
        "evaluated": dict(zip(PHASES, list(s.evaluated))),
        "bounded": dict(zip(PHASES, list(s.bounded))),
        "probes": dict(zip(PHASES, list(s.probes))),
        "cores_bucket_evaluated": list(s.cores_bucket_evaluated),
        "cores_bucket_probes": list(s.cores_bucket_probes),
        "h2d_bytes": s.h2d_bytes,
        "group_split": s.group_split,
    }


def scan_device_alloc(nbytes: int) -> int:
    p = ctypes.c_void_p()
    _check(lib().scan_device_alloc(int(nbytes), ctypes.byref(p)))
    return int(p.value)


def scan_device_free(ptr: int) -> None:
    _check(lib().scan_device_free(ctypes.c_void_p(ptr)))


def scan_memcpy_d2h(dst: np.ndarray, src: int, nbytes: int) -> None:
    assert dst.nbytes >= nbytes
    _check(lib().scan_memcpy_d2h(_vp(dst), ctypes.c_void_p(src), int(nbytes)))


def scan_memcpy_h2d(dst: int, src: np.ndarray, nbytes: int) -> None:
    assert src.nbytes >= nbytes
    _check(lib().scan_memcpy_h2d(ctypes.c_void_p(dst), _vp(np.ascontiguousarray(src)), int(nbytes)))


def scan_device_copy(dst: int, src: int, nbytes: int, iters: int = 1) -> float:
    """Streaming device-to-device copy kernel; returns the mean kernel time in ms."""
    ms = ctypes.c_float()
    _check(lib().scan_device_copy(ctypes.c_void_p(dst), ctypes.c_void_p(src), int(nbytes), int(iters),
                                  ctypes.byref(ms)))
    return float(ms.value)


def scan_device_read(src: int, nbytes: int, iters: int = 1) -> float:
    """Streaming read-only kernel over a device buffer; returns the mean kernel time in ms."""
    ms = ctypes.c_float()
    _check(lib().scan_device_read(ctypes.c_void_p(src), int(nbytes), int(iters), ctypes.byref(ms)))
    return float(ms.value)


def scan_h2d_rate(nbytes: int = 1 << 30, iters: int = 5) -> float:
    """Pinned host-to-device copy rate in bytes per second."""
    r = ctypes.c_double()
    _check(lib().scan_h2d_rate(int(nbytes), int(iters), ctypes.byref(r)))
    return float(r.value)


class Graph:
    """Owning wrapper around a scan_graph handle."""

    def __init__(self, n, row_ptr, col_idx, **opts):
        self.opts = make_opts(**opts)
        self.n = int(n)
        self.nnz = int(row_ptr[-1]) if n > 0 else 0
        self.handle = scan_graph_create(self.n, self.nnz, row_ptr, col_idx, self.opts)

    @classmethod
    def from_csr(cls, g, **opts):
        return cls(g.n, g.row_ptr, g.col_idx, **opts)

    def info(self):
        return scan_graph_info(self.handle)

    def device_bytes(self):
        return scan_graph_device_bytes(self.handle)

    def run(self, p, q, mu, labels=None, roles=None):
        return scan_run(self.handle, p, q, mu, labels, roles)

    def run_device(self, p, q, mu, d_labels, d_roles, stream=None):
        scan_run_device(self.handle, p, q, mu, d_labels, d_roles, stream)

    def run_device_noalloc(self, p, q, mu, d_labels, d_roles, stream=None):
        scan_run_device_noalloc(self.handle, p, q, mu, d_labels, d_roles, stream)

    def similarity(self):
        return scan_similarity(self.handle)

    def stats(self):
        return scan_last_stats(self.handle)

    def close(self):
        if self.handle is not None:
            scan_graph_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Serving

def scan_server_create(opts: scan_opts | None = None, num_slots: int = 4) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().scan_server_create(ctypes.byref(opts) if opts is not None else None, int(num_slots),
                                    ctypes.byref(h)))
    return h


def scan_server_add_graph(s, n: int, nnz: int, row_ptr: np.ndarray, col_idx: np.ndarray) -> int:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    gid = ctypes.c_int32()
    _check(lib().scan_server_add_graph(s, int(n), int(nnz), _vp(rp), _vp(ci) if nnz else None,
                                       ctypes.byref(gid)))
    return gid.value


def scan_server_remove_graph(s, gid: int) -> None:
    _check(lib().scan_server_remove_graph(s, int(gid)))


def scan_server_submit(s, gid: int, eps_num: int, eps_den: int, mu: int) -> int:
    req = ctypes.c_int64()
    _check(lib().scan_server_submit(s, int(gid), int(eps_num), int(eps_den), int(mu), ctypes.byref(req)))
    return req.value


def scan_server_wait(s, req: int, n: int, labels=None, roles=None):
    """Waits for request req of a graph of n vertices; its labels and roles go
    to the given arrays (contiguous int32 / uint8 of at least n entries, reused
    across calls by a caller that wants to avoid fresh allocations) or to new
    ones.  Returns (labels[:n], roles[:n], latency in ms)."""
    if labels is None:
        labels = np.empty(max(n, 1), dtype=np.int32)
    if roles is None:
        roles = np.empty(max(n, 1), dtype=np.uint8)
    if (labels.dtype != np.int32 or roles.dtype != np.uint8 or labels.size < max(n, 1) or roles.size < max(n, 1)
            or not labels.flags.c_contiguous or not roles.flags.c_contiguous):
        raise ValueError("labels / roles must be contiguous int32 / uint8 arrays of at least n entries")
    lat = ctypes.c_double()
    _check(lib().scan_server_wait(s, int(req), _vp(labels), _vp(roles), ctypes.byref(lat)))
    return labels[:n], roles[:n], lat.value


def scan_server_info(s) -> dict:
    rb, ng, nr, done = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().scan_server_info(s, ctypes.byref(rb), ctypes.byref(ng), ctypes.byref(nr), ctypes.byref(done)))
    return {"resident_bytes": rb.value, "graphs": ng.value, "resident_graphs": nr.value,
            "completed": done.value}


def scan_server_destroy(s) -> None:
    _check(lib().scan_server_destroy(s))


class Server:
    """Owning wrapper around a scan_server handle."""

    def __init__(self, num_slots: int = 4, budget: int = 0, **opts):
        self.handle = scan_server_create(make_opts(budget=budget, **opts), num_slots)
        self.sizes = {}

    def add(self, g) -> int:
        gid = scan_server_add_graph(self.handle, g.n, g.nnz, g.row_ptr, g.col_idx)
        self.sizes[gid] = g.n
        return gid

    def remove(self, gid: int) -> None:
        scan_server_remove_graph(self.handle, gid)
        self.sizes.pop(gid, None)

    def set_budget(self, nbytes: int) -> None:
        _check(lib().scan_server_set_budget(self.handle, int(nbytes)))

    def submit(self, gid: int, p: int, q: int, mu: int) -> int:
        return scan_server_submit(self.handle, gid, p, q, mu)

    def wait(self, req: int, gid: int, labels=None, roles=None):
        return scan_server_wait(self.handle, req, self.sizes[gid], labels, roles)

    def info(self) -> dict:
        return scan_server_info(self.handle)

    def close(self):
        if self.handle is not None:
            scan_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Batched

def pack_batch(graphs, eps, mus):
    """Packs CSR graphs (objects with n, row_ptr, col_idx) and per-graph
    parameters into the arrays of struct scan_batch.  Returns (arrays, struct);
    keep `arrays` alive while the struct is used."""
    G = len(graphs)
    vtx_off = np.zeros(G + 1, np.int64)
    arc_off = np.zeros(G + 1, np.int64)
    for k, g in enumerate(graphs):
        vtx_off[k + 1] = vtx_off[k] + g.n
        arc_off[k + 1] = arc_off[k] + int(g.row_ptr[-1])
    row_ptr = np.concatenate([np.asarray(g.row_ptr, np.int64) for g in graphs]) if G else np.zeros(1, np.int64)
    col_idx = np.concatenate([np.asarray(g.col_idx, np.int32) for g in graphs]) if G else np.zeros(1, np.int32)
    if col_idx.size == 0:
        col_idx = np.zeros(1, np.int32)
    eps_num = np.array([e[0] for e in eps], np.int64)
    eps_den = np.array([e[1] for e in eps], np.int64)
    mu = np.array(mus, np.int32)
    arrays = dict(vtx_off=vtx_off, arc_off=arc_off, row_ptr=row_ptr, col_idx=col_idx, eps_num=eps_num,
                  eps_den=eps_den, mu=mu)
    st = scan_batch(G, *(ctypes.c_void_p(arrays[k].ctypes.data) for k in
                         ("vtx_off", "arc_off", "row_ptr", "col_idx", "eps_num", "eps_den", "mu")), 0)
    return arrays, st


class Batch:
    """Owning wrapper around a scan_batch_graph handle."""

    def __init__(self, graphs, eps, mus, autotune: bool = False, **opts):
        self.arrays, st = pack_batch(graphs, eps, mus)
        st.autotune = int(bool(autotune))
        self.N = int(self.arrays["vtx_off"][-1])
        self.vtx_off = self.arrays["vtx_off"]
        o = make_opts(**opts)
        self.handle = ctypes.c_void_p()
        _check(lib().scan_batch_create(ctypes.byref(st), ctypes.byref(o), ctypes.byref(self.handle)))

    def run(self, replay: bool = True):
        labels = np.empty(max(self.N, 1), np.int32)
        roles = np.empty(max(self.N, 1), np.uint8)
        _check(lib().scan_batch_run(self.handle, int(bool(replay)), _vp(labels), _vp(roles)))
        return labels[:self.N], roles[:self.N]

    def split(self, arr):
        return [arr[self.vtx_off[k]:self.vtx_off[k + 1]] for k in range(len(self.vtx_off) - 1)]

    def config(self):
        """(lane-group width per degree bucket, edges per tile)."""
        lanes = np.zeros(NUM_BUCKETS, np.int32)
        tile = ctypes.c_int32()
        _check(lib().scan_batch_config(self.handle, _vp(lanes), ctypes.byref(tile)))
        return lanes.tolist(), int(tile.value)

    def set_params(self, eps, mus):
        eps_num = np.array([e[0] for e in eps], np.int64)
        eps_den = np.array([e[1] for e in eps], np.int64)
        mu = np.array(mus, np.int32)
        _check(lib().scan_batch_set_params(self.handle, _vp(eps_num), _vp(eps_den), _vp(mu)))

    def stats(self):
        s = scan_stats()
        _check(lib().scan_batch_stats(self.handle, ctypes.byref(s)))
        return {"ms_total": s.ms_total, "evaluated_cores": s.evaluated[1], "edges": s.edges,
                "evaluated": dict(zip(PHASES, list(s.evaluated))), "probes": dict(zip(PHASES, list(s.probes)))}

    def close(self):
        if self.handle is not None:
            _check(lib().scan_batch_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scan_run_batch(graphs, eps, mus, **opts):
    arrays, st = pack_batch(graphs, eps, mus)
    N = int(arrays["vtx_off"][-1])
    labels = np.empty(max(N, 1), np.int32)
    roles = np.empty(max(N, 1), np.uint8)
    o = make_opts(**opts)
    _check(lib().scan_run_batch(ctypes.byref(st), ctypes.byref(o), _vp(labels), _vp(roles)))
    return labels[:N], roles[:N]
