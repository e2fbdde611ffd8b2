"""Content digests of graphs and clustering results, shared by the script that
writes the stored expected values (``make_golden.py``, which calls only the
oracle and the input generators) and by the tests that compare the GPU
library's outputs with them.  No clustering arithmetic lives here.

Every digest is the SHA-256 of the little-endian bytes of the arrays, in a
fixed order and dtype, so it does not depend on the machine or on numpy's
default types.
"""
from __future__ import annotations

import hashlib

import numpy as np


def _update(h, a, dtype):
    a = np.ascontiguousarray(a, dtype=np.dtype(dtype).newbyteorder("<"))
    h.update(memoryview(a).cast("B"))


def csr_digest(g) -> str:
    """row_ptr as int64 then col_idx as int32."""
    h = hashlib.sha256()
    _update(h, g.row_ptr, np.int64)
    _update(h, g.col_idx[: g.nnz], np.int32)
    return h.hexdigest()


def result_digest(labels, roles) -> str:
    """labels as int32 then roles as uint8."""
    h = hashlib.sha256()
    _update(h, labels, np.int32)
    _update(h, roles, np.uint8)
    return h.hexdigest()


def counts_digest(counts) -> str:
    """Per-arc closed counts as int32 (CSR order)."""
    h = hashlib.sha256()
    _update(h, counts, np.int32)
    return h.hexdigest()


def summary(labels, roles) -> dict:
    """Plain figures of a result, stored beside its digest for a readable diff."""
    roles = np.asarray(roles)
    labels = np.asarray(labels)
    core = roles == 1
    return {"cores": int(core.sum()), "borders": int((roles == 2).sum()),
            "clusters": int(np.unique(labels[core]).size) if core.any() else 0}
