"""Shared helpers for the GPU tests: every call goes through the C-ABI."""
from __future__ import annotations

import numpy as np

import paper_2311_12281_amd as S


def note(*args):
    """Name the case before a GPU step (and flush), so a failing run says which."""
    print("[gpu-case]", *args, flush=True)


def assert_groups_whole(G, ctx=""):
    """The LDS-hash kernel's groups of lanes must each claim one chunk together."""
    split = G.stats()["group_split"]
    assert split == 0, f"{ctx}: {split} lanes claimed a chunk apart from their group"


def gpu_run(g, p, q, mu, **opts):
    with S.Graph.from_csr(g, **opts) as G:
        out = G.run(p, q, mu)
        assert_groups_whole(G, f"run eps={p}/{q} mu={mu}")
        return out


def gpu_counts(g, **opts):
    with S.Graph.from_csr(g, **opts) as G:
        out = G.similarity()
        assert_groups_whole(G, "similarity")
        return out


def assert_same(gl, gr, ol, orr, ctx=""):
    if not np.array_equal(gr, orr):
        bad = np.nonzero(gr != orr)[0]
        raise AssertionError(f"{ctx}: roles differ at {bad.size} vertices, first {bad[:10].tolist()} "
                             f"gpu {gr[bad[:10]].tolist()} oracle {orr[bad[:10]].tolist()}")
    if not np.array_equal(gl, ol):
        bad = np.nonzero(gl != ol)[0]
        raise AssertionError(f"{ctx}: labels differ at {bad.size} vertices, first {bad[:10].tolist()} "
                             f"gpu {gl[bad[:10]].tolist()} oracle {ol[bad[:10]].tolist()}")
