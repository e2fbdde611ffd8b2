"""Planted mistakes in copies of the oracle (CPU only): every mutant must fail
at least one pin, so that the pins in pins.py are shown to constrain each part
of the oracle (closed sets, the eps comparison, the core count, the cluster
search, the border rule and the per-arc bookkeeping).  Equivalent rewrites
(for example counting each edge from its other endpoint, which gives the same
integers) are not mistakes and are not listed."""
import os
import shutil
import subprocess

import pytest

import oracle
import pins

MUTANTS = {
    "open_neighbourhood_in_counts": ("mark[u] = 1;\n      for", "mark[u] = 0;\n      for"),
    "drop_self_of_smaller_side": ("int64_t c = mark[v];", "int64_t c = 0;"),
    "strict_eps_comparison": ("return lhs >= rhs;", "return lhs > rhs;"),
    "open_sizes_in_similarity": ("rp[u + 1] - rp[u] + 1, rp[v + 1] - rp[v] + 1",
                                 "rp[u + 1] - rp[u], rp[v + 1] - rp[v]"),
    "p_q_swapped": ("(uint64_t)(c * q) * (uint64_t)(c * q)", "(uint64_t)(c * p) * (uint64_t)(c * p)"),
    "core_count_without_self": ("int64_t ne = 1;", "int64_t ne = 0;"),
    "core_strict_threshold": ("core[u] = (uint8_t)(ne >= mu);", "core[u] = (uint8_t)(ne > mu);"),
    "bfs_through_non_cores": ("if (sim[i] && core[v] && labels[v] == -1)", "if (sim[i] && labels[v] == -1)"),
    "bfs_ignores_similarity": ("if (sim[i] && core[v] && labels[v] == -1)", "if (core[v] && labels[v] == -1)"),
    "label_is_last_core": ("labels[v] = s;", "labels[v] = x;"),
    "border_max_label": ("labels[u] < best)) best", "labels[u] > best)) best"),
    "border_ignores_similarity": ("if (core[u] && sim[i] && (best", "if (core[u] && (best"),
    "twin_arc_not_written": ("counts[rp[v] + row_find(ci + rp[v], dv, u)] = (int32_t)c;", ""),
    "closed_merge_off_by_one": ("if (k < at) return row[k];", "if (k <= at) return row[k];"),
    "hub_needs_one_cluster": ("else if (c != first) distinct = 2;", "else distinct = 2;"),
    "hub_counts_unclustered_neighbours": ("if (c < 0) continue;", ""),
    "hub_relabels_clustered": ("if (roles[u] != ROLE_UNCLASSIFIED) continue;", ""),
    "validate_allows_asymmetry": ("if (row_find(ci + rp[v], rp[v + 1] - rp[v], u) < 0) return OR_GRAPH;",
                                  ""),
}


@pytest.fixture(scope="module")
def source():
    with open(oracle.SRC) as f:
        return f.read()


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(src)],
                   check=True, capture_output=True)
    orc = oracle.Oracle(str(lib))
    failures = []
    for check in pins.QUICK_CHECKS:
        try:
            check(orc)
        except AssertionError:
            failures.append(check)
            break
    assert failures, f"mutant {name} passed every pin"
