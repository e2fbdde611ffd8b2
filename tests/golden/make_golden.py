"""Writes the stored expected results of the full-size workloads.

Every value written here comes from the CPU oracle (``oracle/``) run on inputs
from the seeded generators (``graphgen/``); nothing is taken from the GPU
library.  The GPU tests regenerate the same inputs, check their digests, and
compare the library's outputs with the digests stored here.

    python tests/golden/make_golden.py chunglu   # partition-based path workload
    python tests/golden/make_golden.py batch     # 10,000 planted-partition graphs
    python tests/golden/make_golden.py serving   # 72 R-MAT graphs, sampled queries

Outputs (JSON, next to this script):
  chunglu_n50m_seed3.json     Chung-Lu n = 50,000,000, exponent 2.1, mean degree
                              30, degree cap 1e6, seed 3: CSR digest, per-arc
                              closed-count digest, and the result digest at
                              (eps, mu) = (1/2, 10) and (1/10, 3)
  planted_batch_10000_seed4.json
                              per graph of the batch: the first 12 hex digits of
                              its result digest at its own (eps, mu); one digest
                              over all graphs' CSR digests
  serving_rmat72_seed5.json   per graph (64 resident + 8 uploads): CSR digest
                              and two (eps, mu) queries with their result digests
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402
from digest import counts_digest, csr_digest, result_digest, summary  # noqa: E402

CHUNGLU = dict(n=50_000_000, mean_deg=30.0, exponent=2.1, max_deg=1.0e6, seed=3)
CHUNGLU_RUNS = [((1, 2), 10), ((1, 10), 3)]
BATCH = dict(count=10_000, seed=4)
SERVING = dict(count=64, uploads=8, seed=5)
SERVING_CHECKS_PER_GRAPH = 2
SERVING_CHECK_SEED = 55


def log(*a):
    print("[golden]", *a, file=sys.stderr, flush=True)


def make_chunglu(out):
    t = time.perf_counter()
    g = gg.chung_lu(CHUNGLU["n"], CHUNGLU["mean_deg"], CHUNGLU["exponent"], CHUNGLU["max_deg"],
                    seed=CHUNGLU["seed"])
    log(f"Chung-Lu n={g.n} m={g.m} generated in {time.perf_counter() - t:.0f}s")
    rec = {"workload": "chunglu", **CHUNGLU, "m": g.m, "nnz": g.nnz,
           "max_degree": int(g.degrees().max()), "csr_sha256": csr_digest(g)}
    t = time.perf_counter()
    cnt = oracle.counts(g, threads=oracle.max_threads())
    rec["oracle_counts_s"] = round(time.perf_counter() - t, 1)
    rec["oracle_threads"] = oracle.max_threads()
    log(f"oracle counts in {rec['oracle_counts_s']}s")
    rec["counts_sha256"] = counts_digest(cnt)
    rec["runs"] = []
    for (p, q), mu in CHUNGLU_RUNS:
        t = time.perf_counter()
        lab, rol = oracle.cluster(g, cnt, p, q, mu)
        r = {"eps": [p, q], "mu": mu, "result_sha256": result_digest(lab, rol), **summary(lab, rol)}
        log(f"eps={p}/{q} mu={mu}: {r} ({time.perf_counter() - t:.0f}s)")
        rec["runs"].append(r)
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)


def _batch_one(k):
    spec = gg.planted_batch_specs(BATCH["count"], seed=BATCH["seed"])[k]
    g = gg.planted(spec.n, spec.blocks, spec.p_in, spec.p_out, spec.seed)
    lab, rol = oracle.scan(g, spec.eps[0], spec.eps[1], spec.mu)
    return csr_digest(g), result_digest(lab, rol)[:12], g.m, int((rol == 1).sum())


def _batch_chunk(ks):
    return [_batch_one(k) for k in ks]


def make_batch(out):
    count = BATCH["count"]
    specs = gg.planted_batch_specs(count, seed=BATCH["seed"])
    t = time.perf_counter()
    chunks = [list(range(i, min(count, i + 100))) for i in range(0, count, 100)]
    with ProcessPoolExecutor(max_workers=os.cpu_count()) as ex:
        res = [r for part in ex.map(_batch_chunk, chunks) for r in part]
    log(f"{count} graphs through the oracle in {time.perf_counter() - t:.0f}s")
    h = hashlib.sha256()
    for c, _, _, _ in res:
        h.update(bytes.fromhex(c))
    rec = {"workload": "planted_batch", **BATCH, "csr_sha256_of_digests": h.hexdigest(),
           "edges": int(sum(r[2] for r in res)), "graphs_with_cores": int(sum(r[3] > 0 for r in res)),
           "eps": [list(s.eps) for s in specs], "mu": [s.mu for s in specs],
           "result_sha256_12": [r[1] for r in res]}
    with open(out, "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))


def serving_checks(n_graphs):
    """(eps, mu) pairs checked against the oracle for every serving graph."""
    rng = np.random.default_rng(SERVING_CHECK_SEED)
    return [[(int(rng.integers(1, 10)), 10, int(rng.integers(2, 21))) for _ in range(SERVING_CHECKS_PER_GRAPH)]
            for _ in range(n_graphs)]


def make_serving(out):
    resident, uploads = gg.serving_specs(**SERVING)
    specs = resident + uploads
    checks = serving_checks(len(specs))
    graphs = []
    t0 = time.perf_counter()
    for k, sp in enumerate(specs):
        g = sp.make()
        cnt = oracle.counts(g, threads=oracle.max_threads())
        runs = []
        for p, q, mu in checks[k]:
            lab, rol = oracle.cluster(g, cnt, p, q, mu)
            runs.append({"eps": [p, q], "mu": mu, "result_sha256": result_digest(lab, rol), **summary(lab, rol)})
        graphs.append({"scale": sp.scale, "edge_factor": sp.edge_factor, "seed": sp.seed, "n": g.n, "m": g.m,
                       "csr_sha256": csr_digest(g), "runs": runs})
        log(f"graph {k}: scale {sp.scale} ef {sp.edge_factor} m={g.m} ({time.perf_counter() - t0:.0f}s)")
        del g, cnt
    rec = {"workload": "serving", **SERVING, "check_seed": SERVING_CHECK_SEED, "graphs": graphs}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["chunglu", "batch", "serving"])
    a = ap.parse_args()
    if a.which == "chunglu":
        make_chunglu(os.path.join(HERE, "chunglu_n50m_seed3.json"))
    elif a.which == "batch":
        make_batch(os.path.join(HERE, "planted_batch_10000_seed4.json"))
    else:
        make_serving(os.path.join(HERE, "serving_rmat72_seed5.json"))


if __name__ == "__main__":
    main()
