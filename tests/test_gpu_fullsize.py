"""Full-size workloads against digests of the CPU oracle's results, written by
tests/golden/make_golden.py (which calls only the oracle and the seeded
generators).  Each test regenerates its input, checks the input's digest, and
compares the GPU library's results digest for digest.

- Chung-Lu n = 50,000,000 (exponent 2.1, mean degree 30, degree cap 1e6,
  seed 3; about 708 M edges) on the partition-based path under a 4 GiB device
  budget and on the in-memory path: labels and roles at (1/2, 10) and (1/10, 3),
  and the per-arc closed counts (Def. 5.1, Lemma 5.1, Alg. 5).
- 10,000 planted-partition graphs (n log-uniform in [100, 20000], mean degree
  U[8, 64], 5-200 blocks, per-graph eps in {1/5, 2/5, 3/5, 4/5} and mu in
  2..10, seed 4; about 677 M edges in all) clustered in one persistent batched
  run: every graph's labels and roles.
- Serving: 64 resident R-MAT graphs (scale 16..23, edge factor 8..32) and 8
  more added while queries run, under a device budget that keeps the last one
  on the host (its queries take the partition-based path): two stored oracle
  results per graph, and every query of a concurrent stream equal to the same
  query run alone.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import paper_2311_12281_amd as S
from gpu_helpers import note

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from digest import counts_digest, csr_digest, result_digest  # noqa: E402

pytestmark = pytest.mark.gpu


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as fh:
        return json.load(fh)


def test_chunglu_50m_partitioned_and_in_memory_match_oracle():
    gold = _golden("chunglu_n50m_seed3.json")
    t = time.perf_counter()
    g = gg.chung_lu(gold["n"], gold["mean_deg"], gold["exponent"], gold["max_deg"], seed=gold["seed"])
    note("chung-lu 50M generated", f"m={g.m}", f"{time.perf_counter() - t:.0f}s")
    assert g.m == gold["m"] and csr_digest(g) == gold["csr_sha256"], "input differs from the one the oracle saw"
    for budget in (4 << 30, 0):
        t = time.perf_counter()
        with S.Graph.from_csr(g, budget=budget) as G:
            note("chung-lu 50M", f"budget={budget}", f"created in {time.perf_counter() - t:.0f}s")
            for run in gold["runs"]:
                (p, q), mu = run["eps"], run["mu"]
                t = time.perf_counter()
                labels, roles = G.run(p, q, mu)
                note(f"budget={budget} eps={p}/{q} mu={mu}", f"{time.perf_counter() - t:.2f}s",
                     f"cores={int((roles == 1).sum())}")
                assert int((roles == 1).sum()) == run["cores"] and int((roles == 2).sum()) == run["borders"]
                assert result_digest(labels, roles) == run["result_sha256"], f"budget={budget} eps={p}/{q} mu={mu}"
                del labels, roles
            counts = G.similarity()
            assert counts_digest(counts) == gold["counts_sha256"], f"budget={budget}: closed counts differ"
            del counts


def test_planted_batch_10000_matches_oracle():
    gold = _golden("planted_batch_10000_seed4.json")
    t = time.perf_counter()
    graphs, specs = gg.planted_batch(gold["count"], seed=gold["seed"])
    import hashlib
    h = hashlib.sha256()
    for g in graphs:
        h.update(bytes.fromhex(csr_digest(g)))
    note("planted batch generated", len(graphs), f"{time.perf_counter() - t:.0f}s")
    assert h.hexdigest() == gold["csr_sha256_of_digests"], "inputs differ from the ones the oracle saw"
    eps = [s.eps for s in specs]
    mus = [s.mu for s in specs]
    assert [list(e) for e in eps] == gold["eps"] and mus == gold["mu"]
    t = time.perf_counter()
    with S.Batch(graphs, eps, mus) as B:
        note("batch created", f"{time.perf_counter() - t:.0f}s")
        for rep in range(2):
            labels, roles = B.run(replay=True)
            note("batch run", rep, f"{B.stats()['ms_total']:.1f} ms")
            bad = [k for k, (l, r) in enumerate(zip(B.split(labels), B.split(roles)))
                   if result_digest(l, r)[:12] != gold["result_sha256_12"][k]]
            assert not bad, f"{len(bad)} graphs differ from the oracle, first {bad[:10]}"


def test_serving_64_graphs_with_uploads_match_oracle():
    import threading

    gold = _golden("serving_rmat72_seed5.json")
    res_specs, up_specs = gg.serving_specs(count=gold["count"], uploads=gold["uploads"], seed=gold["seed"])
    t = time.perf_counter()
    graphs = [sp.make() for sp in res_specs + up_specs]
    note("serving graphs generated", len(graphs), f"{time.perf_counter() - t:.0f}s")
    for k, (g, gr) in enumerate(zip(graphs, gold["graphs"])):
        assert g.m == gr["m"] and csr_digest(g) == gr["csr_sha256"], f"graph {k} differs from the oracle's input"
    resident, uploads = graphs[:gold["count"]], graphs[gold["count"]:]
    nslots = 4
    rng = np.random.default_rng(11)
    with S.Server(num_slots=nslots) as srv:
        t = time.perf_counter()
        gids = [srv.add(g) for g in resident]
        note("resident graphs added", f"{time.perf_counter() - t:.0f}s", srv.info())
        stream = []  # (gid, p, q, mu, labels digest) of every query of the concurrent stream
        lock = threading.Lock()
        up_gids = []

        def uploader():
            for j, g in enumerate(uploads):
                if j == len(uploads) - 1:
                    # the admission limit drops to what is held now: the last upload stays on the host
                    srv.set_budget(srv.info()["resident_bytes"] + (32 << 20))
                gid = srv.add(g)
                with lock:
                    up_gids.append(gid)

        th = threading.Thread(target=uploader)
        th.start()
        pending = []
        while th.is_alive() or len(pending) < 600:
            with lock:
                pool = gids + up_gids[:-1] if len(up_gids) == len(uploads) else gids + up_gids
            gid = pool[int(rng.integers(len(pool)))]
            p, mu = int(rng.integers(1, 10)), int(rng.integers(2, 21))
            pending.append((srv.submit(gid, p, 10, mu), gid, p, mu))
            if len(pending) % 50 == 0:
                for r, gid_, p_, mu_ in pending[-50:]:
                    lab, rol, _ = srv.wait(r, gid_)
                    stream.append((gid_, p_, mu_, result_digest(lab, rol)))
            if len(pending) > 3000:
                break
        th.join()
        for r, gid_, p_, mu_ in pending[len(stream):]:
            lab, rol, _ = srv.wait(r, gid_)
            stream.append((gid_, p_, mu_, result_digest(lab, rol)))
        info = srv.info()
        note("stream done", len(stream), info)
        assert info["graphs"] == len(graphs) and info["resident_graphs"] == len(graphs) - 1
        all_gids = gids + up_gids
        for k, gr in enumerate(gold["graphs"]):
            for run in gr["runs"]:
                (p, q), mu = run["eps"], run["mu"]
                lab, rol, _ = srv.wait(srv.submit(all_gids[k], p, q, mu), all_gids[k])
                assert result_digest(lab, rol) == run["result_sha256"], f"graph {k} eps={p}/{q} mu={mu}"
        note("oracle digests matched", sum(len(gr["runs"]) for gr in gold["graphs"]))
        alone = {}
        for gid, p, mu, d in stream:
            if (gid, p, mu) not in alone:
                lab, rol, _ = srv.wait(srv.submit(gid, p, 10, mu), gid)
                alone[(gid, p, mu)] = result_digest(lab, rol)
            assert alone[(gid, p, mu)] == d, f"graph {gid} eps={p}/10 mu={mu}: differs from its alone-run"
        note("alone-runs matched", len(stream), "queries,", len(alone), "distinct")
