"""Benchmark: exact structural clustering of an R-MAT graph on one MI355X.

Workload: R-MAT scale 22 (4,194,304 vertices), edge factor 16,
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), symmetrised, deduplicated,
self-loops removed (seeded synthetic stand-in for the paper's real graphs).
One step clusters the resident graph at eps = 1/5, 1/2 and 4/5 with mu = 5
(three scan_run_device calls, outputs left in device memory).

value = (3 * |E| per step) / (wall time per step): undirected edges per second
of solve time with the graph resident in HBM.  The result of every eps is
compared with the CPU oracle and the line reports whether all match exactly.

roofline: the dominant kernel is the similarity/core kernel of the degree
bucket with the most device time; its algorithmic bytes per launch are
sum over intersected edges of (4 * smaller-list elements consumed + 8 bytes of
endpoints + 1 byte of edge state), divided by its launch duration measured
with HIP events on the library's stream, against 8 TB/s.

cpu_baseline: the oracle (not tuned) on the host cores, on the same graph at
eps = 1/2, mu = 5: closed counts of every edge plus clustering.

Other workloads (their own JSON line, not the default):
  --workload partitioned  Chung-Lu power-law graph under a device budget,
                          partition-based path vs in-memory path;
  --workload serving      resident R-MAT graphs, Poisson query stream,
                          served (cached counts, continuous batching) vs
                          plain per-query scan_run: p50/p99 latency, edges/s;
  --workload batched      many planted-partition graphs in one captured
                          launch vs one scan_run per graph;
  --workload sweep        R-MAT scale 22 over eps at mu = 6 and over mu at eps = 1/2;
  --workload planted      planted partition n = 10,000 with the oracle at
                          one thread and at all threads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
EPS_SET = [(1, 5), (1, 2), (4, 5)]
MU = 5


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-eps10", action="store_true",
                    help="skip the eps=1/10 timing (profiler runs: only the headline eps launch the kernels)")
    ap.add_argument("--workload", default="rmat",
                    choices=["rmat", "planted", "partitioned", "serving", "batched", "sweep"])
    ap.add_argument("--cl-n", type=int, default=50_000_000, help="partitioned: Chung-Lu vertices")
    ap.add_argument("--budget-gb", type=float, default=4.0, help="partitioned: device budget")
    ap.add_argument("--serve-graphs", type=int, default=64, help="serving: resident R-MAT graphs")
    ap.add_argument("--serve-uploads", type=int, default=8, help="serving: graphs added during the stream")
    ap.add_argument("--serve-upload-every", type=float, default=1.0, help="serving: seconds between uploads")
    ap.add_argument("--serve-queries", type=int, default=10000)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-waiters", type=int, default=4, help="serving: client threads collecting results")
    ap.add_argument("--serve-plain-seconds", type=float, default=10.0,
                    help="serving: arrivals of the plain comparison (bounded run)")
    ap.add_argument("--batch-count", type=int, default=10000)
    ap.add_argument("--batch-trace", action="store_true",
                    help="batched: default launch parameters, only the timed replays (for a kernel trace)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the HBM copy calibration")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="DIR",
                    help="print the HBM traffic summary of rocprofv3 --pmc runs of this bench (FETCH_SIZE, "
                         "WRITE_SIZE, read requests by size, DRAM requests)")
    ap.add_argument("--pmc-kernel", default="k_hub<0>")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="print a markdown table of the rocprofv3 --stats kernel summary under DIR and exit")
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(args.summarize_stats)
        return
    if args.summarize_pmc:
        return summarize_pmc(args)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr, flush=True)
        sys.exit(2)

    if args.workload == "partitioned":
        return bench_partitioned(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "planted":
        return bench_planted(args)

    import graphgen as gg
    import paper_2311_12281_amd as S

    t = time.perf_counter()
    g = gg.rmat(args.scale, args.edge_factor, seed=args.seed)
    gen_s = time.perf_counter() - t
    log(f"R-MAT scale {args.scale} ef {args.edge_factor}: n={g.n} m={g.m} "
        f"max_deg={int(g.degrees().max())} generated in {gen_s:.1f}s")

    t = time.perf_counter()
    G = S.Graph.from_csr(g, timing=True)
    create_s = time.perf_counter() - t
    log(f"scan_graph_create (upload + validate + layout): {create_s * 1e3:.1f} ms")
    n, m = g.n, g.m
    outs = []
    for _ in EPS_SET:
        outs.append((S.scan_device_alloc(4 * n), S.scan_device_alloc(n)))

    def step(collect=None):
        for (p, q), (dl, dr) in zip(EPS_SET, outs):
            G.run_device(p, q, MU, dl, dr)
            if collect is not None:
                collect.append(G.stats())

    for _ in range(args.warmup):
        step()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(stats)
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = len(EPS_SET) * m * args.steps / (t1 - t0)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value / 1e9:.3f} G edges/s")

    # dominant kernel: the cores-phase bucket kernel with the most device time
    nb = len(stats[0]["ms_cores_bucket"])
    ms_b = np.zeros(nb)
    bytes_b = np.zeros(nb)
    for st in stats:
        ms_b += np.array(st["ms_cores_bucket"])
        bytes_b += 4.0 * np.array(st["cores_bucket_probes"], dtype=np.float64) + \
            9.0 * np.array(st["cores_bucket_evaluated"], dtype=np.float64)
    dom = int(np.argmax(ms_b))
    launches = len(stats)
    achieved = (bytes_b[dom] / launches) / (ms_b[dom] / launches * 1e-3) / 1e9 if ms_b[dom] > 0 else 0.0
    per_eps = []
    for k, (p, q) in enumerate(EPS_SET):
        sts = stats[k::len(EPS_SET)]
        per_eps.append({
            "eps": f"{p}/{q}",
            "ms_device": float(np.mean([s["ms_total"] for s in sts])),
            "ms_phase": {ph: float(np.mean([s["ms_phase"][ph] for s in sts])) for ph in S.PHASES},
            "evaluated_cores": int(sts[-1]["evaluated"]["cores"]),
            "bounded_cores": int(sts[-1]["bounded"]["cores"]),
            "probes_cores": int(sts[-1]["probes"]["cores"]),
            "evaluated_merge": int(sts[-1]["evaluated"]["merge"]),
            "evaluated_attach": int(sts[-1]["evaluated"]["attach"]),
            "ms_cores_bucket": [float(np.mean([s["ms_cores_bucket"][b] for s in sts])) for b in range(nb)],
        })
        log(f"eps={p}/{q}: {per_eps[-1]}")

    # HBM reference: a plain streaming copy of --copy-mib MiB (read once, written once); the byte
    # counters of the dominant kernel are scaled by what they read for this copy
    copy_bytes = args.copy_mib << 20
    csrc_ = S.scan_device_alloc(copy_bytes)
    cdst_ = S.scan_device_alloc(copy_bytes)
    copy_ms = S.scan_device_copy(cdst_, csrc_, copy_bytes, iters=5)
    read_bytes = 8 * copy_bytes  # long enough for a steady rate
    S.scan_device_free(cdst_)
    S.scan_device_free(csrc_)
    copy_gbps = 2.0 * copy_bytes / (copy_ms * 1e-3) / 1e9
    rbuf = S.scan_device_alloc(read_bytes)
    read_ms = S.scan_device_read(rbuf, read_bytes, iters=5)
    S.scan_device_free(rbuf)
    read_gbps = read_bytes / (read_ms * 1e-3) / 1e9
    log(f"streaming copy {args.copy_mib} MiB: {copy_ms:.3f} ms -> {copy_gbps:.0f} GB/s; "
        f"read-only stream {read_bytes >> 20} MiB: {read_ms:.3f} ms -> {read_gbps:.0f} GB/s")
    dom_kernel = "k_hub<0>" if dom == nb - 1 else f"k_group<0, *> (bucket {dom})"
    traffic = _traffic_from_profile(dom_kernel)
    byte_models = solve_byte_models(g, stats[-len(EPS_SET):], traffic,
                                    float(bytes_b[dom] / launches) if launches else None)
    log(f"byte models: {byte_models}")
    # every bucket's kernel against the same roofline, and the whole cores pass
    # (the intersection bytes above, and beside them the same plus the classification stream:
    # 8 bytes of endpoints, 8 of degrees and 1 of edge state for every edge of the bucket)
    buckets = []
    for b in range(nb):
        ms_l = ms_b[b] / launches
        alg_l = bytes_b[b] / launches
        eb = int(stats[0]["bucket_edges"][b])
        cls_l = alg_l + 17.0 * eb
        buckets.append({"bucket": b, "launch_ms": float(ms_l), "alg_bytes_per_launch": float(alg_l),
                        "achieved_GBs": float(alg_l / (ms_l * 1e-3) / 1e9) if ms_l > 0 else 0.0,
                        "frac": float(alg_l / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS) if ms_l > 0 else 0.0,
                        "edges": eb,
                        "edges_per_s": float(eb / (ms_l * 1e-3)) if ms_l > 0 else 0.0,
                        "bytes_incl_classify_per_launch": float(cls_l),
                        "frac_incl_classify": float(cls_l / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS) if ms_l > 0 else 0.0})
    cores_ms = sum(st["ms_phase"]["cores"] for st in stats) / launches
    cores_alg = float(bytes_b.sum() / launches)
    cores_pass = {"launch_ms": cores_ms, "alg_bytes_per_launch": cores_alg,
                  "frac": cores_alg / (cores_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if cores_ms > 0 else 0.0}
    # the non-degenerate point of this graph (eps = 1/10 has cores and clusters), timed beside the step
    dl10, dr10 = S.scan_device_alloc(4 * n), S.scan_device_alloc(n)
    eps10 = None
    if not args.no_eps10:
        for _ in range(2):
            G.run_device(1, 10, MU, dl10, dr10)
        t10 = []
        st10 = None
        for _ in range(max(3, args.steps // 2)):
            t = time.perf_counter()
            G.run_device(1, 10, MU, dl10, dr10)
            t10.append(time.perf_counter() - t)
            st10 = G.stats()
        eps10 = {"eps": "1/10", "ms_wall": float(np.median(t10) * 1e3), "ms_device": st10["ms_total"],
                 "ms_phase": st10["ms_phase"], "edges_per_s": float(m / np.median(t10))}
        log(f"eps=1/10 (not in the headline step): {eps10['ms_wall']:.1f} ms, "
            f"{eps10['edges_per_s'] / 1e9:.2f} G edges/s")

    # PCIe-inclusive rate (host outputs), reported beside the value
    t = time.perf_counter()
    host_out = [G.run(p, q, MU) for (p, q) in EPS_SET]
    e2e_rate = len(EPS_SET) * m / (time.perf_counter() - t)

    t = time.perf_counter()
    G.similarity()
    sim_ms = (time.perf_counter() - t) * 1e3
    sim_stats = G.stats()

    exact = None
    cpu = None
    if not args.no_cpu_baseline or not args.no_verify:
        import oracle
        threads = oracle.max_threads()
        log(f"oracle on {threads} host threads (counts of every edge + clustering, eps=1/2)")
        t = time.perf_counter()
        ol, orr, oc = oracle.scan(g, 1, 2, MU, threads=threads, want_counts=True)
        cpu_s = time.perf_counter() - t
        cpu = {"value": m / cpu_s, "unit": "edges/s", "cores": threads, "kind": "oracle",
               "sample": f"full R-MAT scale {args.scale} graph (m={m}) at eps=1/2 mu={MU}: "
                         f"closed counts of every edge + clustering, {cpu_s:.1f} s",
               "cpu_model": _cpu_model()}
        log(f"oracle: {cpu_s:.1f} s -> {m / cpu_s / 1e6:.2f} M edges/s")
        if not args.no_cpu_baseline:
            # one thread, on a bounded sample: R-MAT scale 20 from the same generator
            g1 = gg.rmat(args.scale - 2, args.edge_factor, seed=args.seed)
            t = time.perf_counter()
            oracle.scan(g1, 1, 2, MU, threads=1)
            t1 = time.perf_counter() - t
            cpu["t1"] = {"value": g1.m / t1, "unit": "edges/s", "cores": 1,
                         "sample": f"R-MAT scale {args.scale - 2} ef {args.edge_factor} (m={g1.m}) at eps=1/2 "
                                   f"mu={MU}, one thread: {t1:.1f} s"}
            log(f"oracle, one thread, R-MAT scale {args.scale - 2}: {t1:.1f} s -> {g1.m / t1 / 1e6:.2f} M edges/s")
            del g1
        if not args.no_verify:
            exact = True
            for k, (p, q) in enumerate(EPS_SET):
                dl, dr = outs[k]
                gl = np.empty(n, np.int32)
                gr = np.empty(n, np.uint8)
                S.scan_memcpy_d2h(gl, dl, 4 * n)
                S.scan_memcpy_d2h(gr, dr, n)
                rl, rr = oracle.cluster(g, oc, p, q, MU)
                ok = (np.array_equal(gl, rl) and np.array_equal(gr, rr)
                      and np.array_equal(host_out[k][0], rl) and np.array_equal(host_out[k][1], rr))
                log(f"eps={p}/{q}: exact match with oracle: {ok} "
                    f"(cores {int((rr == 1).sum())}, borders {int((rr == 2).sum())})")
                exact = exact and ok
        if args.no_cpu_baseline:
            cpu = None

    for dl, dr in outs:
        S.scan_device_free(dl)
        S.scan_device_free(dr)
    G.close()

    line = {
        "metric": "edges/s (|E|/solve) exact-match",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef{args.edge_factor}_scan",
                   "generator": "R-MAT (0.57,0.19,0.19,0.05), symmetrised, dedup, no self-loops",
                   "seed": args.seed, "n": n, "m": m, "eps": [f"{p}/{q}" for p, q in EPS_SET],
                   "mu": MU, "step": "one scan_run_device per eps, graph resident"},
        "exact_match": exact,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{dom_kernel}: cores pass, degree bucket {dom}",
                     "copy_gbps": copy_gbps, "read_gbps": read_gbps,
                     "launch_ms": float(ms_b[dom] / launches),
                     "alg_bytes_per_launch": float(bytes_b[dom] / launches)},
        "cpu_baseline": cpu,
        "pcie_inclusive_edges_per_s": e2e_rate,
        "scan_similarity_ms": sim_ms,
        "scan_similarity_device_ms": sim_stats["ms_total"],
        "graph_create_ms": create_s * 1e3,
        "per_eps": per_eps,
        "eps_1_10": eps10,
        "cores_pass": cores_pass,
        "buckets": buckets,
        "byte_models": byte_models,
    }
    S.scan_device_free(dl10)
    S.scan_device_free(dr10)
    print(json.dumps(line), flush=True)


def solve_byte_models(g, stats_per_eps, traffic=None, alg_per_launch=None):
    """Byte models of a whole solve: the measured intersections (4 bytes per element consumed + 9 per
    intersected edge, every bucket) plus each row read once as the probe side (4 nnz), the offsets
    (8 (n + 1)) and the per-vertex state (17 n), one figure per run in stats_per_eps (their
    cores_bucket_probes and cores_bucket_evaluated); beside them, for a solve that evaluates every edge
    without pruning, whole smaller lists (4 sum_e min(d_u, d_v) + 9 m) and both lists (the merge model,
    4 sum_e (d_u + d_v) = 4 sum_v d_v^2); and the dominant kernel's counted traffic over its algorithmic
    bytes per launch (None without a traffic figure)."""
    n = int(g.n)
    deg = np.diff(np.asarray(g.row_ptr)).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = np.asarray(g.col_idx, dtype=np.int64)
    own = src < dst
    m = int(g.m)
    sum_min = int(np.minimum(deg[src[own]], deg[dst[own]]).sum())
    sum_both = int((deg * deg).sum())
    fixed = 4.0 * int(g.nnz) + 8.0 * (n + 1) + 17.0 * n
    return {
        "per_eps_probe_model_bytes": [
            float(4.0 * np.sum(s_["cores_bucket_probes"]) + 9.0 * np.sum(s_["cores_bucket_evaluated"]) + fixed)
            for s_ in stats_per_eps],
        "full_evaluation_min_model_bytes": 4.0 * sum_min + 9.0 * m + fixed,
        "full_evaluation_merge_model_bytes": 4.0 * sum_both,
        "dominant_kernel_traffic_over_alg": (traffic / alg_per_launch) if traffic and alg_per_launch else None,
    }


def _cpu_model():
    """CPU model name and logical CPU count of this host (lscpu)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return None
    info = {}
    for ln in out.splitlines():
        if ":" in ln:
            k, v = ln.split(":", 1)
            info[k.strip()] = v.strip()
    return {"model": info.get("Model name"), "cpus": info.get("CPU(s)"), "nproc": os.cpu_count()}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_k_hub_cores_rmat22.md")
# counter passes beside the traffic ones (each within one pass's per-block limits)
LDS_COUNTERS = ["SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS", "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD",
                "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY"]
ATOMIC_COUNTERS = ["TCC_ATOMIC_sum", "TCC_EA0_ATOMIC_sum", "TCP_TCC_ATOMIC_WITH_RET_REQ_sum",
                   "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"]
KERNEL_SOURCES = ["kernels.hip", "layout.hip", "api.hip", "scan_internal.h"]


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_12281_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_from_profile(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when there is
    none for this kernel or the kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = {}
    with open(TRAFFIC_PROFILE) as fh:
        for ln in fh:
            if ln.startswith("- ") and ": " in ln:
                k, v = ln[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel") != kernel or kv.get("kernel_sources_sha256") != _kernel_source_hash():
        log(f"traffic: counter summary is for {kv.get('kernel')} / sources "
            f"{kv.get('kernel_sources_sha256')}, current {kernel} / {_kernel_source_hash()}: null")
        return None
    return float(kv["traffic_bytes_per_launch"])


def _pmc_rows(d):
    """(dispatch id, kernel name, counter, value) rows from rocprofv3 counter CSVs under d."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def _per_dispatch_mean(rows, counter, match):
    per = {}
    for did, name, c, v in rows:
        if c == counter and match(name):
            per[did] = per.get(did, 0.0) + v
    return (sum(per.values()) / len(per), len(per)) if per else (None, 0)


def summarize_pmc(args):
    """Markdown summary of HBM bytes per launch of the dominant kernel from
    rocprofv3 counter runs of this bench (one directory per run): FETCH_SIZE
    and WRITE_SIZE scaled by what they read for the plain copy kernel, the read
    requests by size (32, 64, 128 bytes: bytes without any scaling) and the
    share of read requests that went to DRAM."""
    rows = []
    for d in args.summarize_pmc:
        rows += _pmc_rows(d)
    is_copy = lambda nm: "k_copy16" in nm  # noqa: E731
    want = args.pmc_kernel
    is_k = lambda nm: want in nm  # noqa: E731
    got = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
              "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_DRAM_sum"):
        got[c] = (_per_dispatch_mean(rows, c, is_copy), _per_dispatch_mean(rows, c, is_k))
    (cf, ncf), (kf, nkf) = got["FETCH_SIZE"]
    (cw, ncw), (kw, nkw) = got["WRITE_SIZE"]
    if None in (cf, cw, kf, kw):
        sys.exit(f"missing dispatches: copy {ncf}/{ncw}, {want} {nkf}/{nkw}")
    copy_kib = (args.copy_mib << 20) / 1024.0
    sf, sw = copy_kib / cf, copy_kib / cw
    fetch_scaled = kf * sf * 1024.0
    write_bytes = kw * sw * 1024.0

    def by_size(which):
        vals = [got[c][which][0] for c in ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")]
        return None if None in vals else 32.0 * vals[0] + 64.0 * vals[1] + 128.0 * vals[2]

    read_copy, read_k = by_size(0), by_size(1)
    read_bytes = read_k if read_k is not None else fetch_scaled
    traffic = read_bytes + write_bytes
    dram = got["TCC_EA0_RDREQ_DRAM_sum"][1][0]
    req = got["TCC_EA0_RDREQ_sum"][1][0]
    cmd = "python bench.py --summarize-pmc " + " ".join(args.summarize_pmc) + f" --pmc-kernel '{want}'"
    size_rows = ""
    for label, which in (("k_copy16", 0), (want, 1)):
        vals = [got[c][which][0] for c in ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum",
                                            "TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_DRAM_sum")]
        size_rows += "| " + label + " | " + " | ".join("-" if v is None else f"{v:.4g}" for v in vals) + " |\n"
    print(f"""# HBM traffic of {want} (cores pass, LDS-hash bucket), R-MAT scale 22

Commands (from the repository root on the MI355X host, each its own run):

```
rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o bench -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-verify --no-eps10
rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o bench -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-verify --no-eps10
rocprofv3 --pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum --output-format csv -d gpurun_out/pmc_rdreq -o bench -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-verify --no-eps10
rocprofv3 --pmc TCC_EA0_RDREQ_DRAM_sum TCC_EA0_RDREQ_sum --output-format csv -d gpurun_out/pmc_dram -o bench -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-verify --no-eps10
rocprofv3 --pmc {' '.join(LDS_COUNTERS)} --output-format csv -d gpurun_out/pmc_lds -o bench -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-verify --no-eps10
rocprofv3 --pmc {' '.join(ATOMIC_COUNTERS)} --output-format csv -d gpurun_out/pmc_atomic -o bench -- python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-verify --no-eps10
{cmd}
```

The copy kernel `k_copy16` moves {args.copy_mib} MiB (read once, written once) per dispatch; FETCH_SIZE
and WRITE_SIZE of the kernel are scaled by what they read for it (KiB per dispatch, mean over dispatches).

| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |
|---|---|---|---|
| k_copy16 | {ncf}/{ncw} | {cf:.0f} | {cw:.0f} |
| {want} | {nkf}/{nkw} | {kf:.0f} | {kw:.0f} |

Read requests by size (per dispatch; bytes = 32 n32 + 64 n64 + 128 n128, no scaling), all requests, and
those that went to DRAM:

| kernel | 32 B | 64 B | 128 B | all | to DRAM |
|---|---|---|---|---|---|
{size_rows}
- copy: read bytes by request size {"-" if read_copy is None else f"{read_copy:.4g}"} (moved: {args.copy_mib << 20}); FETCH_SIZE scale {sf:.4f}, WRITE_SIZE scale {sw:.4f}
- kernel read bytes: by request size {"-" if read_k is None else f"{read_k:.4g}"}, by scaled FETCH_SIZE {fetch_scaled:.4g}
- kernel write bytes (scaled WRITE_SIZE): {write_bytes:.4g}
- read requests that went to DRAM: {"-" if dram is None or not req else f"{dram / req:.3f}"}
- kernel: `{want}`
- kernel_sources_sha256: `{_kernel_source_hash()}`
- traffic_bytes_per_launch: {traffic:.0f}
""")
    # any further counters of the runs (LDS, atomics, instructions): per-dispatch means for the kernel
    known = {"FETCH_SIZE", "WRITE_SIZE", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum",
             "TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_DRAM_sum"}
    extra = sorted({c for _, nm, c, _ in rows if c not in known and is_k(nm)})
    if extra:
        print("Further counters of the kernel (per dispatch, mean over dispatches; SQ counters are sums over\n"
              "the shader engines, LDS cycle counters in the units rocprofv3 reports):\n")
        print("| counter | value |")
        print("|---|---|")
        vals = {}
        for c in extra:
            v, nd = _per_dispatch_mean(rows, c, is_k)
            vals[c] = v
            print(f"| {c} | {v:.4g} ({nd} dispatches) |")
        if vals.get("SQ_LDS_IDX_ACTIVE") and "SQ_LDS_BANK_CONFLICT" in vals:
            act, bc = vals["SQ_LDS_IDX_ACTIVE"], vals["SQ_LDS_BANK_CONFLICT"]
            print(f"\n- LDS bank-conflict cycles per conflict-free LDS cycle: {bc / max(act - bc, 1.0):.3f}")
        if vals.get("SQ_INSTS_LDS") and vals.get("SQ_INSTS_VALU"):
            print(f"- VALU instructions per LDS instruction: {vals['SQ_INSTS_VALU'] / vals['SQ_INSTS_LDS']:.2f}")
        print()
    bt = _bucket_traffic(rows, sf, sw)
    print("Every cores-pass kernel, by degree bucket (scaled FETCH_SIZE and WRITE_SIZE per dispatch, GB;")
    print("dispatches are those of the FETCH and WRITE runs together):\n")
    print("| bucket | kernel | dispatches | read GB | written GB |")
    print("|---|---|---|---|---|")
    kn = ["k_group<0, 4>", "k_group<0, 8>", "k_group<0, 16>", "k_group<0, 32>", "k_group<0, 64, staged>",
          "k_group<0, 64, staged>", "k_hub<0>"]
    for b in range(7):
        nd, f, w = bt.get(b, (0, None, None))
        print(f"| {b} | `{kn[b]}` | {nd} | {'-' if f is None else f'{f / 1e9:.3f}'} | "
              f"{'-' if w is None else f'{w / 1e9:.3f}'} |")


def _short_kernel(name):
    """Kernel name without namespaces, argument list and the default template arguments."""
    nm = name
    for pre in ("void ", "(anonymous namespace)::", "scan::"):
        nm = nm.replace(pre, "")
    nm = nm.split("(")[0].replace(", false>", ">").replace(", true>", ", staged>")
    return nm.strip()


def summarize_stats(d):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (csv output) under d."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        sys.exit(f"no kernel_stats.csv under {d}")
    rows = {}
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = _short_kernel(r["Name"])
                c, t = rows.get(k, (0, 0.0))
                rows[k] = (c + int(r["Calls"]), t + float(r["TotalDurationNs"]))
    total = sum(t for _, t in rows.values())
    print("| kernel | calls | total ms | average ms | % |")
    print("|---|---|---|---|---|")
    for k, (c, t) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        if t / total < 0.001:
            continue
        print(f"| `{k}` | {c} | {t / 1e6:.2f} | {t / c / 1e6:.3f} | {100 * t / total:.2f} |")


def _bucket_traffic(rows, sf, sw):
    """Scaled FETCH/WRITE bytes per dispatch of every cores-pass kernel, by degree bucket.  Buckets 4
    and 5 share one kernel (lanes 64, staged) and are told apart by launch order (4 before 5)."""
    names = [("k_group<0, 4,", (0,)), ("k_group<0, 8,", (1,)), ("k_group<0, 16,", (2,)),
             ("k_group<0, 32,", (3,)), ("k_group<0, 64, true", (4, 5)), ("k_hub<0>", (6,))]
    out = {}
    for key, bks in names:
        per = {}
        for did, nm, c, v in rows:
            if key in nm.replace("(scan::Mode)", "") and c in ("FETCH_SIZE", "WRITE_SIZE"):
                per.setdefault(int(did), {}).setdefault(c, 0.0)
                per[int(did)][c] += v
        ids = sorted(per)
        for j, b in enumerate(bks):
            mine = [per[i] for i in ids[j::len(bks)]]
            f = [x["FETCH_SIZE"] for x in mine if "FETCH_SIZE" in x]
            w = [x["WRITE_SIZE"] for x in mine if "WRITE_SIZE" in x]
            out[b] = (len(mine), sum(f) / len(f) * sf * 1024.0 if f else None,
                      sum(w) / len(w) * sw * 1024.0 if w else None)
    return out


def _line(metric, value, unit, config, **rest):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "higher_is_better": True,
         "vs_baseline": None, "dtype": "int32", "data": "synthetic", "config": config}
    d.update(rest)
    print(json.dumps(d), flush=True)


def bench_partitioned(args):
    """Chung-Lu (exponent 2.1, mean degree 30, degree cap 1e6) under a device
    budget: the partition-based path streams blocks over the host link; the
    in-memory path on the same graph gives the reference result and time."""
    import graphgen as gg
    import paper_2311_12281_amd as S

    t = time.perf_counter()
    g = gg.chung_lu(args.cl_n, 30.0, 2.1, 1.0e6, seed=3)
    log(f"Chung-Lu n={g.n} m={g.m} max_deg={int(g.degrees().max())} generated in {time.perf_counter() - t:.1f}s")
    budget = int(args.budget_gb * (1 << 30))
    t = time.perf_counter()
    P = S.Graph.from_csr(g, budget=budget, timing=True)
    create_p = time.perf_counter() - t
    t = time.perf_counter()
    M = S.Graph.from_csr(g, timing=True)
    create_m = time.perf_counter() - t
    rows = []
    exact = True
    for (p, q), mu in [((1, 2), 10), ((1, 10), 3)]:
        t = time.perf_counter()
        pl, pr = P.run(p, q, mu)
        tp = time.perf_counter() - t
        st = P.stats()
        t = time.perf_counter()
        ml, mr = M.run(p, q, mu)
        tm = time.perf_counter() - t
        same = bool(np.array_equal(pl, ml) and np.array_equal(pr, mr))
        exact = exact and same
        rows.append({"eps": f"{p}/{q}", "mu": mu, "partitioned_s": tp, "in_memory_s": tm,
                     "partitioned_ms_phase": st["ms_phase"],
                     "partitioned_edges_per_s": g.m / tp, "in_memory_edges_per_s": g.m / tm,
                     "h2d_GB": st["h2d_bytes"] / 1e9, "h2d_GB_per_s": st["h2d_bytes"] / 1e9 / tp,
                     "identical_to_in_memory": same, "cores": int((pr == 1).sum()),
                     "borders": int((pr == 2).sum())})
        log(rows[-1])
    P.close()
    M.close()
    link = S.scan_h2d_rate(1 << 30, 5)
    log(f"pinned H2D copy rate: {link / 1e9:.1f} GB/s")
    for r in rows:
        r["h2d_frac_of_link"] = r["h2d_GB_per_s"] * 1e9 / link
    _line("edges/s (|E|/solve) exact-match, partition-based path", g.m / rows[0]["partitioned_s"], "edges/s",
          {"workload": f"chunglu_n{g.n}_budget{args.budget_gb}GB", "n": g.n, "m": g.m, "eps": "1/2", "mu": 10},
          identical_to_in_memory=exact, h2d_link_GB_per_s=link / 1e9, create_partitioned_s=create_p, create_in_memory_s=create_m, runs=rows)


def bench_serving(args):
    """Resident R-MAT graphs (scale 16..23, edge factor 8..32) plus uploads
    added while the queries run; a Poisson stream of (graph, eps = k/10,
    mu) queries at 0.5x and 0.9x of the served path's saturation rate.
    Served: cached closed counts, re-thresholding, continuous batching over
    slots, memory admission (an upload that does not fit stays on the host
    and its queries take the partition-based path on the fallback thread).
    Plain: one scan_run per query on resident graphs, first come first served,
    at 0.5x and 0.9x of its own saturation and at the served path's rates.
    Latency = completion - arrival.  Exactness: the
    stored oracle digests of two queries per graph, and every query of the
    Poisson runs against the same query run alone afterwards."""
    import threading

    import xxhash

    import graphgen as gg
    import paper_2311_12281_amd as S
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from digest import result_digest

    def fast_digest(labels, roles):
        # compares the stream's results with their alone-runs (the oracle
        # digests use result_digest); quick enough for the waiting thread
        h = xxhash.xxh3_128()
        h.update(np.ascontiguousarray(labels))
        h.update(np.ascontiguousarray(roles))
        return h.hexdigest()

    res_specs, up_specs = gg.serving_specs(count=args.serve_graphs, uploads=args.serve_uploads, seed=5)
    t = time.perf_counter()
    graphs = [sp.make() for sp in res_specs]
    uploads = [sp.make() for sp in up_specs]
    log(f"{len(graphs)} resident + {len(uploads)} upload R-MAT graphs, {sum(g.m for g in graphs)} + "
        f"{sum(g.m for g in uploads)} edges, generated in {time.perf_counter() - t:.0f}s")
    nslots = args.serve_slots
    srv = S.Server(num_slots=nslots)
    t = time.perf_counter()
    gids = [srv.add(g) for g in graphs]
    add_s = time.perf_counter() - t
    log(f"added {len(gids)} graphs in {add_s:.1f}s; held {srv.info()['resident_bytes'] / 2**30:.1f} GiB")
    budget = None
    all_graphs = graphs + uploads
    rng = np.random.default_rng(7)
    nq = args.serve_queries
    picks = rng.random(nq)
    eps_k = rng.integers(1, 10, size=nq)
    mus = rng.integers(2, 21, size=nq)

    def query(k, ngraphs):
        return int(picks[k] * ngraphs), int(eps_k[k]), 10, int(mus[k])

    # results are collected by --serve-waiters client threads, each copying into buffers of its own
    # (allocated once: a fresh array per result would be page-faulted in on every copy)
    nwait = max(1, args.serve_waiters)
    nmax = max(g.n for g in graphs + uploads)
    bufs = [(np.empty(nmax, np.int32), np.empty(nmax, np.uint8)) for _ in range(nwait)]

    # saturation: the whole query list on the resident graphs, submitted at once
    t0 = time.perf_counter()
    reqs = [(srv.submit(gids[gi], p, q, mu), gi) for gi, p, q, mu in (query(k, len(gids)) for k in range(nq))]

    def sat_waiter(t):
        lb, rb = bufs[t]
        for r, gi in reqs[t::nwait]:
            srv.wait(r, gids[gi], lb, rb)

    ths = [threading.Thread(target=sat_waiter, args=(t,)) for t in range(nwait)]
    for x in ths:
        x.start()
    for x in ths:
        x.join()
    sat_edges = float(sum(graphs[gi].m for _, gi in reqs))
    sat_s = time.perf_counter() - t0
    sat = nq / sat_s
    log(f"served saturation ({nwait} client threads): {sat:.0f} queries/s, {sat_edges / sat_s / 1e9:.2f} G edges/s")

    res_gids = list(gids)       # graphs queries may target (resident ones and uploads that became resident)
    upload_gids = []

    def run_served(qps, with_uploads):
        arr = np.cumsum(np.random.default_rng(int(qps)).exponential(1.0 / qps, size=nq))
        lat = [0.0] * nq
        dig = [None] * nq
        keys = [None] * nq
        ready = threading.Semaphore(0)
        take = threading.Lock()
        nxt = [0]
        start = time.perf_counter()

        def waiter(t):
            lb, rb = bufs[t]
            while True:
                ready.acquire()
                with take:
                    k = nxt[0]
                    nxt[0] += 1
                if k >= nq:
                    return
                r, gid = keys[k][0], keys[k][1]
                lab, rol, ms = srv.wait(r, gid, lb, rb)
                lat[k] = ms
                dig[k] = fast_digest(lab, rol)

        def uploader():
            nonlocal budget
            for j, g in enumerate(uploads):
                d = start + (j + 1) * args.serve_upload_every - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                if j == len(uploads) - 1:
                    # admission limit: what is held now; the last upload stays on the host
                    budget = srv.info()["resident_bytes"] + (32 << 20)
                    srv.set_budget(budget)
                gid = srv.add(g)
                g_index[gid] = len(graphs) + j
                upload_gids.append(gid)
                if srv.info()["resident_graphs"] == len(res_gids) + 1:
                    res_gids.append(gid)

        ths = [threading.Thread(target=waiter, args=(t,)) for t in range(nwait)]
        for x in ths:
            x.start()
        up = threading.Thread(target=uploader) if with_uploads else None
        if up:
            up.start()
        for k in range(nq):
            d = start + arr[k] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            pool = list(res_gids)
            gi, p, q, mu = query(k, len(pool))
            gid = pool[gi]
            keys[k] = (srv.submit(gid, p, q, mu), gid, p, q, mu)
            ready.release()
        for _ in range(nwait):  # one stop token per waiter
            ready.release()
        for x in ths:
            x.join()
        if up:
            up.join()
        wall = time.perf_counter() - start
        lat = np.array(lat)
        # latency from arrival: the submit happens at the arrival (to within the sleep's precision)
        edges = float(sum(all_graphs[g_index[key[1]]].m for key in keys))
        return lat, wall, edges, keys, dig

    g_index = {gid: i for i, gid in enumerate(gids)}
    out = {}
    checks = []
    for frac in (0.5, 0.9):
        qps = frac * sat
        with_up = frac == 0.5
        lat, wall, edges, keys, dig = run_served(qps, with_up)
        checks += [(k[1], k[2], k[3], k[4], d) for k, d in zip(keys, dig)]
        out[f"{frac}x"] = {"qps": qps, "queries": nq, "served_p50_ms": float(np.percentile(lat, 50)),
                           "served_p99_ms": float(np.percentile(lat, 99)), "served_edges_per_s": edges / wall,
                           "served_wall_s": wall}
        log(f"served {frac}x: {out[f'{frac}x']}")
    info = srv.info()
    log(f"server: {info}")
    # the upload kept on the host: its queries take the partition-based path
    fb_gid = [gid for gid in upload_gids if gid not in res_gids]
    fallback = None
    if fb_gid:
        gid = fb_gid[0]
        ms = [srv.wait(srv.submit(gid, k, 10, 5), gid)[2] for k in (3, 5, 7)]
        fallback = {"graph_edges": all_graphs[g_index[gid]].m, "latency_ms": ms}
        log(f"fallback queries: {fallback}")

    # plain: one scan_run per query on the resident graphs, first come first served, the same
    # query list; its own saturation (queries back to back), then Poisson arrivals at 0.5x and 0.9x
    # of that rate and at the served path's rates (where its queue grows).  Each run stops after
    # --serve-plain-seconds: latencies are those of the queries completed by then, and `backlog`
    # counts the queries that had arrived but were still waiting.
    plain_graphs = {gid: S.Graph.from_csr(all_graphs[g_index[gid]]) for gid in res_gids}

    def run_plain(qps, cnt):
        arr = np.cumsum(np.random.default_rng(int(qps)).exponential(1.0 / qps, size=cnt)) if qps else np.zeros(cnt)
        lat = []
        edges = 0.0
        lb, rb = bufs[0]
        start = time.perf_counter()
        for k in range(cnt):
            if time.perf_counter() - start > args.serve_plain_seconds:
                break
            d = start + arr[k] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            gi, p, q, mu = query(k, len(res_gids))
            gid = res_gids[gi]
            plain_graphs[gid].run(p, q, mu, lb, rb)
            lat.append((time.perf_counter() - start - arr[k]) * 1e3)
            edges += all_graphs[g_index[gid]].m
        wall = time.perf_counter() - start
        backlog = int(np.searchsorted(arr, wall, side="right")) - len(lat)
        return np.array(lat), edges, wall, backlog

    lat, edges, wall, _ = run_plain(0.0, nq)
    plain_sat = len(lat) / wall
    plain = {"saturation_qps": plain_sat, "saturation_edges_per_s": edges / wall, "saturation_queries": len(lat)}
    log(f"plain saturation: {plain_sat:.0f} queries/s, {edges / wall / 1e9:.2f} G edges/s")

    # plain with as many client threads as the served path's waiters (scan_run on different graphs
    # runs concurrently; calls on one graph take turns)
    done_q = [0] * nwait
    done_e = [0.0] * nwait
    t0 = time.perf_counter()

    def plain_client(t):
        lb, rb = bufs[t]
        for k in range(t, nq, nwait):
            if time.perf_counter() - t0 > args.serve_plain_seconds:
                return
            gi, p, q, mu = query(k, len(res_gids))
            gid = res_gids[gi]
            plain_graphs[gid].run(p, q, mu, lb, rb)
            done_q[t] += 1
            done_e[t] += all_graphs[g_index[gid]].m

    ths = [threading.Thread(target=plain_client, args=(t,)) for t in range(nwait)]
    for x in ths:
        x.start()
    for x in ths:
        x.join()
    wall = time.perf_counter() - t0
    plain["saturation_threads"] = {"threads": nwait, "qps": sum(done_q) / wall, "edges_per_s": sum(done_e) / wall}
    log(f"plain saturation, {nwait} client threads: {plain['saturation_threads']}")
    for frac in (0.5, 0.9):
        for label, qps in ((f"own_{frac}x", frac * plain_sat), (f"served_rate_{frac}x", frac * sat)):
            lat, edges, wall, backlog = run_plain(qps, nq)
            plain[label] = {"qps": qps, "queries": len(lat), "p50_ms": float(np.percentile(lat, 50)),
                            "p99_ms": float(np.percentile(lat, 99)), "edges_per_s": edges / wall,
                            "backlog": backlog}
            log(f"plain {label}: {plain[label]}")
    for G in plain_graphs.values():
        G.close()

    # exactness 1: two stored oracle results per graph (64 resident + uploads)
    gold_path = os.path.join(ROOT, "tests", "golden", "serving_rmat72_seed5.json")
    oracle_ok = None
    if os.path.exists(gold_path) and args.serve_graphs == 64 and args.serve_uploads == 8:
        import json as _json
        with open(gold_path) as fh:
            gold = _json.load(fh)
        oracle_ok = True
        all_gids = gids + upload_gids
        for i, gr in enumerate(gold["graphs"]):
            gid = all_gids[i]
            for run in gr["runs"]:
                (p, q), mu = run["eps"], run["mu"]
                lab, rol, _ = srv.wait(srv.submit(gid, p, q, mu), gid)
                oracle_ok = oracle_ok and result_digest(lab, rol) == run["result_sha256"]
        log(f"oracle digests ({sum(len(gr['runs']) for gr in gold['graphs'])} queries): {oracle_ok}")
    # exactness 2: every query of the Poisson runs equals the same query alone
    alone = {}
    alone_ok = True
    for gid, p, q, mu, d in checks:
        key = (gid, p, q, mu)
        if key not in alone:
            lab, rol, _ = srv.wait(srv.submit(gid, p, q, mu), gid)
            alone[key] = fast_digest(lab, rol)
        alone_ok = alone_ok and alone[key] == d
    log(f"every query equals its alone-run: {alone_ok} ({len(checks)} queries, {len(alone)} distinct)")
    srv.close()
    _line("queries/s at saturation, served (cached counts, continuous batching)", sat, "queries/s",
          {"workload": f"serving_rmat{len(graphs)}+{len(uploads)}_s16-23_ef8-32", "resident_graphs": len(graphs),
           "uploads": len(uploads), "queries": nq, "slots": nslots, "client_threads": nwait,
           "budget_bytes": budget},
          saturation_edges_per_s=sat_edges / sat_s, add_graphs_s=add_s, oracle_digests_exact=oracle_ok,
          alone_run_exact=alone_ok, fallback=fallback, poisson=out, plain=plain)


def bench_batched(args):
    """Many planted-partition graphs (n log-uniform in [100, 20000], mean
    degree U[8, 64], 5-200 blocks, per-graph eps in {1/5..4/5}, mu in 2..10):
    one persistent batched launch (autotuned, captured in a HIP graph) vs the
    plain path, one scan_run per graph.  Every graph's result is compared with
    the stored oracle digests (10,000 graphs, seed 4) or, for other counts,
    with the oracle on a sample."""
    import graphgen as gg
    import oracle
    import paper_2311_12281_amd as S
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from digest import result_digest

    t = time.perf_counter()
    graphs, specs = gg.planted_batch(args.batch_count, seed=4)
    eps = [s.eps for s in specs]
    mus = [s.mu for s in specs]
    m = sum(g.m for g in graphs)
    log(f"{len(graphs)} graphs, {sum(g.n for g in graphs)} vertices, {m} edges, generated in "
        f"{time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    B = S.Batch(graphs, eps, mus, autotune=not args.batch_trace)
    create_s = time.perf_counter() - t
    lanes, tile = B.config()
    log(f"batch created and autotuned in {create_s:.1f}s: lanes {lanes}, {tile} edges per tile")
    for _ in range(args.warmup):
        B.run(replay=True)
    dev_ms = []
    t = time.perf_counter()
    for _ in range(args.steps):
        labels, roles = B.run(replay=True)
        dev_ms.append(B.stats()["ms_total"])
    wall_s = (time.perf_counter() - t) / args.steps
    batch_ms = float(np.median(dev_ms))
    log(f"batched: {batch_ms:.1f} ms device per run ({m / batch_ms / 1e6:.2f} G edges/s), "
        f"{wall_s * 1e3:.1f} ms wall with host outputs")
    if args.batch_trace:
        B.close()
        _line("edges/s (|E|/solve), batched, trace run", m / (batch_ms * 1e-3), "edges/s",
              {"workload": f"planted_batch_{len(graphs)}", "graphs": len(graphs), "m": m},
              replays=args.warmup + args.steps, ms_per_batch_device=batch_ms, lanes=lanes, tile_edges=tile)
        return
    ls, rs = B.split(labels), B.split(roles)
    gold_path = os.path.join(ROOT, "tests", "golden", "planted_batch_10000_seed4.json")
    if args.batch_count == 10000 and os.path.exists(gold_path):
        with open(gold_path) as fh:
            gold = json.load(fh)["result_sha256_12"]
        bad = sum(result_digest(l, r)[:12] != gd for l, r, gd in zip(ls, rs, gold))
        exact = {"checked": "every graph against the oracle digests", "graphs_differing": bad}
    else:
        rng = np.random.default_rng(0)
        sample = rng.choice(len(graphs), size=min(200, len(graphs)), replace=False)
        bad = 0
        for k in sample:
            ol, orr = oracle.scan(graphs[k], *eps[k], mus[k])
            bad += not (np.array_equal(ol, ls[k]) and np.array_equal(orr, rs[k]))
        exact = {"checked": f"{len(sample)} sampled graphs against the oracle", "graphs_differing": bad}
    log(f"exactness: {exact}")
    # plain: one graph at a time (created, one timed scan_run, destroyed), the same results
    plain_s = 0.0
    same = True
    for k, g in enumerate(graphs):
        with S.Graph.from_csr(g) as G:
            t = time.perf_counter()
            gl, gr = G.run(*eps[k], mus[k])
            plain_s += time.perf_counter() - t
        same = same and bool(np.array_equal(gl, ls[k]) and np.array_equal(gr, rs[k]))
    log(f"plain: {plain_s * 1e3:.0f} ms for {len(graphs)} scan_run calls ({m / plain_s / 1e9:.3f} G edges/s); "
        f"identical to batched: {same}")
    B.close()
    _line("edges/s (|E|/solve) exact-match, batched", m / (batch_ms * 1e-3), "edges/s",
          {"workload": f"planted_batch_{len(graphs)}", "graphs": len(graphs), "m": m},
          ms_per_batch_device=batch_ms, ms_per_batch_wall=wall_s * 1e3, plain_edges_per_s=m / plain_s,
          plain_ms=plain_s * 1e3, identical_to_plain=same, exactness=exact, autotuned_lanes=lanes,
          tile_edges=tile, create_s=create_s)


def bench_planted(args):
    """Planted partition n = 10,000 (50 blocks, p_in 0.15, p_out 0.0005, seed 1) at eps = 1/2,
    1/5, 1/10 and mu = 5: device time per solve (median of --steps after --warmup) and the oracle
    on one host thread and on all of them (closed counts of every edge plus clustering), each
    result compared with the oracle's."""
    import graphgen as gg
    import oracle
    import paper_2311_12281_amd as S

    g = gg.planted(10000, 50, 0.15, 0.0005, 1)
    n, m = g.n, g.m
    threads = oracle.max_threads()
    points = []
    exact = True
    with S.Graph.from_csr(g, timing=True) as G:
        dl, dr = S.scan_device_alloc(4 * n), S.scan_device_alloc(n)
        for p, q in ((1, 2), (1, 5), (1, 10)):
            for _ in range(args.warmup):
                G.run_device(p, q, MU, dl, dr)
            wall, dev = [], []
            for _ in range(args.steps):
                t = time.perf_counter()
                G.run_device(p, q, MU, dl, dr)
                wall.append(time.perf_counter() - t)
                dev.append(G.stats()["ms_total"])
            gl = np.empty(n, np.int32)
            gr = np.empty(n, np.uint8)
            S.scan_memcpy_d2h(gl, dl, 4 * n)
            S.scan_memcpy_d2h(gr, dr, n)
            cpu = {}
            for T in (1, threads):
                ts = []
                for _ in range(3):
                    t = time.perf_counter()
                    ol, orr = oracle.scan(g, p, q, MU, threads=T)
                    ts.append(time.perf_counter() - t)
                cpu[T] = float(np.median(ts))
            ok = bool(np.array_equal(gl, ol) and np.array_equal(gr, orr))
            exact = exact and ok
            pt = {"eps": f"{p}/{q}", "mu": MU, "ms_wall": float(np.median(wall) * 1e3),
                  "ms_device": float(np.median(dev)), "edges_per_s": float(m / np.median(wall)),
                  "oracle_t1_edges_per_s": m / cpu[1], "oracle_tall_edges_per_s": m / cpu[threads],
                  "cores": int((orr == 1).sum()), "exact_match": ok}
            points.append(pt)
            log(f"planted n={n} m={m}: {pt}")
        S.scan_device_free(dl)
        S.scan_device_free(dr)
    _line("edges/s (|E|/solve) exact-match, small planted graph", float(np.median([p["edges_per_s"] for p in points])),
          "edges/s", {"workload": "planted_n10000_b50_seed1", "n": n, "m": m},
          exact_match=exact, points=points,
          cpu_baseline={"kind": "oracle", "cores": threads, "cpu_model": _cpu_model(),
                        "sample": "the same graph and eps, closed counts of every edge plus clustering, "
                                  "median of 3 runs at 1 thread and at all threads"})


def bench_sweep(args):
    """R-MAT scale 22: eps in {0.2 .. 0.8} at mu = 6, and mu in {3, 6, 11, 16,
    31} at eps = 0.5 (the axes of the paper's experiments on eps and mu), with
    the device time of every phase; every result is compared with the oracle
    (closed counts once, then the clustering of each point)."""
    import graphgen as gg
    import oracle
    import paper_2311_12281_amd as S

    g = gg.rmat(args.scale, args.edge_factor, seed=args.seed)
    n, m = g.n, g.m
    G = S.Graph.from_csr(g, timing=True)
    dl, dr = S.scan_device_alloc(4 * n), S.scan_device_alloc(n)
    oc = oracle.counts(g, threads=oracle.max_threads())
    points = [((k, 10), 6) for k in range(2, 9)] + [((1, 2), mu) for mu in (3, 6, 11, 16, 31)]
    rows = []
    for (p, q), mu in points:
        G.run_device(p, q, mu, dl, dr)  # warm-up
        walls, sts = [], []
        for _ in range(max(3, args.steps // 2)):
            t = time.perf_counter()
            G.run_device(p, q, mu, dl, dr)
            walls.append(time.perf_counter() - t)
            sts.append(G.stats())
        gl = np.empty(n, np.int32)
        gr = np.empty(n, np.uint8)
        S.scan_memcpy_d2h(gl, dl, 4 * n)
        S.scan_memcpy_d2h(gr, dr, n)
        ol, orr = oracle.cluster(g, oc, p, q, mu)
        exact = bool(np.array_equal(gl, ol) and np.array_equal(gr, orr))
        wall = float(np.median(walls))
        row = {"eps": f"{p}/{q}", "mu": mu, "ms_wall": wall * 1e3, "edges_per_s": m / wall,
               "ms_phase": {ph: float(np.median([st["ms_phase"][ph] for st in sts])) for ph in S.PHASES},
               "ms_cores_bucket": [float(np.median([st["ms_cores_bucket"][b] for st in sts])) for b in range(7)],
               "evaluated_cores": int(sts[-1]["evaluated"]["cores"]), "evaluated_merge": int(sts[-1]["evaluated"]["merge"]),
               "cores": int((orr == 1).sum()), "clusters": int(np.unique(ol[orr == 1]).size),
               "exact_match": exact}
        rows.append(row)
        log(f"eps={p}/{q} mu={mu}: {row['ms_wall']:.1f} ms, cores {row['cores']}, exact {exact}, "
            f"phases {{{', '.join(f'{k}: {v:.2f}' for k, v in row['ms_phase'].items())}}}")
    S.scan_device_free(dl)
    S.scan_device_free(dr)
    G.close()
    _line("edges/s (|E|/solve) exact-match, eps and mu sweep", float(np.median([r["edges_per_s"] for r in rows])),
          "edges/s", {"workload": f"rmat{args.scale}_ef{args.edge_factor}_sweep", "n": n, "m": m},
          exact_match=all(r["exact_match"] for r in rows), points=rows)


if __name__ == "__main__":
    main()
