"""Host-side logic of the benchmark script, on the CPU: the one-GPU guard, the
kernel-time table of a rocprofv3 --kernel-trace --stats run, the counter
summary (FETCH_SIZE and WRITE_SIZE scaled by what they read for the plain copy
kernel, per-bucket traffic, LDS ratios), the rule that the committed traffic
figure is used only while the kernel sources are the ones it was measured on,
and the byte models of a solve on a graph small enough to count by hand.  The
CSV fixtures use rocprofv3's column names and kernel-name
strings, with made-up values chosen so that every expected figure is exact."""
import argparse
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HUB0 = "void scan::(anonymous namespace)::k_hub<0>(scan::EdgeArgs, scan::HubJob const*, long, unsigned long long*, int*)"
HUB1 = "void scan::(anonymous namespace)::k_hub<1>(scan::EdgeArgs, scan::HubJob const*, long, unsigned long long*, int*)"
GROUP4 = "void scan::(anonymous namespace)::k_group<0, 4, false>(scan::EdgeArgs)"
STAGED = "void scan::(anonymous namespace)::k_group<0, 64, true>(scan::EdgeArgs)"
COPY = ("scan::(anonymous namespace)::k_copy16(HIP_vector_type<unsigned int, 4u> const*, "
        "HIP_vector_type<unsigned int, 4u>*, long)")


def _counter_csv(path, rows):
    """rows: (dispatch id, kernel name, counter, value) in rocprofv3's counter_collection.csv layout."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write('"Correlation_Id","Dispatch_Id","Agent_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for did, name, c, v in rows:
            fh.write(f'{did},{did},"Agent 1","{name}","{c}",{v:.6f}\n')


def test_more_than_one_gpu_is_refused():
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                           env={**os.environ, **env}, timeout=120)
        assert r.returncode == 2, r.stderr
        assert "exactly one GPU" in r.stderr
        assert r.stdout == ""


def test_short_kernel_names():
    assert bench._short_kernel(HUB0) == "k_hub<0>"
    assert bench._short_kernel(GROUP4) == "k_group<0, 4>"
    assert bench._short_kernel(STAGED) == "k_group<0, 64, staged>"
    assert bench._short_kernel(COPY) == "k_copy16"


def test_kernel_time_table(tmp_path, capsys):
    # two result files (two processes of one run): calls and times add up per kernel
    hdr = '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
    for sub, rows in (("a", [(HUB0, 3, 30_000_000), (GROUP4, 3, 3_000_000), (COPY, 1, 50_000)]),
                      ("b", [(HUB0, 1, 10_000_000), (STAGED, 2, 6_950_000)])):
        os.makedirs(tmp_path / sub)
        with open(tmp_path / sub / "run_kernel_stats.csv", "w") as fh:
            fh.write(hdr)
            for name, calls, ns in rows:
                fh.write(f'"{name}",{calls},{ns},{ns / calls:.6f},0,0,0,0\n')
    bench.summarize_stats(str(tmp_path))
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("| `")]
    # 50 us of 50 ms is 0.1 %: kept; sorted by total time
    assert lines == [
        "| `k_hub<0>` | 4 | 40.00 | 10.000 | 80.00 |",
        "| `k_group<0, 64, staged>` | 2 | 6.95 | 3.475 | 13.90 |",
        "| `k_group<0, 4>` | 3 | 3.00 | 1.000 | 6.00 |",
        "| `k_copy16` | 1 | 0.05 | 0.050 | 0.10 |",
    ]


def test_kernel_time_table_needs_a_stats_file(tmp_path):
    with pytest.raises(SystemExit):
        bench.summarize_stats(str(tmp_path))


def _pmc_dirs(tmp_path):
    """A FETCH_SIZE run, a WRITE_SIZE run and an LDS-counter run of the same program (the same
    dispatch ids in each).  The copy moves 1 GiB: FETCH_SIZE reads 2 GiB for it (scale 0.5),
    WRITE_SIZE 1 GiB (scale 1)."""
    kib = 1 << 20  # KiB in 1 GiB
    fetch = [(1, COPY, "FETCH_SIZE", 2 * kib), (2, GROUP4, "FETCH_SIZE", 2_000_000),
             (3, STAGED, "FETCH_SIZE", 4_000_000), (4, STAGED, "FETCH_SIZE", 6_000_000),
             (5, HUB0, "FETCH_SIZE", 40_000_000), (6, HUB1, "FETCH_SIZE", 9_999_999),
             (7, HUB0, "FETCH_SIZE", 60_000_000)]
    write = [(1, COPY, "WRITE_SIZE", kib), (2, GROUP4, "WRITE_SIZE", 100_000),
             (3, STAGED, "WRITE_SIZE", 200_000), (4, STAGED, "WRITE_SIZE", 300_000),
             (5, HUB0, "WRITE_SIZE", 1_000_000), (6, HUB1, "WRITE_SIZE", 7_777_777),
             (7, HUB0, "WRITE_SIZE", 3_000_000)]
    # SQ counters arrive as one row per shader engine: per-dispatch values are their sums
    lds = [(5, HUB0, "SQ_LDS_IDX_ACTIVE", 600), (5, HUB0, "SQ_LDS_IDX_ACTIVE", 400),
           (5, HUB0, "SQ_LDS_BANK_CONFLICT", 200), (5, HUB0, "SQ_INSTS_LDS", 10),
           (5, HUB0, "SQ_INSTS_VALU", 103), (6, HUB1, "SQ_INSTS_VALU", 5)]
    dirs = []
    for name, rows in (("pmc_fetch", fetch), ("pmc_write", write), ("pmc_lds", lds)):
        _counter_csv(str(tmp_path / name / "host" / "bench_counter_collection.csv"), rows)
        dirs.append(str(tmp_path / name))
    return dirs


def test_counter_summary(tmp_path, capsys):
    args = argparse.Namespace(summarize_pmc=_pmc_dirs(tmp_path), pmc_kernel="k_hub<0>", copy_mib=1024)
    bench.summarize_pmc(args)
    out = capsys.readouterr().out
    kv = {}
    for ln in out.splitlines():
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            kv[k] = v
    # k_hub<0>: FETCH_SIZE mean 50e6 KiB x 0.5, WRITE_SIZE mean 2e6 KiB x 1 (k_hub<1> not counted)
    assert kv["traffic_bytes_per_launch"] == str(25_000_000 * 1024 + 2_000_000 * 1024)
    assert kv["kernel"] == "`k_hub<0>`"
    assert kv["kernel_sources_sha256"] == f"`{bench._kernel_source_hash()}`"
    assert "FETCH_SIZE scale 0.5000, WRITE_SIZE scale 1.0000" in out
    assert "| k_hub<0> | 2/2 | 50000000 | 2000000 |" in out
    # the LDS counters: conflict cycles per conflict-free cycle 200 / (1000 - 200), VALU per LDS 103 / 10
    assert "- LDS bank-conflict cycles per conflict-free LDS cycle: 0.250" in out
    assert "- VALU instructions per LDS instruction: 10.30" in out
    assert "| SQ_LDS_IDX_ACTIVE | 1000 (1 dispatches) |" in out
    # per bucket: buckets 4 and 5 share the staged kernel and alternate in launch order
    rows = [ln for ln in out.splitlines() if ln[:4] in {f"| {b} " for b in range(7)}]
    assert rows == [
        "| 0 | `k_group<0, 4>` | 1 | 1.024 | 0.102 |",
        "| 1 | `k_group<0, 8>` | 0 | - | - |",
        "| 2 | `k_group<0, 16>` | 0 | - | - |",
        "| 3 | `k_group<0, 32>` | 0 | - | - |",
        "| 4 | `k_group<0, 64, staged>` | 1 | 2.048 | 0.205 |",
        "| 5 | `k_group<0, 64, staged>` | 1 | 3.072 | 0.307 |",
        "| 6 | `k_hub<0>` | 2 | 25.600 | 2.048 |",
    ]


def test_counter_summary_needs_both_runs(tmp_path):
    dirs = _pmc_dirs(tmp_path)
    args = argparse.Namespace(summarize_pmc=[dirs[0]], pmc_kernel="k_hub<0>", copy_mib=1024)
    with pytest.raises(SystemExit):
        bench.summarize_pmc(args)


def test_traffic_figure_follows_the_sources(tmp_path, monkeypatch, capsys):
    args = argparse.Namespace(summarize_pmc=_pmc_dirs(tmp_path), pmc_kernel="k_hub<0>", copy_mib=1024)
    bench.summarize_pmc(args)
    prof = tmp_path / "hbm_traffic.md"
    prof.write_text(capsys.readouterr().out)
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    # the summary as printed is what the bench reads back
    assert bench._traffic_from_profile("k_hub<0>") == 27_000_000 * 1024
    # another kernel, or sources changed since the counters were taken: no figure
    assert bench._traffic_from_profile("k_hub<1>") is None
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "0000000000000000")
    assert bench._traffic_from_profile("k_hub<0>") is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench._traffic_from_profile("k_hub<0>") is None


def test_solve_byte_models():
    import graphgen as gg
    # a triangle 0-1-2 with a pendant 3 on vertex 2: degrees 2, 2, 3, 1
    g = gg.from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)])
    fixed = 4 * 8 + 8 * 5 + 17 * 4  # rows, offsets, per-vertex state
    stats = [{"cores_bucket_probes": [1, 2, 0, 0, 0, 0, 3], "cores_bucket_evaluated": [1, 0, 0, 0, 0, 0, 1]},
             {"cores_bucket_probes": [0] * 7, "cores_bucket_evaluated": [0] * 7}]
    bm = bench.solve_byte_models(g, stats, traffic=300.0, alg_per_launch=150.0)
    assert bm["per_eps_probe_model_bytes"] == [4 * 6 + 9 * 2 + fixed, fixed]
    # smaller sides 2, 2, 2, 1 over the four edges; squares of the degrees 4 + 4 + 9 + 1
    assert bm["full_evaluation_min_model_bytes"] == 4 * 7 + 9 * 4 + fixed
    assert bm["full_evaluation_merge_model_bytes"] == 4 * 18
    assert bm["dominant_kernel_traffic_over_alg"] == 2.0
    assert bench.solve_byte_models(g, [], traffic=None, alg_per_launch=150.0)["dominant_kernel_traffic_over_alg"] is None
