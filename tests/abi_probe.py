"""Library checks run in a child interpreter by test_abi.py.

On a host without a GPU, loading the HIP runtime and then forking (pytest's
other tests build with gcc, call nm, ...) is not safe, so the parent test
process never loads the library; this script does, and exits non-zero on
the first failed check."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import paper_2311_12281_amd as S  # noqa: E402


def check_symbols(names):
    lib = S.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(S.EXPORTED) == sorted(names), (sorted(S.EXPORTED), sorted(names))
    assert "gfx950" in S.scan_version()
    o = S.scan_opts_default()
    assert o.validate == 1 and o.pruning == 1 and o.timing == 0 and o.device_budget_bytes == 0
    assert o.hub_ranked == 1 and o.hub_outlier == 0 and o.strategy == 0 and not o.hip_stream


def check_threshold():
    sim = oracle.similar
    for p in range(1, 8):
        for q in range(p, 9):
            for a in range(1, 30):
                for b in range(a, 30, 3):
                    t = S.scan_eps_threshold(p, q, a, b)
                    assert t >= 0
                    assert sim(t, a, b, p, q)
                    assert t == 0 or not sim(t - 1, a, b, p, q)
    rng = np.random.default_rng(1)
    for _ in range(20000):
        q = int(rng.integers(1, 5000))
        p = int(rng.integers(1, q + 1))
        amax = (1 << 32) // q - 1
        a = int(rng.integers(1, max(2, min(amax, 2_000_000))))
        b = int(rng.integers(1, max(2, min(amax, 2_000_000))))
        t = S.scan_eps_threshold(p, q, a, b)
        assert sim(t, a, b, p, q), (p, q, a, b, t)
        assert t == 0 or not sim(t - 1, a, b, p, q), (p, q, a, b, t)
    for k in range(1, 2000):  # eps = 1/2 with a b = 4 k^2: threshold exactly k
        assert S.scan_eps_threshold(1, 2, 2 * k, 2 * k) == k
    assert S.scan_eps_threshold(0, 2, 3, 3) == -1
    assert S.scan_eps_threshold(3, 2, 3, 3) == -1
    assert S.scan_eps_threshold(1, 2, 0, 3) == -1
    assert S.scan_eps_threshold(1, 1 << 20, 1 << 12, 1) == -1


def check_no_device():
    import graphgen as gg
    g = gg.planted(50, 2, 0.3, 0.05, 1)
    try:
        h = S.scan_graph_create(g.n, g.nnz, g.row_ptr, g.col_idx)
    except S.ScanError as e:
        assert e.code == S.SCAN_E_DEVICE, e
        return 0
    S.scan_graph_destroy(h)
    return 4  # a GPU is present


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "symbols":
        check_symbols(sys.argv[2:])
    elif what == "threshold":
        check_threshold()
    elif what == "nodevice":
        sys.exit(check_no_device())
    print("ok")
