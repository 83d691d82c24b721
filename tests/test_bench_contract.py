"""Host-side checks of bench.py's measurement code: the one-GPU refusal,
the traffic figure taken only from a summary of the current sources, and
the exact in-support pair count behind the compact-support metric."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_from_current_sources():
    """The committed summaries carry the sources' digest; the figure is used
    only while the sources still hash to it."""
    import re
    for summary, sources in (("fit_f64_c2_1024_traffic.md", bench.F64_SOURCES),
                             ("fit_lp_c5_traffic.md", bench.LP_SOURCES)):
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        recorded = re.search(r"source_sha256: `([0-9a-f]+)`", text).group(1)
        t = bench.profiled_traffic(summary, sources)
        if recorded == bench.source_digest(sources):
            assert isinstance(t, int) and t > 0
        else:
            assert t is None
        assert bench.profiled_traffic(summary, sources + ["bench.py"]) is None
    assert bench.profiled_traffic("no_such_summary.md", bench.F64_SOURCES) is None


def test_support_pairs_matches_brute_force():
    rng = np.random.default_rng(3)
    pts = rng.random((400, 2))
    grid = {"x0": 0.5 / 37, "y0": 0.5 / 29, "dx": 1 / 37, "dy": 1 / 29, "width": 37,
            "height": 29}
    h = 0.09
    gx = grid["x0"] + grid["dx"] * np.arange(37)
    gy = grid["y0"] + grid["dy"] * np.arange(29)
    d2 = ((gx[None, None, :] - pts[:, 0, None, None]) ** 2 +
          (gy[None, :, None] - pts[:, 1, None, None]) ** 2)
    assert bench.support_pairs(pts, grid, h) == int(np.sum(d2 < h * h))
    rows = np.arange(0, 29, 4)
    assert bench.support_pairs(pts, grid, h, rows=rows) == int(np.sum(d2[:, rows, :] < h * h))


def test_traffic_summary_is_keyed_by_workload():
    """Only the workload a summary was taken on reports its traffic: the
    timing-table workloads have none."""
    from paper_1408_0677_amd import workloads as wl
    assert bench.TRAFFIC_SUMMARIES.get(wl.c2().name) == "fit_f64_c2_1024_traffic.md"
    for n in (306, 1000, 2245):
        assert wl.t1(n).name not in bench.TRAFFIC_SUMMARIES


def test_layout_pair_count_counts_fused_multiply_adds_once():
    assert bench.LAYOUT_OPS_PER_PAIR == 10
