"""The committed rocprofv3 summaries under profiles/ describe the committed
map kernel: their kernel-source hash is that of csrc/map_kernel.hip, and the
benchmark can read its traffic and VALU-issue figures from them (no GPU)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_profiles_match_the_kernel_source():
    h = bench.kernel_source_hash()
    pdir = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(pdir) if f.startswith("k_map_") and f.endswith(".txt"))
    assert names, "no profile summaries"
    for f in names:
        lines = [l for l in open(os.path.join(pdir, f)) if l.startswith("kernel_source_sha256_16:")]
        assert lines and lines[0].split(":", 1)[1].strip() == h, f"{f} was taken on another kernel source"
        assert any(l.startswith("# command") for l in open(os.path.join(pdir, f))), f"{f} names no command"


def test_bench_reads_traffic_and_valu_issue():
    for w, n, ms in (("large", 1_000_000, 28.6), ("pet", 100544, 1.6)):
        t = bench.measured_traffic(w)
        assert t is not None and t > 0
        v = bench.measured_valu(w, n, ms)
        assert v is not None and 0.0 < v["issue_utilisation"] < 1.5
        assert v["valu_insts_per_voxel"] > 1000
