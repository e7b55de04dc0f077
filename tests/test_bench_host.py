"""Host-side logic of the benchmark, no GPU needed: the algorithmic byte model
behind `roofline.achieved`, the lookup of the stored rocprofv3 traffic, and
the one-GPU guard."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1704_07468_amd import workloads as wl  # noqa: E402


def test_accumulate_bytes_of_the_protein_workload():
    """The protein Gram (N = 3312, g = 7, k = 4: 64 position sets) has
    885958 g-mers; the accumulation step of the method reads one 12-byte
    grouped (reduced key, sequence) record per (position set, g-mer) and
    writes every entry of the four C_m once (8 bytes each):
    680415744 + 351019008 = 1031434752 bytes a Gram."""
    d = wl.protein()
    masks = [math.comb(d.g, m) for m in range(d.M + 1)]
    assert sum(masks) == 64
    alg, T = bench.algorithmic(d, masks, {"wave": 1}, 0, 3328)
    assert T == 885958
    assert alg["accumulate"] == 12 * 885958 * 64 + 8 * 4 * 3312 * 3312 == 1031434752
    tri = d.N * (d.N + 1) // 2
    # the epilogue reads the upper C_m entries and writes every N_m entry and K
    assert alg["finalize"] == 8 * (d.M + 1) * tri + 8 * (d.M + 1) * d.N * d.N + 8 * d.N * d.N


def test_sort_bytes_follow_the_kernel_split():
    d = wl.dna(N=20)
    masks = [math.comb(d.g, m) for m in range(d.M + 1)]
    stats = {"wave": 100, "wave_wide": 10, "block": 20, "block_wide": 0, "global": 0, "global_wide": 3}
    alg, _ = bench.algorithmic(d, masks, stats, 0, 128)
    assert alg["sort_wave"] == 100 * 16 + 10 * 20
    assert alg["sort_block"] == 20 * 16
    assert alg["sort_global"] == 3 * 20


def test_traffic_lookup_uses_the_copy_scale_and_the_source_hash(monkeypatch):
    t = json.load(open(bench.TRAFFIC_FILE))
    c, k = t["copy"], t["kernels"]["k_accumulate"]
    want = (k["fetch_kib"] * 1024.0 * c["bytes_read"] / (c["fetch_kib"] * 1024.0)
            + k["write_kib"] * 1024.0 * c["bytes_written"] / (c["write_kib"] * 1024.0))
    import paper_1704_07468_amd.profiling as prof
    monkeypatch.setattr(prof, "source_sha", lambda: t["source_sha"])
    assert bench.traffic_for("k_accumulate") == pytest.approx(want)
    assert bench.traffic_for("k_no_such_kernel") is None
    monkeypatch.setattr(prof, "source_sha", lambda: "0" * 64)
    assert bench.traffic_for("k_accumulate") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
