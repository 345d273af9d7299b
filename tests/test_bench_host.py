"""Host-side logic of bench.py (no GPU): the one-GPU guard, the work model
of the roofline, the bit packing of reference codewords and the workload
table."""
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
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_work_model_per_frame_iteration():
    # 8 B E + 2 B M + 2 B N + 2 (N - K) ceil(N / 64), nine branches
    assert bench.alg_ops_per_iteration(63, 45, 33, 528, 9) == 8 * 9 * 528 + 2 * 9 * 33 + 2 * 9 * 63 + 2 * 18
    assert bench.alg_ops_per_iteration(63, 36, 122, 1867, 9) == 137808
    assert bench.alg_ops_per_iteration(127, 64, 72, 1598, 9) == 8 * 9 * 1598 + 2 * 9 * 72 + 2 * 9 * 127 + 2 * 63 * 2


def test_pack_matches_bit_order():
    rng = np.random.default_rng(4)
    for n in (63, 127):
        bits = rng.integers(0, 2, size=(50, n)).astype(np.uint8)
        w = bench.pack(bits)
        for f in range(50):
            for i in range(n):
                assert ((int(w[f, i // 64]) >> (i % 64)) & 1) == bits[f, i]


def test_workload_table():
    codes, grid, frames, precisions, _ = bench.WORKLOADS["sweep63"][:5]
    assert codes == [("bch63_45", 33), ("bch63_36", 122)] and frames == 1_000_000 and precisions == ["fp32"]
    lo, hi, st = (float(x) for x in grid.split(":"))
    assert round((hi - lo) / st) + 1 == 11
    codes, grid, frames, precisions, _ = bench.WORKLOADS["fix127"][:5]
    assert frames == 4_000_000 and precisions == ["fp32", "fix8"]
    assert abs(sum(bench.WORKLOADS["mixed"][5]) - 1.0) < 1e-12
    assert bench.VALU_PEAK_OPS == 256 * 128 * 2.4e9 and bench.HBM_PEAK_BYTES == 8.0e12
