"""Host-side logic of bench.py (no GPU): the crossing finder of the moment
ratio scans, the refusal of more than one GPU and the algorithmic byte counts
behind the roofline figure."""
import subprocess
import sys
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_crossing_by_linear_interpolation():
    # larger size below the smaller one at T = 1, above it at T = 2: they cross
    # where the difference -0.1 -> +0.1 passes zero, T = 1.5
    out = bench.crossings([1.0, 2.0, 3.0], {32: [1.0, 1.5, 2.0], 64: [0.9, 1.6, 2.3]})
    assert len(out) == 1 and out[0]["L_pair"] == [32, 64] and abs(out[0]["T"] - 1.5) < 1e-12


def test_crossings_of_three_sizes_and_none():
    temps = [0.0, 1.0, 2.0, 3.0]
    curves = {8: [1.0, 1.0, 1.0, 1.0], 16: [0.5, 0.5, 1.5, 1.5], 32: [0.0, 0.0, 0.25, 2.0]}
    out = bench.crossings(temps, curves)
    assert [c["L_pair"] for c in out] == [[8, 16], [16, 32]]
    assert abs(out[0]["T"] - 1.5) < 1e-12          # -0.5 -> +0.5 between T = 1 and 2
    assert abs(out[1]["T"] - (2.0 + 1.25 / 1.75)) < 1e-12  # -1.25 -> +0.5 between T = 2 and 3
    assert bench.crossings(temps, {8: [1, 1, 1, 1], 16: [2, 2, 2, 2]}) == []


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_fused_kernel_bytes_per_site():
    # the fused kernel does the work of the flip (labels read, spins written;
    # the clock model also reads the old spins) and of the bond kernel (spins
    # and the halo read, bond bits and labels written): 5 + 5.28125 B per site
    L = 4096
    assert bench.alg_bytes_per_launch("k_code_flip_bond", L, "potts") == pytest.approx(10.28125 * L * L)
    assert bench.alg_bytes_per_launch("k_code_flip_bond", L, "clock") == pytest.approx(11.28125 * L * L)
    # the merge: per tile-border site one bond bit and two label words
    assert bench.alg_bytes_per_launch("k_node_merge", L, "potts") == pytest.approx(L * 128 * 8.125)
