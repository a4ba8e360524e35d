"""Host checks of bench.py's bookkeeping (no GPU): the algorithmic bytes it
charges each kernel of the CKKS-shaped step, the traffic table's source hash,
and the --gpus rule."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N, L, W = 1 << 16, 36, 8
WORDS = 4 * L * N  # one launch over the four polynomials
TABLE = L * N * 8


@pytest.mark.parametrize("name,want", [
    ("col_fwd_f64l_log4_2pass", 2 * WORDS * W),
    ("col_inv_f64l_log4_2pass", 2 * WORDS * W),
    ("row_fwd_f64l_log12_2pass", 2 * WORDS * W + TABLE),
    ("row8_inv_f64l_log12_2pass", 2 * WORDS * W + TABLE),
    ("row4_fwd_i64_log10_2pass", 2 * WORDS * W + 2 * TABLE),
    ("pointwise_fwd_f64l_log16", 3 * WORDS * W),
    ("polymul_row_fwd_f64l_log12_2pass", 3 * WORDS * W + 2 * TABLE),
    ("fwdmul_row_fwd_f64l_log12_2pass", 5 * WORDS * W + TABLE),
])
def test_algorithmic_bytes_of_every_step_kernel(name, want):
    """Every kernel the step launches is charged its minimum traffic (coefficients
    read and written once, plus the tables a row pass reads); none falls to zero."""
    assert bench.algorithmic_bytes(name, WORDS, N, L, W) == want


def test_dominant_kernel_traffic_matches_its_algorithmic_bytes():
    """When the committed counter table was taken on the current kernel sources,
    it holds the dominant column pass at its algorithmic 151 MB (within 1 %)."""
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    if t["source_hash"] != bench.kernel_source_hash():
        pytest.skip("counter table taken on other kernel sources (bench reports traffic null)")
    col = t["kernels"]["col_fwd_f64l_log4_2pass"]["hbm_bytes_per_launch"]
    assert abs(col - 2 * WORDS * W) / (2 * WORDS * W) < 0.01


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
