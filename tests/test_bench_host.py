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


def test_column_pass_traffic_matches_its_algorithmic_bytes():
    """When the committed counter table was taken on the current kernel sources,
    it holds the memory-bound column pass at its algorithmic 151 MB (within 1 %)."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        pytest.skip("no counter table committed")
    t = json.load(open(path))
    if t["source_hash"] != bench.kernel_source_hash():
        pytest.skip("counter table taken on other kernel sources (bench reports traffic null)")
    col = t["kernels"]["col_fwd_f64l_log4_2pass"]["hbm_bytes_per_launch"]
    assert abs(col - 2 * WORDS * W) / (2 * WORDS * W) < 0.01


@pytest.mark.parametrize("symbol,name", [
    ("void nttk::col_kernel<nttk::ArF64L, 4, false, true, false>(nttk::ColArgs)", "col_fwd_f64l_log4_2pass"),
    ("void nttk::col_kernel<nttk::ArF64L, 4, true, true, false>(nttk::ColArgs)", "col_inv_f64l_log4_2pass"),
    ("void nttk::row_kernel<nttk::ArF64L, 12, false, true, 4>(nttk::RowArgs)", "row_fwd_f64l_log12_2pass"),
    ("void nttk::row_kernel<nttk::ArF64L, 12, true, true, 3>(nttk::RowArgs)", "row8_inv_f64l_log12_2pass"),
    ("void nttk::row_kernel<nttk::ArI64, 10, false, true, 2>(nttk::RowArgs)", "row4_fwd_i64_log10_2pass"),
    ("void nttk::polymul_row_kernel<nttk::ArF64L, 12, true, 4, false>(nttk::RowArgs)",
     "polymul_row_fwd_f64l_log12_2pass"),
    ("void nttk::polymul_row_kernel<nttk::ArF64L, 12, true, 4, true>(nttk::RowArgs)",
     "fwdmul_row_fwd_f64l_log12_2pass"),
    ("void nttk::pointwise_kernel<nttk::ArF64L, 2>(nttk::EltArgs)", "pointwise_fwd_f64l_log16"),
    ("void nttk::bconv_mfma_kernel<unsigned long, 20, 2>(nttk::BconvArgs)", "moddown_mfma_fwd_u64_log16"),
    ("void at::native::vectorized_elementwise_kernel<4>(int)", None),
])
def test_counter_symbols_map_to_the_timer_names(symbol, name):
    """The counter summary keys kernels by the names the library's launch timer
    gives them, so bench can join counters with live durations."""
    assert bench.bench_name(symbol) == name


def test_valu_fraction_and_percentiles():
    # 1024 SIMDs x 2.4 GHz / 4 cycles = 614.4 G instructions per second at full issue
    assert abs(bench.valu_frac(614.4e9 * 1e-6, 1e-6) - 1.0) < 1e-9
    p = bench.percentiles([1.0, 2.0, 3.0, 4.0, 5.0])
    assert p["median_ms"] == 3.0 and p["samples"] == 5 and p["p10_ms"] < p["p90_ms"]


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
