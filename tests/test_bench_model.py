"""The op models behind the roofline fractions in bench.py (CPU)."""
import subprocess
import sys

import bench


def test_op_model_paper_shaped():
    # per step and component: 2l forward NTTs (11 per butterfly), 2 inverse (10), 2Nl pairs (10)
    N, l = 1024, 4
    bfly = (N // 2) * 10
    per_comp = 2 * l * bfly * 11 + 2 * bfly * 10 + 2 * N * l * 10
    assert per_comp == 8 * 5120 * 11 + 2 * 5120 * 10 + 2 * 1024 * 4 * 10 == 634_880
    assert bench.ops_per_bootstrap(630, N, l, 4) == 630 * 4 * per_comp
    assert bench.ops_per_bootstrap(630, N, l, 4) * 4096 == 6_553_180_569_600  # ops_per_launch in the bench line


def test_op_model_wide_two_primes_and_two_keys():
    n, N, l = 512, 2048, 4
    bfly = (N // 2) * 11
    per_prime_1 = 2 * l * bfly * 11 + 2 * N * l * 10 + 2 * bfly * 10
    per_prime_2 = 2 * (2 * l * bfly * 11 + 2 * N * l * 10) + 2 * bfly * 10  # one inverse NTT pair
    assert bench.ops_per_bootstrap_wide(n, N, l, 1, 1) // n == 2 * per_prime_1 == 2_760_704
    assert bench.ops_per_bootstrap_wide(n, N, l, 1, 2) // n == 2 * per_prime_2 == 5_070_848
    assert bench.ops_per_bootstrap_wide(n, N, l, 128, 1) == 2 * bench.ops_per_bootstrap(n, N, l, 128)


def test_peaks():
    assert round(bench.PEAK_LANE_OPS / 1e12, 1) == 78.6
    assert round(bench.SINGLE_ISSUE_LANE_OPS / 1e12, 1) == 39.3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stdout
