"""Host logic of bench.py (no GPU needed): the one-GPU guard and the
confidence bound that the FER comparison uses."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


@pytest.mark.parametrize("n", [10, 1000, 1 << 20])
def test_cp_upper_zero_errors_closed_form(n):
    # with no errors the upper end solves (1 - p)^n = (1 - conf) / 2
    assert math.isclose(bench.cp_upper(0, n), 1 - 0.025 ** (1 / n), rel_tol=1e-9)


def test_cp_upper_all_errors_and_monotone():
    assert bench.cp_upper(7, 7) == 1.0
    ups = [bench.cp_upper(k, 1000) for k in range(0, 50, 7)]
    assert all(a < b for a, b in zip(ups, ups[1:]))
    # the bound lies above the point estimate and tightens with more frames
    assert bench.cp_upper(10, 1000) > 10 / 1000
    assert bench.cp_upper(100, 100000) < bench.cp_upper(10, 10000)


def test_cp_upper_n_one_error_closed_form():
    # k = n - 1 errors in n: the upper end is the 0.975 quantile of Beta(n, 1),
    # whose distribution function is x^n
    n = 20
    assert math.isclose(bench.cp_upper(n - 1, n), 0.975 ** (1 / n), rel_tol=1e-9)
