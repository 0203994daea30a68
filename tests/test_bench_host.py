"""Host-side checks of bench.py's command line: the refusals that come before
any device work (one GPU only; the time-correlated wind only where the
library runs it)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("workload", ["c3", "c4", "c5"])
def test_time_correlated_wind_is_refused_where_not_supported(workload):
    r = _run("--workload", workload, "--wind", "ar1")
    assert r.returncode == 2 and "c1, c2" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("workload", ["c3", "c4"])
def test_literal_weighting_is_refused_where_not_supported(workload):
    r = _run("--workload", workload, "--weighting", "product")
    assert r.returncode == 2 and "c1, c2, c5" in r.stderr and r.stdout == ""


def test_unknown_options_are_refused():
    assert _run("--weighting", "cubic").returncode != 0
    assert _run("--wind", "gusty").returncode != 0
