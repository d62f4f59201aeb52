"""bench.py's contract on the host: one GPU only (more exits with a message
and status 2, before touching a GPU), and the counter-traffic figures read
from the committed profiles only when they were taken on the current kernel
source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_legs():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--no-batched", "--no-pairwise", "--no-density",
                 "--no-spmv", "--spmv-only"):
        assert flag in r.stdout


@pytest.mark.parametrize("tile,alg", [(32, 284e6), (64, 540e6)])
def test_headline_traffic_profile(tile, alg):
    import bench
    t = bench.load_traffic(tile)
    if t is None:
        pytest.skip(f"profile for T={tile} predates the current kernel source")
    # the gathers miss L2: counted traffic well above the algorithmic bytes
    assert alg < t < 10 * alg


def test_reference_spmv_traffic_profile():
    import bench
    t = bench.load_spmv_traffic()
    if t is None:
        pytest.skip("profile predates the current kernel source")
    assert 4e8 < t < 2e10
