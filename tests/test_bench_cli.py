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
                 "--no-spmv", "--spmv-only", "--no-legs", "--no-small", "--no-c2", "--cpu-pairs"):
        assert flag in r.stdout


@pytest.mark.parametrize("tile", [8, 16])
def test_headline_traffic_profile(tile):
    """The committed counter profile of the headline's FP32 apply (1e7-node
    configuration model): when taken on the current kernel source, its
    traffic lies above the algorithmic bytes (the gathers miss L2) and
    within a sane multiple of them."""
    import bench
    n, nnz = 10_000_000, 75_714_946
    alg = 4.0 * nnz + 4.0 * (n + 1) + 2.0 * tile * 4.0 * n
    t = bench.load_traffic(tile)
    if t is None:
        pytest.skip(f"no profile for T={tile} on the current kernel source")
    assert alg < t < 20 * alg


def test_reference_spmv_traffic_profile():
    import bench
    t = bench.load_spmv_traffic()
    if t is None:
        pytest.skip("profile predates the current kernel source")
    assert 4e8 < t < 2e10


def test_sliced_apply_traffic_profile():
    """The committed counters of the column-sliced one-column apply belong to
    the current source and lie between the algorithmic bytes and the
    row-wise apply's traffic."""
    import bench
    t = bench.load_slice_traffic()
    assert t is not None, "profile predates the current slice.hip"
    n, nnz = 10_000_000, 75_714_946
    alg = 4.0 * nnz + 4.0 * (n + 1) + 2.0 * 4.0 * n
    row = bench.load_spmv_traffic()
    assert alg < t < (row if row is not None else 20 * alg)
