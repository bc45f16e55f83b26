"""The benchmark's host-side rules, on the CPU.

* ``bench.py --gpus N`` with N other than 1 exits with status 2 and says why,
  before touching a GPU.
* Figures taken from the committed counter summary (HBM traffic, VALU
  instructions per voxel-transform) are used only when the summary was taken
  on the current sweep sources: a different source hash gives None, the
  summary's own hash gives its figure.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_bench_refuses_more_than_one_gpu(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_figures_follow_the_source_hash():
    sys.path.insert(0, ROOT)
    import bench
    kv = bench.kernel_version()
    assert len(kv) == 16
    assert bench.read_profile("0" * 16, "hbm_bytes_per_launch") is None
    assert bench.read_profile(kv, "no_such_field") is None
    fields = dict(line.split("=", 1) for line in open(bench.PROFILE_TRAFFIC).read().splitlines()
                  if "=" in line and not line.startswith("#"))
    committed = fields["kernel_version"].strip()
    traffic = bench.read_profile(committed, "hbm_bytes_per_launch")
    assert traffic is not None and traffic > 0
    assert (bench.read_profile(kv, "hbm_bytes_per_launch") is not None) == (kv == committed)
