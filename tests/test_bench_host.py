"""The benchmark's host-side rules, on the CPU.

* ``bench.py --gpus N`` with N other than 1 exits with status 2 and says why,
  before touching a GPU.
* Figures taken from the committed counter summary (HBM traffic, VALU
  instructions per voxel-transform) are used only when the summary was taken
  on the current sweep sources: a different source hash gives None, the
  summary's own hash gives its figure.
* The tuning-cache reader behind the line's launch shapes.
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


def test_tune_cache_lines_and_shape_lookup(tmp_path):
    """The three kinds of MI_TUNE_CACHE line, in the library's field order,
    parse into keys and shapes; malformed lines are skipped; the bench's
    lookup returns the last entry of the asked class."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1909_10690_amd import binding as B
    p = tmp_path / "tune.txt"
    p.write_text("gemi-tune 256 256 180 256 256 180 1 128 0 10 0 512 1 2048 0\n"
                 "gemi-tune 256 256 180 256 256 180 1 128 0 10 0 1024 0 0 1\n"
                 "gemi-tune 1 2 3\n"
                 "gemi-tune-parzen 512 512 300 256 256 256 1 256 1 0 1024 128 1024 96 0\n"
                 "gemi-tune-pairs 8 25 12 64 0 1 256 65536 1 1\n"
                 "something else\n")
    e = B.read_tune_cache(str(p))
    assert [x["kind"] for x in e] == ["gemi-tune", "gemi-tune", "gemi-tune-parzen", "gemi-tune-pairs"]
    assert e[0]["n_bucket"] == 10 and e[0]["chunks"] == 2048 and e[2]["bwd_lds_kib"] == 96
    assert e[3]["pairs_bucket"] == 8 and e[3]["transform_major"] == 1
    assert bench.tuned_shape(B, str(p), "gemi-tune", fnx=256, bins=128) == \
        {"block": 1024, "slab_major": 0, "chunks": 0, "packed": 1}
    assert bench.tuned_shape(B, str(p), "gemi-tune-parzen", bins=256) == \
        {"fwd_block": 1024, "fwd_lds_kib": 128, "bwd_block": 1024, "bwd_lds_kib": 96, "chunk_shift": 0}
    assert bench.tuned_shape(B, str(p), "gemi-tune-pairs", bins=32) is None
    assert B.read_tune_cache(str(tmp_path / "missing.txt")) == []


def test_bench_functions_use_only_defined_names():
    """Every name a bench.py function reads is a parameter, a local (an
    assignment, loop or comprehension target, an import inside it or an
    enclosing function), a module-level name or a builtin: the GPU legs run
    only on the GPU, so a missing import would otherwise surface there."""
    import ast
    import builtins
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    module = set(dir(builtins))
    for node in tree.body:
        if isinstance(node, (ast.Import, ast.ImportFrom)):
            module.update((a.asname or a.name).split(".")[0] for a in node.names)
        elif isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            module.add(node.name)
        elif isinstance(node, ast.Assign):
            module.update(t.id for t in node.targets if isinstance(t, ast.Name))

    def bound(fn):
        names = {a.arg for a in fn.args.args + fn.args.kwonlyargs}
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Store):
                names.add(n.id)
            elif isinstance(n, (ast.Import, ast.ImportFrom)):
                names.update((a.asname or a.name).split(".")[0] for a in n.names)
            elif isinstance(n, (ast.FunctionDef, ast.Lambda)) and n is not fn:
                names.update(a.arg for a in n.args.args)
                if isinstance(n, ast.FunctionDef):
                    names.add(n.name)
            elif isinstance(n, ast.arg):
                names.add(n.arg)
        return names

    missing = []
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        known = module | bound(fn)
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load) and n.id not in known:
                missing.append(f"{fn.name}: {n.id} (line {n.lineno})")
    assert not missing, missing
