"""Invariants of the batch plan (the per-cluster block shape, the cut into
smaller i-blocks for occupancy, the item target, the j-splits and the
reduction's row parts), checked on the host over 200,000 seeded random
clusters, tunings and grids: every tile in exactly one non-empty split, at
most max_split splits, blocks covering exactly the cluster's rows, the item
count within the bound the library sizes its item table by, and maximal
reduction parts that fit the grid.  The plan functions are the library's
own (g6mi_batch_common.h), compiled for the host by hipcc; the program
calls no HIP runtime function, so no GPU is needed."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "plan_check.hip")


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_batch_plan_invariants(tmp_path):
    cc = hipcc()
    if cc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "plan_check")
    r = subprocess.run([cc, "--offload-arch=gfx950", "--cuda-host-only", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"), SRC, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "violations 0" in r.stdout
