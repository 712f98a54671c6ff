"""The BVH builder's treelet restructuring, checked on the CPU: the routine
the build kernel runs is compiled for the host by tests/helpers/treelet_check.cpp,
which compares the rebuilt cost of every treelet spanning a whole tree of
3..7 triangles with the minimum over all full binary trees on them
(enumerated one by one), and checks the tree invariants after bottom-up
sweeps over random trees of up to 3000 triangles."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_treelet_restructuring_on_host(tmp_path):
    exe = tmp_path / "treelet_check"
    subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "helpers", "treelet_check.cpp"), "-o", str(exe)],
                   check=True, cwd=str(tmp_path), capture_output=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    lines = res.stdout.strip().split("\n")
    bad = [l for l in lines if " FAIL" in l]
    assert res.returncode == 0 and not bad, "\n".join(bad or lines[-5:])
    assert sum(l.startswith("optimum ") for l in lines) == 5 * 12
    assert sum(l.startswith("sweep ") for l in lines) == 16
    assert lines[-1] == "failures 0"
