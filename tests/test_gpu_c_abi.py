"""The C ABI driven from a plain C99 program (tests/c/hjw_c_example.c: device memory from
the HIP runtime, no Python, no torch): its phi is bitwise the phi of the same FP64 solve
through the Python binding."""
import os
import subprocess

import numpy as np
import pytest

from paper_1909_13263_amd import hjw
from paper_1909_13263_amd import workloads as W

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "hjw_c_example")


@pytest.mark.parametrize("n", [64, 200])
def test_c_program_matches_the_python_path(n, tmp_path):
    import torch
    assert torch.cuda.is_available(), "this test needs the GPU"
    assert os.path.exists(EXE), "build the C example first (__graft_entry__.build())"
    pr = W.burgers2d(n, 0.02)
    phi0 = np.ascontiguousarray(pr.phi0())
    src, dst = tmp_path / "phi0.bin", tmp_path / "phi.bin"
    phi0.tofile(src)
    r = subprocess.run([EXE, str(n), str(src), str(dst)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    phi_c = np.fromfile(dst, dtype=np.float64).reshape(n, n)
    g = hjw.grid_for(pr, hjw.FP64)
    g.set_phi(phi0)
    info = g.step_to(0.02, 0.5)
    ref = g.get_phi()
    g.close()
    assert r.stdout.split()[:2] == ["steps", str(info.steps)], r.stdout
    assert np.array_equal(phi_c, ref)
