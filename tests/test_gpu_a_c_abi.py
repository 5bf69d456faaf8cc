"""The C ABI from plain C: tests/c_abi/qx_solve (built by
__graft_entry__.build() with gcc against include/qx.h, libqx.so and the HIP
runtime; no Python or PyTorch in the process) solves a mixed-precision system
read from files, and the oracle measures the residual of its solution.  The
file name puts this test before every other GPU test, so the child process is
started while this one has not touched the GPU yet."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "qx_solve")


def test_c_caller_solves(tmp_path):
    # a child process started before this process touches the GPU
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi/qx_solve is missing: run __graft_entry__.build()")
    dims, m = (4, 4, 6, 8), 0.1
    U = synth.haar_gauge(dims, 70)
    hv = int(np.prod(dims)) // 2
    b = synth.gauss_source(1, hv, 71)[0]
    paths = [str(tmp_path / n) for n in ("U.bin", "b.bin", "x.bin")]
    np.ascontiguousarray(U).tofile(paths[0])
    np.ascontiguousarray(b).tofile(paths[1])
    r = subprocess.run([EXE, *map(str, dims), repr(m), *paths], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    status, iters, updates, relres = r.stdout.split()
    assert int(status) == 0 and int(iters) > 0 and int(updates) >= 1
    x = np.fromfile(paths[2], dtype=np.complex128).reshape(hv, 3)
    rr = oracle.true_residual(dims, U, m, b, x)
    assert rr <= 1e-10, rr
    assert abs(float(relres) - rr) <= 1e-11
