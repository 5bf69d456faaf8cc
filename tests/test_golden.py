"""Oracle against the fixtures in tests/golden (written by tests/golden/make_golden.py)."""
import os

import numpy as np

import oracle
from paper_1612_02750_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_free_spectrum_fixture():
    """Closed-form free spectrum of A on 4^4, m = 0.1 (values and multiplicities)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "free_spectrum_A_4444_m0.1.txt"))
    expect = np.repeat(tab[:, 0], tab[:, 1].astype(int))
    dims = (4, 4, 4, 4)
    ev = np.linalg.eigvalsh(oracle.dense_A(dims, synth.unit_gauge(dims), 0.1))
    np.testing.assert_allclose(np.sort(ev), expect, rtol=0, atol=1e-11)


def test_oracle_dslash_snapshot():
    tab = np.loadtxt(os.path.join(GOLDEN, "oracle_dslash_2222_haar0.txt"))
    dims = (2, 2, 2, 2)
    out = oracle.dslash_full(dims, synth.haar_gauge(dims, 0), synth.gauss_source(1, 16, 1)[0])
    ref = (tab[:, 2] + 1j * tab[:, 3]).reshape(16, 3)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-15)
