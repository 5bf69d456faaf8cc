"""Writes the fixtures in this folder.  Calls only the CPU oracle and the seeded
input generators (never the HIP path).

free_spectrum_A_4444_m0.1.txt
    distinct eigenvalues of A = m^2 - D_eo D_oe for U = 1 on a periodic 4^4
    lattice at m = 0.1 with their multiplicities, from the closed form
    lambda(p) = m^2 + sum_mu sin^2 p_mu, p_mu = 2 pi n_mu / 4 (each pair of
    momenta p, p + (pi,pi,pi,pi) gives one even-site eigenvector, times three
    colours).  Pure mathematics: no code under test is involved.
oracle_dslash_2222_haar0.txt
    regression snapshot of the oracle's D on a 2^4 lattice (Haar links seed 0,
    source seed 1 on all 16 sites): one line per (site, colour) with the real
    and imaginary parts.  Guards the oracle against unintended changes.
"""
import itertools
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1612_02750_amd import synth  # noqa: E402


def free_spectrum():
    m = 0.1
    vals = {}
    for n in itertools.product(range(4), repeat=4):
        lam = m * m + sum(np.sin(2 * np.pi * k / 4) ** 2 for k in n)
        key = round(lam, 12)
        vals[key] = vals.get(key, 0) + 1
    with open(os.path.join(HERE, "free_spectrum_A_4444_m0.1.txt"), "w") as f:
        f.write("# eigenvalue multiplicity (closed form; see make_golden.py)\n")
        for k in sorted(vals):
            f.write(f"{k:.12f} {vals[k] * 3 // 2}\n")


def dslash_snapshot():
    dims = (2, 2, 2, 2)
    U = synth.haar_gauge(dims, 0)
    chi = synth.gauss_source(1, 16, 1)[0]
    out = oracle.dslash_full(dims, U, chi)
    with open(os.path.join(HERE, "oracle_dslash_2222_haar0.txt"), "w") as f:
        f.write("# lex colour re im  (oracle D on 2^4, Haar seed 0, source seed 1)\n")
        for lex in range(16):
            for a in range(3):
                f.write(f"{lex} {a} {out[lex, a].real:.17e} {out[lex, a].imag:.17e}\n")


if __name__ == "__main__":
    free_spectrum()
    dslash_snapshot()
