"""Plain FP64 oracle of staggered meson correlators from point-source propagators.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP path; the product
library never imports it.  Shares no code with the HIP path.

What it follows.  The paper (Sec. 4) lists spectrum (hadron correlator)
measurements among the framework's uses and prints no formula; the
definitions are the textbook staggered ones:

  propagator  G(x; x_s) = M^-1 delta_{x_s} per source colour, M = m + D;
              for a source on an even site, with A = m^2 - D_eo D_oe,
              G_even = m A^-1 b_e and G_odd = -D_oe A^-1 b_e
              (from M^-1 = (m - D)(m^2 - D^2)^-1, D^2 block-diagonal)
  correlator  C_s(t) = sum_{x: x_3 = (t_s + t) mod L_3} s(x) sum_{a, c} |G_ac(x; x_s)|^2,
              s(x) = (-1)^(sum of x_mu over the directions in the mask);
              mask 0 is the Goldstone pion, whose staggered phases cancel in |G|^2.

Parity status: pinned in tests/test_oracle_meson.py (a dense solve of the
full M, gauge invariance, time reflection of the free correlator).
"""
from __future__ import annotations

import numpy as np

import oracle


def _coords(dims):
    V = int(np.prod(dims))
    lex = np.arange(V)
    x0 = lex % dims[0]
    x1 = (lex // dims[0]) % dims[1]
    x2 = (lex // (dims[0] * dims[1])) % dims[2]
    x3 = lex // (dims[0] * dims[1] * dims[2])
    return np.stack([x0, x1, x2, x3], axis=1)


def point_propagator(dims, U, mass, src, tol=1e-13, flags=0):
    """Full-lattice G (V, 3 sink colours, 3 source colours) for a source at even site src."""
    x = np.asarray(src)
    assert x.sum() % 2 == 0, "the source must be on an even site"
    V = int(np.prod(dims))
    hv = V // 2
    lex_s = int(x[0] + dims[0] * (x[1] + dims[1] * (x[2] + dims[2] * x[3])))
    G = np.zeros((V, 3, 3), dtype=np.complex128)
    c = _coords(dims)
    even = c.sum(axis=1) % 2 == 0
    for col in range(3):
        b = np.zeros((hv, 3), dtype=np.complex128)
        b[lex_s >> 1, col] = 1.0
        xe, st, _, _ = oracle.cg(dims, U, mass, b, tol=tol, flags=flags)
        assert st == oracle.OK
        yo = oracle.dslash_eo(dims, U, xe, 1, flags)
        lex = np.arange(V)
        G[even, :, col] = mass * xe[lex[even] >> 1]
        G[~even, :, col] = -yo[lex[~even] >> 1]
    return G


def correlators(dims, G, src, masks):
    """C[k, t] for each mask (a 4-bit set of directions), t relative to the source time."""
    c = _coords(dims)
    dens = np.sum(np.abs(G) ** 2, axis=(1, 2))
    L3 = dims[3]
    out = np.zeros((len(masks), L3))
    t = (c[:, 3] - src[3]) % L3
    for k, m in enumerate(masks):
        e = sum(c[:, mu] for mu in range(4) if (m >> mu) & 1) if m else np.zeros(len(c), int)
        s = np.where(e % 2 == 0, 1.0, -1.0)
        out[k] = np.bincount(t, weights=s * dens, minlength=L3)
    return out
