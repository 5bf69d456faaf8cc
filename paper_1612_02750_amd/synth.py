"""Seeded synthetic inputs: SU(3) gauge fields and Gaussian colour-vector sources.

This module only draws inputs; it holds none of the Dirac-operator, solver or
force arithmetic, and it imports nothing from the HIP path or from the CPU
checker, so both can consume the same arrays.

Layouts (the canonical layouts of the C ABI):
  gauge field  U : complex128 (4, V, 3, 3); direction mu = x, y, z, t major,
                   then lexicographic site lex = x0 + L0*(x1 + L1*(x2 + L2*x3)),
                   then row, column.
  source       b : complex128 (nrhs, V/2, 3); sites of one parity in
                   checkerboard order cb = lex >> 1.

The paper (Sec. 1 and Sec. 4) works on a 4-D grid carrying one SU(N) matrix per
link; it prints no generator, so the recipes below are the standard ones:
  * Haar SU(3): QR of a complex Gaussian matrix with the diagonal-phase fix of
    Mezzadri, Notices AMS 54 (2007) 592, then division by the principal cube
    root of the determinant so that det U = 1.
  * weak field: U = exp(i*eps*H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0,1)
    and lambda_a the Gell-Mann matrices; the exponential is taken through the
    eigen-decomposition of the Hermitian H.
  * sources: real and imaginary parts i.i.d. N(0,1).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "haar_su3",
    "weak_su3",
    "haar_gauge",
    "weak_gauge",
    "unit_gauge",
    "gauss_source",
    "random_su3_transform",
]


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def _rng(seed):
    if isinstance(seed, np.random.Generator):
        return seed
    return np.random.Generator(np.random.PCG64(seed))


def haar_su3(n: int, seed=0) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, complex128 (n, 3, 3)."""
    rng = _rng(seed)
    g = rng.standard_normal((n, 3, 3, 2))
    z = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return np.ascontiguousarray(q)


_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3.0)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3.0)


def weak_su3(n: int, eps: float, seed=0) -> np.ndarray:
    """n matrices exp(i*eps*H), H = sum_a h_a lambda_a/2, h ~ N(0,1); (n, 3, 3)."""
    rng = _rng(seed)
    h = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, _GELL_MANN / 2.0)
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    u = np.einsum("nij,nj,nkj->nik", v, ph, v.conj())
    return np.ascontiguousarray(u)


def haar_gauge(dims, seed=0) -> np.ndarray:
    V = volume(dims)
    return haar_su3(4 * V, seed).reshape(4, V, 3, 3)


def weak_gauge(dims, eps: float, seed=0) -> np.ndarray:
    V = volume(dims)
    return weak_su3(4 * V, eps, seed).reshape(4, V, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    V = volume(dims)
    u = np.zeros((4, V, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def gauss_source(nrhs: int, half_volume: int, seed=1) -> np.ndarray:
    """complex128 (nrhs, V/2, 3) with i.i.d. N(0,1) real and imaginary parts."""
    rng = _rng(seed)
    g = rng.standard_normal((nrhs, half_volume, 3, 2))
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1])


def random_su3_transform(dims, seed=7) -> np.ndarray:
    """A Haar SU(3) matrix per site, (V, 3, 3): a random gauge transformation."""
    return haar_su3(volume(dims), seed)
