"""CPU oracle for the staggered Dslash, even-odd CG and fermion force.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the HIP path.  The arithmetic lives in ``oracle.c`` (plain C99, FP64,
OpenMP loops over lexicographic array-of-structures fields); this module loads
it through ctypes and adds small NumPy helpers (dense matrices built by applying
the oracle to unit vectors, and the su(3) projection of a link gradient).

Definitions (the paper, Sec. 4, names a staggered Dirac operator on SU(N)
links and single/double precision CG without formulas; the textbook
Kogut-Susskind forms are used, see ``oracle.c``):
  D chi(x) = 1/2 sum_mu eta_mu(x) [bc U_mu(x) chi(x+mu) - bc U_mu(x-mu)^dag chi(x-mu)]
  A        = m^2 - D_eo D_oe   (even sites)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_T_ANTIPERIODIC = 1
NAIK = 2  # improved operator: one-hop term x 9/8 plus the three-hop (Naik) term x (-1/24)
OK, NOTCONVERGED, BREAKDOWN, EINVAL = 0, 1, 2, 3

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(L):
    L.oracle_threads.argtypes = []
    L.oracle_set_threads.argtypes = [_I]
    L.oracle_set_threads.restype = None
    L.oracle_index_maps.argtypes = [_P, _P, _P]
    L.oracle_dslash_full.argtypes = [_P, _I, _P, _P, _P]
    L.oracle_dslash_eo.argtypes = [_P, _I, _P, _I, _P, _P]
    L.oracle_apply_A.argtypes = [_P, _I, _P, _D, _P, _P]
    L.oracle_cg.argtypes = [_P, _I, _P, _D, _P, _P, _I, _D, _I, _P, _P]
    L.oracle_true_residual.argtypes = [_P, _I, _P, _D, _P, _P]
    L.oracle_true_residual.restype = _D
    L.oracle_cg_mixed.argtypes = [_P, _I, _P, _D, _P, _P, _D, _D, _I, _P, _P, _P]
    L.oracle_force_from_fields.argtypes = [_P, _I, _P, _P, _P, _P]
    L.oracle_force.argtypes = [_P, _I, _P, _D, _P, _D, _I, _P, _P, _P]


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,)
    return d


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(st, what):
    if st == EINVAL:
        raise ValueError(f"oracle {what}: invalid lattice dimensions")
    return st


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def threads() -> int:
    """OpenMP threads of the oracle's parallel loops."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n threads from now on."""
    lib().oracle_set_threads(int(n))


def index_maps(dims):
    """(lex_of_eo[V], nbr_eo[V, 8]) int32; neighbour k = +mu (k < 4), -mu (k >= 4)."""
    d = _dims(dims)
    V = volume(d)
    lex = np.empty(V, dtype=np.int32)
    nbr = np.empty((V, 8), dtype=np.int32)
    _check(lib().oracle_index_maps(_ptr(d), _ptr(lex), _ptr(nbr)), "index_maps")
    return lex, nbr


def dslash_full(dims, U, chi, flags=0):
    """D chi on the full lattice: U (4,V,3,3), chi (V,3) -> (V,3)."""
    d = _dims(dims)
    U = _c128(U)
    chi = _c128(chi)
    out = np.empty_like(chi)
    _check(lib().oracle_dslash_full(_ptr(d), flags, _ptr(U), _ptr(chi), _ptr(out)), "dslash")
    return out


def dslash_eo(dims, U, chi_half, out_parity, flags=0):
    """Half-lattice D: chi (V/2,3) on parity 1-p -> (V/2,3) on parity p."""
    d = _dims(dims)
    U = _c128(U)
    chi = _c128(chi_half)
    out = np.empty_like(chi)
    _check(lib().oracle_dslash_eo(_ptr(d), flags, _ptr(U), out_parity, _ptr(chi), _ptr(out)),
           "dslash_eo")
    return out


def apply_A(dims, U, mass, v, flags=0):
    """(m^2 - D_eo D_oe) v for v (V/2,3) on even sites."""
    d = _dims(dims)
    U = _c128(U)
    v = _c128(v)
    out = np.empty_like(v)
    _check(lib().oracle_apply_A(_ptr(d), flags, _ptr(U), float(mass), _ptr(v), _ptr(out)), "A")
    return out


def cg(dims, U, mass, b, tol=1e-10, max_iter=100000, x0=None, flags=0):
    """FP64 CG; returns (x, status, iterations, true relative residual)."""
    d = _dims(dims)
    U = _c128(U)
    b = _c128(b)
    x = _c128(x0).copy() if x0 is not None else np.zeros_like(b)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0)
    st = lib().oracle_cg(_ptr(d), flags, _ptr(U), float(mass), _ptr(b), _ptr(x),
                         1 if x0 is not None else 0, float(tol), int(max_iter),
                         ctypes.byref(it), ctypes.byref(rr))
    _check(st, "cg")
    return x, st, it.value, rr.value


def true_residual(dims, U, mass, b, x, flags=0):
    d = _dims(dims)
    return lib().oracle_true_residual(_ptr(d), flags, _ptr(_c128(U)), float(mass),
                                      _ptr(_c128(b)), _ptr(_c128(x)))


def cg_mixed(dims, U, mass, b, tol=1e-10, delta=0.1, max_iter=100000, flags=0):
    """Reliable-update CG in single-precision emulation; (x, status, iters, updates, relres)."""
    d = _dims(dims)
    U = _c128(U)
    b = _c128(b)
    x = np.zeros_like(b)
    it, up, rr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
    st = lib().oracle_cg_mixed(_ptr(d), flags, _ptr(U), float(mass), _ptr(b), _ptr(x),
                               float(tol), float(delta), int(max_iter), ctypes.byref(it),
                               ctypes.byref(up), ctypes.byref(rr))
    _check(st, "cg_mixed")
    return x, st, it.value, up.value, rr.value


def force_from_fields(dims, U, x, lam, flags=0):
    """Link gradient (4,V,3,3) of L(x), x = A^-1 b, given lam = A^-1 dL/dx (see oracle.c)."""
    d = _dims(dims)
    U = _c128(U)
    G = np.empty_like(U)
    _check(lib().oracle_force_from_fields(_ptr(d), flags, _ptr(U), _ptr(_c128(x)),
                                          _ptr(_c128(lam)), _ptr(G)), "force_from_fields")
    return G


def force(dims, U, mass, phi, tol=1e-13, max_iter=100000, flags=0):
    """S = phi^dag A^-1 phi and G = dS/dRe U + i dS/dIm U; returns (S, G, x, status)."""
    d = _dims(dims)
    U = _c128(U)
    phi = _c128(phi)
    G = np.empty_like(U)
    x = np.empty_like(phi)
    S = ctypes.c_double(0)
    st = lib().oracle_force(_ptr(d), flags, _ptr(U), float(mass), _ptr(phi), float(tol),
                            int(max_iter), _ptr(G), ctypes.byref(S), _ptr(x))
    _check(st, "force")
    return S.value, G, x, st


# ------------------------------------------------------------ NumPy helpers

def dense_D(dims, U, flags=0):
    """The full-lattice D as a dense (3V, 3V) matrix, one oracle application per column."""
    V = volume(dims)
    n = 3 * V
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 3), dtype=np.complex128)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        M[:, j] = dslash_full(dims, U, e, flags).reshape(-1)
        e.reshape(-1)[j] = 0.0
    return M


def dense_A(dims, U, mass, flags=0):
    """A = m^2 - D_eo D_oe as a dense (3V/2, 3V/2) matrix (columns from oracle applications)."""
    hv = volume(dims) // 2
    n = 3 * hv
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((hv, 3), dtype=np.complex128)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        M[:, j] = apply_A(dims, U, mass, e, flags).reshape(-1)
        e.reshape(-1)[j] = 0.0
    return M


def gell_mann():
    """The eight Gell-Mann matrices lambda_a, (8,3,3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3.0)
    lam[7][2, 2] = -2 / np.sqrt(3.0)
    return lam


def su3_force(U, G):
    """F^a = d/de S(exp(i e T_a) U) at e = 0 with T_a = lambda_a / 2, from the link
    gradient G: F^a = Re[i tr(T_a Q)], Q = U G^dag.  Shape (..., 8)."""
    Q = U @ np.conj(np.swapaxes(G, -1, -2))
    T = gell_mann() / 2.0
    return np.real(1j * np.einsum("aij,...ji->...a", T, Q))


def traceless_antihermitian(Q):
    """TA(Q) = (Q - Q^dag)/2 - tr(Q - Q^dag)/6 * 1."""
    A = 0.5 * (Q - np.conj(np.swapaxes(Q, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1)
    return A - (tr / 3.0)[..., None, None] * np.eye(3)
