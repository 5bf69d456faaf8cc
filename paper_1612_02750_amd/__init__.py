"""MI355X-native staggered Dslash, even-odd CG and fermion force.

A thin ctypes binding of libqx.so (see include/qx.h for the C ABI).  PyTorch
provides device memory and streams only; every step of the computation runs in
the library's gfx950 kernels.  There is no CPU fallback: every entry point
raises if libqx.so is missing or no GPU is present.

Canonical layouts (complex128, on the GPU):
  gauge field  U   (4, V, 3, 3)        mu-major, lexicographic sites (x fastest)
  half field   b/x (nrhs, V/2, 3)      one parity, checkerboard order cb = lex >> 1
  link gradient G  (4, V, 3, 3)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqx.so")

OK, EINVAL, ENOMEM, EHIP, ENOTUNITARY, ENOTCONVERGED, EBREAKDOWN, ENOLIB = range(8)
BC_T_ANTIPERIODIC = 1
PREC_F64, PREC_F32, PREC_F16 = 0, 1, 2
CG_FP64, CG_MIXED_F32 = 0, 1
ENGINE_AUTO, ENGINE_LAUNCH, ENGINE_PERSISTENT, ENGINE_FUSED, ENGINE_FUSED2 = 0, 1, 2, 3, 4

_PREC = {"f64": PREC_F64, "f32": PREC_F32, "f16": PREC_F16, PREC_F64: PREC_F64,
         PREC_F32: PREC_F32, PREC_F16: PREC_F16}


class QXError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qx error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("mode", ctypes.c_int),
                ("delta", ctypes.c_double), ("use_x0", ctypes.c_int), ("chunk", ctypes.c_int),
                ("engine", ctypes.c_int)]


class _MdParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mass", ctypes.c_double), ("eps", ctypes.c_double),
                ("nsteps", ctypes.c_int), ("cg", _Params)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("reliable_updates", ctypes.c_int), ("true_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class _PassStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int), ("active_launches", ctypes.c_int),
                ("source_launches", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("active_ms", ctypes.c_double)]


PASS_NAMES = ("p", "doe", "deo", "xr", "finalize", "update")


class _System(ctypes.Structure):
    _fields_ = [("g64", ctypes.c_void_p), ("glo", ctypes.c_void_p), ("nrhs", ctypes.c_int),
                ("masses", ctypes.POINTER(ctypes.c_double)), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p)]


@dataclass
class Stats:
    status: int
    iters: int
    reliable_updates: int
    true_rel_residual: float
    seconds: float


_lib = None
_P, _I, _U32, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t


def load():
    """Load libqx.so (built by paper_1612_02750_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QXError(ENOLIB, f"{LIB_PATH} is missing: build it with python -m paper_1612_02750_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "qx_version": ([], _I),
        "qx_last_error": ([], ctypes.c_char_p),
        "qx_lattice_create": ([_P, _U32, _P], _I),
        "qx_lattice_destroy": ([_P], _I),
        "qx_lattice_volume": ([_P], ctypes.c_int64),
        "qx_debug_index_maps": ([_P, _P, _P, _P], _I),
        "qx_gauge_bytes": ([_P, _I, _I, _P], _I),
        "qx_gauge_load": ([_P, _P, _I, _I, _P, _P, _P], _I),
        "qx_gauge_destroy": ([_P], _I),
        "qx_field_bytes": ([_P, _I, _I, _P], _I),
        "qx_field_pack": ([_P, _I, _I, _P, _P, _P], _I),
        "qx_field_unpack": ([_P, _I, _I, _P, _P, _P], _I),
        "qx_dslash": ([_P, _I, _I, _P, _P, _P], _I),
        "qx_apply_A": ([_P, _I, _P, _P, _P, _P, _P], _I),
        "qx_cg_workspace_bytes": ([_P, _P, _I, _P], _I),
        "qx_cg_solve": ([_P, _P, _P, _I, _P, _P, _P, _P, _SZ, _P, _P], _I),
        "qx_batch_workspace_bytes": ([_I, _P, _P, _P], _I),
        "qx_batch_create": ([_I, _P, _P, _P, _SZ, _P, _P], _I),
        "qx_batch_solve": ([_P, _P, _P], _I),
        "qx_batch_solve_async": ([_P, _I, _P, _P], _I),
        "qx_batch_info": ([_P, _P, _P], _I),
        "qx_batch_tune": ([_P, _I, _P, _P, _P, _P], _I),
        "qx_tune_cache_load": ([ctypes.c_char_p], _I),
        "qx_tune_cache_save": ([ctypes.c_char_p], _I),
        "qx_batch_destroy": ([_P], _I),
        "qx_force_from_fields": ([_P, _I, _P, _P, _P, _P, _P], _I),
        "qx_force_workspace_bytes": ([_P, _P, _I, _P], _I),
        "qx_force": ([_P, _P, _P, _I, ctypes.c_double, _P, _P, _P, _P, _P, _SZ, _P, _P], _I),
        "qx_force_su3": ([_P, _P, _P, _P, _P], _I),
        "qx_action_backward": ([_P, _I, ctypes.c_double, _P, _P, _P, _P, _P], _I),
        "qx_batch_profile": ([_P, _I, _P, _P, _P], _I),
        "qx_apply_A_noalloc": ([_P, _I, _P, _P, _P, _P], _I),
        "qx_batch_set_launch": ([_P, _I, _I, _I, _P], _I),
        "qx_batch_get_launch": ([_P, _P, _P, _P, _P, _P], _I),
        "qx_batch_set_deo_launch": ([_P, _I, _I, _P], _I),
        "qx_tune_dslash": ([_P, _I, _P, _P], _I),
        "qx_gauge_action": ([_P, _P, ctypes.c_double, _P, _SZ, _P, _P], _I),
        "qx_gauge_force": ([_P, _P, ctypes.c_double, _P, _I, _P], _I),
        "qx_md_update_momenta": ([_P, _P, _P, ctypes.c_double, _P, _P], _I),
        "qx_md_update_links": ([_P, _P, ctypes.c_double, _P, _P], _I),
        "qx_md_kinetic": ([_P, _P, _P, _SZ, _P, _P], _I),
        "qx_md_workspace_bytes": ([_P, _P, _P], _I),
        "qx_meson_workspace_bytes": ([_P, _P, _P], _I),
        "qx_meson_correlators": ([_P, _P, _P, ctypes.c_double, _P, _I, _P, _P, _P, _SZ, _P, _P],
                                 _I),
        "qx_md_trajectory": ([_P, _P, _P, _P, _P, _P, _P, _SZ, _P, _P, _P, _P], _I),
        "qx_time_dslash": ([_P, _I, _I, _P, _P, _I, _P, _P], _I),
        "qx_get_launch": ([_P, _I, _P, _P, _P], _I),
        "qx_set_launch": ([_P, _I, _I, _I, _I], _I),
        "qx_probe_copy": ([_P, _P, _SZ, _P], _I),
        "qx_probe_read": ([_P, _SZ, _P, _P], _I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise QXError(ENOLIB, "no GPU: the qx library has no CPU path")
    return torch


def _check(rc, allowed=(OK,)):
    if rc not in allowed:
        raise QXError(rc, load().qx_last_error().decode())
    return rc


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype=None, shape=None, name="tensor"):
    torch = _torch()
    if not t.is_cuda:
        raise QXError(EINVAL, f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise QXError(EINVAL, f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise QXError(EINVAL, f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise QXError(EINVAL, f"{name} must be contiguous")
    return t


def _bytes(n):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device="cuda")


# ----------------------------------------------------------------- lattice

class Lattice:
    """A 4-D lattice with even extents (the even-odd split needs them)."""

    def __init__(self, dims: Sequence[int], antiperiodic_t: bool = False):
        L = load()
        self.dims = tuple(int(d) for d in dims)
        arr = (ctypes.c_int32 * 4)(*self.dims)
        h = ctypes.c_void_p()
        _check(L.qx_lattice_create(arr, BC_T_ANTIPERIODIC if antiperiodic_t else 0,
                                   ctypes.byref(h)))
        self._h = h
        self.V = int(L.qx_lattice_volume(h))
        self.hv = self.V // 2
        self.flags = BC_T_ANTIPERIODIC if antiperiodic_t else 0

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qx_lattice_destroy(self._h)
            self._h = None

    def field_bytes(self, nrhs: int, prec="f64") -> int:
        n = ctypes.c_size_t()
        _check(load().qx_field_bytes(self._h, nrhs, _PREC[prec], ctypes.byref(n)))
        return n.value

    def index_maps(self, stream=None):
        """(lex_of_eo[V], nbr_eo[V, 8]) int32 computed by the device geometry code."""
        torch = _torch()
        lex = torch.empty(self.V, dtype=torch.int32, device="cuda")
        nbr = torch.empty((self.V, 8), dtype=torch.int32, device="cuda")
        _check(load().qx_debug_index_maps(self._h, _ptr(lex), _ptr(nbr), _stream(stream)))
        return lex, nbr


# ------------------------------------------------------------------- gauge

RECON_18, RECON_12, RECON_NAIK = 18, 12, 36


class Gauge:
    """Packed gauge field (eta and boundary signs folded in) of one precision.
    recon: 18 or 12 reals per link for the one-hop operator, or RECON_NAIK (36)
    for the improved operator with the Naik three-hop term (one-hop and
    three-hop links of 18 reals each)."""

    def __init__(self, lat: Lattice, U, prec="f64", recon: int = 18, stream=None):
        torch = _torch()
        L = load()
        _dev(U, torch.complex128, (4, lat.V, 3, 3), "U")
        self.lat = lat
        self.prec = _PREC[prec]
        self.recon = int(recon)
        n = ctypes.c_size_t()
        _check(L.qx_gauge_bytes(lat._h, self.prec, self.recon, ctypes.byref(n)))
        self.packed = _bytes(n.value)
        h = ctypes.c_void_p()
        _check(L.qx_gauge_load(lat._h, _ptr(U), self.prec, self.recon, _ptr(self.packed),
                               _stream(stream), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qx_gauge_destroy(self._h)
            self._h = None

    def tune(self, nrhs: int = 1, stream=None):
        scratch = _bytes(2 * self.lat.field_bytes(nrhs, self.prec))
        _check(load().qx_tune_dslash(self._h, nrhs, _ptr(scratch), _stream(stream)))
        return self.launch(nrhs)

    def launch(self, nrhs: int = 1):
        """(sources per thread, wavefronts per site, XCD order) of the stencil kernels."""
        n, l, x = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().qx_get_launch(self._h, nrhs, ctypes.byref(n), ctypes.byref(l), ctypes.byref(x)))
        return n.value, l.value, x.value

    def set_launch(self, nrhs: int, nbt: int, lps: int, xcd_order: int):
        _check(load().qx_set_launch(self._h, nrhs, nbt, lps, xcd_order))


def tune_cache_load(path: str):
    """Merge the launch shapes of a JSON cache file into the process cache."""
    _check(load().qx_tune_cache_load(os.fsencode(path)))


def tune_cache_save(path: str):
    """Write the process cache of launch shapes to a JSON file."""
    _check(load().qx_tune_cache_save(os.fsencode(path)))


# ------------------------------------------------------------------ fields

def pack(lat: Lattice, canon, prec="f64", stream=None):
    """canonical complex128 (nrhs, V/2, 3) -> packed bytes."""
    torch = _torch()
    _dev(canon, torch.complex128, None, "field")
    nrhs = canon.shape[0]
    assert tuple(canon.shape[1:]) == (lat.hv, 3), "field must be (nrhs, V/2, 3)"
    out = _bytes(lat.field_bytes(nrhs, prec))
    _check(load().qx_field_pack(lat._h, nrhs, _PREC[prec], _ptr(canon), _ptr(out), _stream(stream)))
    return out


def unpack(lat: Lattice, packed, nrhs: int, prec="f64", stream=None):
    torch = _torch()
    out = torch.empty((nrhs, lat.hv, 3), dtype=torch.complex128, device="cuda")
    _check(load().qx_field_unpack(lat._h, nrhs, _PREC[prec], _ptr(packed), _ptr(out),
                                  _stream(stream)))
    return out


def dslash(g: Gauge, packed_in, out_parity: int, nrhs: int = 1, out=None, stream=None):
    """D (with 1/2) from parity 1 - out_parity to out_parity on packed fields."""
    if out is None:
        out = _bytes(g.lat.field_bytes(nrhs, g.prec))
    _check(load().qx_dslash(g._h, out_parity, nrhs, _ptr(packed_in), _ptr(out), _stream(stream)))
    return out


def time_dslash(g: Gauge, packed_in, out_parity: int, nrhs: int = 1, out=None, reps: int = 100,
                stream=None) -> float:
    """Average device seconds of one half-Dslash launch, from `reps` launches
    replayed out of a HIP graph between two HIP events."""
    if out is None:
        out = _bytes(g.lat.field_bytes(nrhs, g.prec))
    ms = ctypes.c_double()
    _check(load().qx_time_dslash(g._h, out_parity, nrhs, _ptr(packed_in), _ptr(out), reps,
                                 ctypes.byref(ms), _stream(stream)))
    return ms.value * 1e-3


def apply_A(g: Gauge, packed_in, masses: Sequence[float], out=None, tmp=None, stream=None):
    """(m^2 - D_eo D_oe) on packed even fields, one mass per source."""
    nrhs = len(masses)
    fb = g.lat.field_bytes(nrhs, g.prec)
    out = _bytes(fb) if out is None else out
    tmp = _bytes(fb) if tmp is None else tmp
    m = (ctypes.c_double * nrhs)(*masses)
    _check(load().qx_apply_A(g._h, nrhs, m, _ptr(packed_in), _ptr(out), _ptr(tmp),
                             _stream(stream)))
    return out


def apply_A_noalloc(g: Gauge, packed_in, masses: Sequence[float], out=None, stream=None):
    """apply_A with the odd intermediate in the library's device array (no
    workspace; at most 32 MiB of it)."""
    nrhs = len(masses)
    out = _bytes(g.lat.field_bytes(nrhs, g.prec)) if out is None else out
    m = (ctypes.c_double * nrhs)(*masses)
    _check(load().qx_apply_A_noalloc(g._h, nrhs, m, _ptr(packed_in), _ptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------------ solver

def _params(tol, max_iter, mode, delta, use_x0, chunk, engine=ENGINE_AUTO):
    return _Params(float(tol), int(max_iter), int(mode), float(delta), int(use_x0), int(chunk),
                   int(engine))


def _stats(arr, n):
    return [Stats(arr[i].status, arr[i].iters, arr[i].reliable_updates,
                  arr[i].true_rel_residual, arr[i].seconds) for i in range(n)]


def cg(g64: Gauge, b, masses, glo: Optional[Gauge] = None, tol=1e-10, max_iter=100000,
       mode=None, delta=0.1, x0=None, chunk=0, ws=None, stream=None, raise_on_fail=True,
       engine=ENGINE_AUTO):
    """Solve (m_s^2 - D_eo D_oe) x_s = b_s; b (nrhs, V/2, 3) complex128.  Returns (x, stats).
    mode defaults to mixed FP32/FP64 when glo (an FP32 or FP16 Gauge: the inner links) is
    given, else FP64."""
    torch = _torch()
    L = load()
    lat = g64.lat
    _dev(b, torch.complex128, None, "b")
    nrhs = b.shape[0]
    if isinstance(masses, (int, float)):
        masses = [float(masses)] * nrhs
    if mode is None:
        mode = CG_MIXED_F32 if glo is not None else CG_FP64
    p = _params(tol, max_iter, mode, delta, x0 is not None, chunk, engine)
    n = ctypes.c_size_t()
    _check(L.qx_cg_workspace_bytes(lat._h, ctypes.byref(p), nrhs, ctypes.byref(n)))
    if ws is None:
        ws = _bytes(n.value)
    x = x0.clone() if x0 is not None else torch.empty_like(b)
    st = (_Stats * nrhs)()
    m = (ctypes.c_double * nrhs)(*masses)
    rc = L.qx_cg_solve(g64._h, glo._h if glo is not None else None, ctypes.byref(p), nrhs, m,
                       _ptr(b), _ptr(x), _ptr(ws), ws.numel(), st, _stream(stream))
    if raise_on_fail:
        _check(rc)
    return x, _stats(st, nrhs)


class Batch:
    """Many systems (lattices of any size, several sources each) solved together:
    one launch per CG step for all of them, replayed from a captured HIP graph."""

    def __init__(self, systems, tol=1e-10, max_iter=100000, mode=CG_MIXED_F32, delta=0.1,
                 chunk=0, stream=None, engine=ENGINE_AUTO):
        """systems: list of (g64, glo_or_None, b (nrhs,V/2,3), masses, x_out)."""
        L = load()
        self.systems = systems
        self.p = _params(tol, max_iter, mode, delta, 0, chunk, engine)
        arr = (_System * len(systems))()
        self._masses = []
        self.nsrc = 0
        for i, (g64, glo, b, masses, x) in enumerate(systems):
            nrhs = b.shape[0]
            m = (ctypes.c_double * nrhs)(*masses)
            self._masses.append(m)
            arr[i] = _System(g64._h, glo._h if glo is not None else None, nrhs,
                             ctypes.cast(m, ctypes.POINTER(ctypes.c_double)), b.data_ptr(),
                             x.data_ptr())
            self.nsrc += nrhs
        self._arr = arr
        n = ctypes.c_size_t()
        _check(L.qx_batch_workspace_bytes(len(systems), arr, ctypes.byref(self.p),
                                          ctypes.byref(n)))
        self.ws = _bytes(n.value)
        h = ctypes.c_void_p()
        _check(L.qx_batch_create(len(systems), arr, ctypes.byref(self.p), _ptr(self.ws),
                                 self.ws.numel(), _stream(stream), ctypes.byref(h)))
        self._h = h

    def solve(self, stream=None, raise_on_fail=True):
        st = (_Stats * self.nsrc)()
        rc = load().qx_batch_solve(self._h, st, _stream(stream))
        if raise_on_fail:
            _check(rc)
        return _stats(st, self.nsrc)

    def tune(self, nchunks: int = 2, stream=None):
        """Time nchunks chunks of this batch's solve under every launch shape
        it admits and keep the fastest; returns (nbt, lps, order)."""
        n, l, o = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().qx_batch_tune(self._h, int(nchunks), ctypes.byref(n), ctypes.byref(l),
                                    ctypes.byref(o), _stream(stream)))
        return n.value, l.value, o.value

    def set_launch(self, nbt: int, lps: int, order: int, stream=None):
        """Solve under this launch shape from now on (as a tuner result)."""
        _check(load().qx_batch_set_launch(self._h, int(nbt), int(lps), int(order), _stream(stream)))

    def set_deo_launch(self, nbt: int, lps: int, stream=None):
        """Launch-per-pass engine: run the D_eo pass under (nbt, lps)."""
        _check(load().qx_batch_set_deo_launch(self._h, int(nbt), int(lps), _stream(stream)))

    def launch(self):
        """((nbt, lps, order) of the stencil passes, (nbt, lps) of the
        launch-per-pass engine's D_eo pass)."""
        v = [ctypes.c_int() for _ in range(5)]
        _check(load().qx_batch_get_launch(self._h, *(ctypes.byref(x) for x in v)))
        return (v[0].value, v[1].value, v[2].value), (v[3].value, v[4].value)

    def profile(self, nchunks: int = 2, stream=None):
        """Event timing of nchunks chunks of this batch's solve, pass by pass:
        {pass name: {launches, active_launches, source_launches, ms, active_ms}}
        and the statistics after the last chunk."""
        ps = (_PassStats * len(PASS_NAMES))()
        st = (_Stats * self.nsrc)()
        _check(load().qx_batch_profile(self._h, int(nchunks), ps, st, _stream(stream)))
        out = {n: {f: getattr(ps[i], f) for f, _ in _PassStats._fields_}
               for i, n in enumerate(PASS_NAMES)}
        return out, _stats(st, self.nsrc)

    def chunk(self) -> int:
        c = ctypes.c_int()
        _check(load().qx_batch_info(self._h, None, ctypes.byref(c)))
        return c.value

    def solve_async(self, nchunks: int, stats=None, stream=None):
        """Enqueue a whole solve of at most nchunks chunks with no host
        synchronisation; returns the device buffer the statistics land in
        (decode with stats_from_device once the stream has reached it)."""
        if stats is None:
            stats = _bytes(ctypes.sizeof(_Stats) * self.nsrc)
        _check(load().qx_batch_solve_async(self._h, int(nchunks), _ptr(stats), _stream(stream)))
        return stats

    def stats_from_device(self, stats):
        host = stats.cpu().numpy().tobytes()
        arr = (_Stats * self.nsrc).from_buffer_copy(host)
        return _stats(arr, self.nsrc)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.qx_batch_destroy(self._h)
            self._h = None


# ------------------------------------------------------------------- force

def force(g64: Gauge, phi, mass: float, glo: Optional[Gauge] = None, tol=1e-10,
          max_iter=100000, mode=None, delta=0.1, stream=None):
    """S = sum_s phi_s^dag A^-1 phi_s and G = dS/dRe U + i dS/dIm U (4,V,3,3).
    Returns (S, G, x, stats)."""
    torch = _torch()
    L = load()
    lat = g64.lat
    _dev(phi, torch.complex128, None, "phi")
    nrhs = phi.shape[0]
    if mode is None:
        mode = CG_MIXED_F32 if glo is not None else CG_FP64
    p = _params(tol, max_iter, mode, delta, 0, 0)
    n = ctypes.c_size_t()
    _check(L.qx_force_workspace_bytes(lat._h, ctypes.byref(p), nrhs, ctypes.byref(n)))
    ws = _bytes(n.value)
    G = torch.empty((4, lat.V, 3, 3), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(phi)
    S = ctypes.c_double()
    st = (_Stats * nrhs)()
    _check(L.qx_force(g64._h, glo._h if glo is not None else None, ctypes.byref(p), nrhs,
                      float(mass), _ptr(phi), _ptr(G), ctypes.byref(S), _ptr(x), _ptr(ws),
                      ws.numel(), st, _stream(stream)))
    return S.value, G, x, _stats(st, nrhs)


def action_backward(lat: Lattice, gS: float, G, x, need_U=True, need_phi=True, stream=None):
    """Backward of S = sum_s phi_s^dag A^-1 phi_s for the upstream gradient gS:
    (gS * G, 2 gS x), either None when not needed (computed by the library)."""
    torch = _torch()
    gU = torch.empty_like(G) if need_U else None
    gphi = torch.empty_like(x) if need_phi else None
    _check(load().qx_action_backward(lat._h, x.shape[0], float(gS), _ptr(G), _ptr(x),
                                     _ptr(gU) if need_U else None,
                                     _ptr(gphi) if need_phi else None, _stream(stream)))
    return gU, gphi


# ------------------------------------------------------- molecular dynamics

_MD_RED_BYTES = 8200 + 256


def gauge_action(lat: Lattice, U, beta: float, stream=None) -> float:
    """Wilson plaquette action beta sum_{x, mu<nu} (1 - Re tr P_munu / 3)."""
    ws = _bytes(_MD_RED_BYTES)
    S = ctypes.c_double()
    _check(load().qx_gauge_action(lat._h, _ptr(U), float(beta), _ptr(ws), ws.numel(),
                                  ctypes.byref(S), _stream(stream)))
    return S.value


def gauge_force(lat: Lattice, U, beta: float, G=None, accumulate=False, stream=None):
    """Link gradient of the plaquette action, -(beta/3) A^dag (4, V, 3, 3); added to G
    when accumulate."""
    torch = _torch()
    if G is None:
        G = torch.empty((4, lat.V, 3, 3), dtype=torch.complex128, device="cuda")
    _check(load().qx_gauge_force(lat._h, _ptr(U), float(beta), _ptr(G), 1 if accumulate else 0,
                                 _stream(stream)))
    return G


def md_update_momenta(lat: Lattice, U, G, eps: float, p, stream=None):
    """p^a -= eps Re[i tr(T_a U G^dag)] in place; p float64 (4, V, 8)."""
    _check(load().qx_md_update_momenta(lat._h, _ptr(U), _ptr(G), float(eps), _ptr(p),
                                       _stream(stream)))
    return p


def md_update_links(lat: Lattice, p, eps: float, U, stream=None):
    """U <- exp(i eps sum_a p^a T_a) U in place."""
    _check(load().qx_md_update_links(lat._h, _ptr(p), float(eps), _ptr(U), _stream(stream)))
    return U


def md_kinetic(lat: Lattice, p, stream=None) -> float:
    ws = _bytes(_MD_RED_BYTES)
    K = ctypes.c_double()
    _check(load().qx_md_kinetic(lat._h, _ptr(p), _ptr(ws), ws.numel(), ctypes.byref(K),
                                _stream(stream)))
    return K.value


def md_trajectory(g64: Gauge, U, p, beta: float, eps: float, nsteps: int, phi=None,
                  mass: float = 0.1, glo: Optional[Gauge] = None, tol=1e-10, max_iter=100000,
                  mode=None, delta=0.1, stream=None):
    """One leapfrog trajectory: U (4, V, 3, 3) complex128 and p (4, V, 8) float64 advanced
    in place; g64 (and glo) are repacked from U.  Returns (H_start, H_end, CG iterations)."""
    L = load()
    if mode is None:
        mode = CG_MIXED_F32 if glo is not None else CG_FP64
    mp = _MdParams(float(beta), float(mass), float(eps), int(nsteps),
                   _params(tol, max_iter, mode, delta, 0, 0))
    n = ctypes.c_size_t()
    _check(L.qx_md_workspace_bytes(g64.lat._h, ctypes.byref(mp), ctypes.byref(n)))
    ws = _bytes(n.value)
    h0, h1, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _check(L.qx_md_trajectory(g64._h, glo._h if glo is not None else None, ctypes.byref(mp),
                              _ptr(U), _ptr(p), _ptr(phi) if phi is not None else None, _ptr(ws),
                              ws.numel(), ctypes.byref(h0), ctypes.byref(h1), ctypes.byref(it),
                              _stream(stream)))
    return h0.value, h1.value, it.value


def meson_correlators(g64: Gauge, mass: float, src, masks=(0,), glo: Optional[Gauge] = None,
                      tol=1e-10, max_iter=100000, mode=None, delta=0.1, stream=None):
    """Point-source staggered meson correlators C[k][t] (numpy (nmask, L_t)) for the
    direction masks (mask 0: Goldstone pion); src: even site (x, y, z, t)."""
    import numpy as np

    L = load()
    if mode is None:
        mode = CG_MIXED_F32 if glo is not None else CG_FP64
    p = _params(tol, max_iter, mode, delta, 0, 0)
    n = ctypes.c_size_t()
    _check(L.qx_meson_workspace_bytes(g64.lat._h, ctypes.byref(p), ctypes.byref(n)))
    ws = _bytes(n.value)
    srcs = (ctypes.c_int * 4)(*[int(v) for v in src])
    mk = (ctypes.c_int * len(masks))(*[int(v) for v in masks])
    Lt = g64.lat.dims[3]
    C = (ctypes.c_double * (len(masks) * Lt))()
    st = (_Stats * 3)()
    _check(L.qx_meson_correlators(g64._h, glo._h if glo is not None else None, ctypes.byref(p),
                                  float(mass), srcs, len(masks), mk, C, _ptr(ws), ws.numel(), st,
                                  _stream(stream)))
    return np.array(C[:]).reshape(len(masks), Lt), _stats(st, 3)


def force_from_fields(g64: Gauge, x, lam, stream=None):
    """Link gradient of L(x), x = A^-1 b, given lam = A^-1 dL/dx; x, lam canonical."""
    torch = _torch()
    lat = g64.lat
    nrhs = x.shape[0]
    xp = pack(lat, x, "f64", stream)
    lp = xp if lam is x else pack(lat, lam, "f64", stream)
    tmp = _bytes(2 * lat.field_bytes(nrhs, "f64"))
    G = torch.empty((4, lat.V, 3, 3), dtype=torch.complex128, device="cuda")
    _check(load().qx_force_from_fields(g64._h, nrhs, _ptr(xp), _ptr(lp), _ptr(tmp), _ptr(G),
                                       _stream(stream)))
    return G


def probe_copy(dst, src, nbytes: int, stream=None):
    """dst = src with the library's streaming copy kernel (bandwidth reference)."""
    _check(load().qx_probe_copy(_ptr(dst), _ptr(src), int(nbytes), _stream(stream)))


def probe_read(src, nbytes: int, scratch, stream=None):
    """Read nbytes of src once with the library's streaming read kernel."""
    _check(load().qx_probe_read(_ptr(src), int(nbytes), _ptr(scratch), _stream(stream)))


def force_su3(lat: Lattice, U, G, stream=None):
    """F^a = Re[i tr(T_a U G^dag)], T_a = lambda_a / 2: (4, V, 8) float64."""
    torch = _torch()
    F = torch.empty((4, lat.V, 8), dtype=torch.float64, device="cuda")
    _check(load().qx_force_su3(lat._h, _ptr(U), _ptr(G), _ptr(F), _stream(stream)))
    return F


def __getattr__(name):
    # the autograd wrappers import torch; load them on first use only
    if name in ("StaggeredSolve", "staggered_action", "StaggeredAction"):
        from . import autograd

        return getattr(autograd, name)
    raise AttributeError(name)
