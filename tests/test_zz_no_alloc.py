"""qx_apply_A_noalloc, the allocation-free variant of qx_apply_A (its odd
intermediate in the library's device array instead of a caller workspace),
called through the C ABI: bit for bit the output of qx_apply_A, on two calls
in a row, the second with a smaller input (fewer sources, smaller lattice,
lower precision) than the first; an input beyond the array is rejected."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import gauge, rel, to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu


def _noalloc(qx, g, packed_in, masses, out):
    import torch

    m = (ctypes.c_double * len(masses))(*masses)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return qx.load().qx_apply_A_noalloc(g._h, len(masses), m, ctypes.c_void_p(packed_in.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), stream)


def test_apply_A_noalloc_matches_apply_A(qx):
    import torch

    # (dims, precision, link storage, masses): the second call is smaller
    cases = [((16, 16, 16, 16), "f64", 18, [0.1, 0.35, 0.02]),
             ((8, 4, 6, 8), "f32", 12, [0.2, 0.05])]
    for n, (dims, prec, recon, masses) in enumerate(cases):
        lat = qx.Lattice(dims, antiperiodic_t=True)
        U = gauge(dims, seed=70 + n)
        g = qx.Gauge(lat, to_dev(U), prec, recon)
        nrhs = len(masses)
        b = synth.gauss_source(nrhs, lat.hv, 80 + n)
        pin = qx.pack(lat, to_dev(b), prec)
        ref = qx.apply_A(g, pin, masses)
        out = torch.full_like(ref, 0x5a)  # stale bytes: every output must be written
        assert _noalloc(qx, g, pin, masses, out) == qx.OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (dims, prec)
        # and against the oracle, to the precision's bar
        got = to_host(qx.unpack(lat, out, nrhs, prec))
        tol = 1e-13 if prec == "f64" else 1e-5
        for k in range(nrhs):
            want = oracle.apply_A(dims, U, masses[k], b[k], oracle.BC_T_ANTIPERIODIC)
            assert rel(got[k], want) <= tol, (dims, k)


def test_apply_A_noalloc_rejects_oversize(qx):
    import torch

    dims = (16, 16, 16, 16)
    lat = qx.Lattice(dims)
    g = qx.Gauge(lat, to_dev(gauge(dims, seed=72)), "f64", 18)
    nrhs = 22  # 22 x 1.5 MiB > 32 MiB
    masses = [0.1] * nrhs
    pin = torch.zeros(lat.field_bytes(nrhs, "f64"), dtype=torch.uint8, device="cuda")
    out = torch.zeros_like(pin)
    assert _noalloc(qx, g, pin, masses, out) == qx.EINVAL
    assert "holds" in qx.load().qx_last_error().decode()
    assert not out.any()
