"""FP16 storage (links and colour vectors with a per-site FP32 scale, FP32
arithmetic) against the FP64 oracle.

Bar: 1e-3 global relative L2 for the half-Dslash and A (about 2u).  binary16
keeps 11 significant bits, so each stored number carries a rounding error of
at most u = 2^-11 (4.9e-4) relative to its own binade; a colour vector is
stored as pairs scaled into [-1, 1] by the largest component of its site, and
links are stored directly (|U_ij| <= 1).  The half-Dslash output carries three
such roundings (input vector, links, output vector), each about u/sqrt(3) rms
relative for Gaussian inputs and adding in quadrature to about u (measured:
2.8e-4 to 3.0e-4 at 16^4 and 32^4 for 18-real, 12-real and improved-operator
links); 1e-3 leaves room for the worst of the small lattices.

The pack/unpack format itself is checked bit for bit against a numpy
transcription of its definition (scale = largest |re| or |im| of the site as
FP32; pair = component / scale in FP64, rounded once to binary16).
"""
import numpy as np
import pytest

import oracle
from gpu_util import gauge, rel, to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu

TOL16 = 1e-3
SHAPES_NL = [(1, 1), (1, 2), (1, 4), (1, 8), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2)]


def _quantise(b):
    """Numpy transcription of the FP16 field format: (pairs as float16 (n, hv, 3, 2), scales)."""
    parts = np.stack([b.real, b.imag], -1)
    m = np.abs(parts).max(axis=(2, 3))
    sc = m.astype(np.float32)
    inv = np.where(sc > 0, 1.0 / np.where(sc > 0, sc, 1).astype(np.float64), 0.0)
    q = (parts * inv[:, :, None, None]).astype(np.float16)
    return q, sc


def test_field_pack_f16_format(qx):
    """Pack and unpack against the format's definition, bit for bit, with an all-zero
    site and sites of very different magnitude; the per-site error bound holds."""
    dims = (6, 4, 2, 8)
    lat = qx.Lattice(dims)
    b = synth.gauss_source(3, lat.hv, 2)
    b[1, 7] = 0.0
    b[2, 11] *= 1e-6
    b[0, 5] *= 1e4
    # quotients just above a binary16 tie whose FP32 rounding lands on the tie:
    # one rounding from FP64 goes up, a detour through FP32 would go to even
    b[1, 9] = [1.0, 0.5 + 2.0 ** -12 + 2.0 ** -40, -(0.25 + 2.0 ** -13 + 2.0 ** -41) * 1j]
    b[2, 13] = [-1.0, 1j * (0.75 + 2.0 ** -12 + 2.0 ** -38), 0.125 + 2.0 ** -14 + 2.0 ** -43]
    back = to_host(qx.unpack(lat, qx.pack(lat, to_dev(b), "f16"), 3, "f16"))
    q, sc = _quantise(b)
    deq = q.astype(np.float64) * sc.astype(np.float64)[:, :, None, None]
    assert np.array_equal(back, deq[..., 0] + 1j * deq[..., 1])
    assert np.all(back[1, 7] == 0)
    m = np.abs(np.stack([b.real, b.imag], -1)).max(axis=(2, 3))
    err = np.abs(np.stack([(back - b).real, (back - b).imag], -1)).max(axis=(2, 3))
    assert np.all(err <= 2.0 ** -11 * m * (1 + 1e-6))


def _dslash16(qx, dims, recon, nrhs, parity, anti, seed, shape=None):
    lat = qx.Lattice(dims, antiperiodic_t=anti)
    flags = (oracle.BC_T_ANTIPERIODIC if anti else 0) | (oracle.NAIK if recon == 36 else 0)
    U = gauge(dims, seed=seed)
    g = qx.Gauge(lat, to_dev(U), "f16", recon)
    if shape is not None:
        g.set_launch(nrhs, *shape)
    chi = synth.gauss_source(nrhs, lat.hv, seed + 1)
    out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), "f16"), parity, nrhs), nrhs,
                            "f16"))
    return max(rel(out[k], oracle.dslash_eo(dims, U, chi[k], parity, flags)) for k in range(nrhs))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 6), (6, 4, 2, 8),
                                  (8, 8, 8, 12)])
@pytest.mark.parametrize("recon", [18, 12, 36])
def test_dslash_f16_parity(qx, dims, recon):
    for parity in (0, 1):
        for anti in (False, True):
            err = _dslash16(qx, dims, recon, 1, parity, anti, 40)
            assert err <= TOL16, (dims, recon, parity, anti, err)


@pytest.mark.parametrize("nbt,lps", SHAPES_NL)
@pytest.mark.parametrize("recon", [12, 36])
def test_dslash_f16_launch_shapes(qx, nbt, lps, recon):
    """Every compiled launch shape with 5 sources (partly filled groups, the
    cross-wavefront gather of whole colour vectors when lps > 1) on V/2 = 192."""
    err = _dslash16(qx, (6, 4, 2, 8), recon, 5, 1, True, 42, (nbt, lps, (nbt + lps) % 4))
    assert err <= TOL16, (nbt, lps, err)


@pytest.mark.parametrize("nrhs", [2, 12, 13])
def test_dslash_f16_multi_rhs(qx, nrhs):
    err = _dslash16(qx, (4, 6, 4, 8), 12, nrhs, 0, True, 44)
    assert err <= TOL16


def test_dslash_f16_32_4(qx):
    """Full-size lattice, FP16 12-real and improved-operator links."""
    dims = (32, 32, 32, 32)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    chi = synth.gauss_source(1, lat.hv, 1)
    pin = qx.pack(lat, to_dev(chi), "f16")
    for recon in (12, 36):
        ref = oracle.dslash_eo(dims, U, chi[0], 0, oracle.NAIK if recon == 36 else 0)
        g = qx.Gauge(lat, to_dev(U), "f16", recon)
        out = to_host(qx.unpack(lat, qx.dslash(g, pin, 0, 1), 1, "f16"))
        assert rel(out[0], ref) <= TOL16, recon


def test_dslash_f16_tuner_and_timer(qx):
    dims = (8, 8, 8, 12)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=46)
    g = qx.Gauge(lat, to_dev(U), "f16", 12)
    for nrhs in (1, 4):
        nbt, lps, xcd = g.tune(nrhs)
        assert (nbt, lps) in SHAPES_NL and xcd in range(6)
        chi = synth.gauss_source(nrhs, lat.hv, 47 + nrhs)
        pin = qx.pack(lat, to_dev(chi), "f16")
        out = qx.dslash(g, pin, 1, nrhs)
        out.zero_()
        assert 0.0 < qx.time_dslash(g, pin, 1, nrhs, out=out, reps=5) < 1.0
        got = to_host(qx.unpack(lat, out, nrhs, "f16"))
        for k in range(nrhs):
            ref = oracle.dslash_eo(dims, U, chi[k], 1, oracle.BC_T_ANTIPERIODIC)
            assert rel(got[k], ref) <= TOL16


@pytest.mark.parametrize("recon", [18, 12, 36])
def test_apply_A_f16_parity(qx, recon):
    dims = (4, 6, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=48)
    g = qx.Gauge(lat, to_dev(U), "f16", recon)
    v = synth.gauss_source(3, lat.hv, 49)
    masses = [0.1, 0.05, 0.5]
    out = to_host(qx.unpack(lat, qx.apply_A(g, qx.pack(lat, to_dev(v), "f16"), masses), 3, "f16"))
    flags = oracle.NAIK if recon == 36 else 0
    for k in range(3):
        assert rel(out[k], oracle.apply_A(dims, U, masses[k], v[k], flags)) <= TOL16


def test_f16_rejected_by_solvers(qx):
    """An FP16 handle serves a solve only as its inner links (glo, covered in
    test_gpu_f16_solve.py), never as the FP64 handle."""
    dims = (4, 4, 4, 4)
    lat = qx.Lattice(dims)
    Ud = to_dev(gauge(dims, seed=50))
    g64 = qx.Gauge(lat, Ud, "f64")
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    b = to_dev(synth.gauss_source(1, lat.hv, 51))
    with pytest.raises(qx.QXError) as e:
        qx.cg(g16, b, [0.1])
    assert e.value.code == qx.EINVAL
    with pytest.raises(qx.QXError):
        qx.cg(g16, b, [0.1], glo=g16)
    with pytest.raises(qx.QXError):
        qx.force(g16, b, 0.1)
    with pytest.raises(qx.QXError):
        qx.meson_correlators(g16, 0.1, (0, 0, 0, 0), glo=g16)
    U = gauge(dims, seed=50)
    p = np.zeros((4, lat.V, 8))
    Ud2, pd = to_dev(U), to_dev(p)
    g16b = qx.Gauge(lat, Ud2, "f16", 12)
    with pytest.raises(qx.QXError):
        qx.md_trajectory(g16b, Ud2, pd, 5.5, 0.01, 1)
    assert np.array_equal(to_host(Ud2), U)  # rejected before any update
