"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: index maps bit-exact; Dslash / A within 1e-13 (FP64) and 1e-5 (FP32)
global relative L2; solves reach a true FP64 relative residual <= 1e-10 measured
by the oracle on the returned x, with the error against the oracle's own
solution reported and bounded by cond(A) * tol.
"""
import numpy as np
import pytest

import oracle
from gpu_util import gauge, half_vol, rel, to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 6), (6, 4, 2, 8), (8, 8, 8, 12), (16, 16, 16, 32)]


# ---------------------------------------------------------------- a1 geometry

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 6), (6, 6, 6, 6),
                                  (8, 8, 8, 12), (16, 16, 16, 32)])
def test_index_maps_bit_exact(qx, dims):
    lat = qx.Lattice(dims)
    lex, nbr = lat.index_maps()
    lex_o, nbr_o = oracle.index_maps(dims)
    assert np.array_equal(to_host(lex), lex_o)
    assert np.array_equal(to_host(nbr), nbr_o)


# ------------------------------------------------------------- a2/a3 packing

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_field_pack_roundtrip(qx, prec):
    dims = (6, 4, 2, 8)
    lat = qx.Lattice(dims)
    b = synth.gauss_source(3, lat.hv, 2)
    bd = to_dev(b)
    back = to_host(qx.unpack(lat, qx.pack(lat, bd, prec), 3, prec))
    if prec == "f64":
        assert np.array_equal(back, b)
    else:
        ref = b.real.astype(np.float32).astype(np.float64) + 1j * b.imag.astype(np.float32)
        assert np.array_equal(back, ref)


def test_recon12_rejects_non_su3(qx):
    dims = (4, 4, 4, 4)
    lat = qx.Lattice(dims)
    U = gauge(dims)
    U[2, 17] *= 1.001
    with pytest.raises(qx.QXError) as e:
        qx.Gauge(lat, to_dev(U), "f64", 12)
    assert e.value.code == qx.ENOTUNITARY
    with pytest.raises(qx.QXError) as e:
        qx.Gauge(lat, to_dev(synth.unit_gauge(dims) * 1j ** (1 / 3)), "f32", 12)
    assert e.value.code == qx.ENOTUNITARY
    # a NaN only in row 2 (the row that 12-real storage drops)
    U = gauge(dims)
    U[1, 5, 2, 1] = np.nan
    with pytest.raises(qx.QXError) as e:
        qx.Gauge(lat, to_dev(U), "f32", 12)
    assert e.value.code == qx.ENOTUNITARY
    # rows 0 and 1 scaled by a phase pair whose product keeps row 2 consistent
    # but breaks the orthonormality of the rows: U' = diag(2, 1/2, 1) U
    U = gauge(dims)
    U[0, 9, 0] *= 2.0
    U[0, 9, 1] *= 0.5
    with pytest.raises(qx.QXError) as e:
        qx.Gauge(lat, to_dev(U), "f64", 12)
    assert e.value.code == qx.ENOTUNITARY
    # SU(3) links pass
    qx.Gauge(lat, to_dev(gauge(dims)), "f32", 12)


def test_invalid_lattice(qx):
    for dims in [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 1, 4)]:
        with pytest.raises(qx.QXError) as e:
            qx.Lattice(dims)
        assert e.value.code == qx.EINVAL


# ---------------------------------------------------------------- a4 Dslash

def _dslash_case(qx, dims, prec, recon, nrhs, parity, anti, kind="haar"):
    lat = qx.Lattice(dims, antiperiodic_t=anti)
    flags = oracle.BC_T_ANTIPERIODIC if anti else 0
    U = gauge(dims, kind, seed=1)
    g = qx.Gauge(lat, to_dev(U), prec, recon)
    chi = synth.gauss_source(nrhs, lat.hv, 3)
    out = qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), parity, nrhs), nrhs, prec)
    out = to_host(out)
    errs = []
    for k in range(nrhs):
        ref = oracle.dslash_eo(dims, U, chi[k], parity, flags)
        errs.append(rel(out[k], ref))
    return max(errs)


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("prec,recon,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13),
                                            ("f32", 18, 1e-5), ("f32", 12, 1e-5)])
def test_dslash_parity(qx, dims, prec, recon, tol):
    for parity in (0, 1):
        for anti in (False, True):
            err = _dslash_case(qx, dims, prec, recon, 1, parity, anti)
            assert err <= tol, (dims, prec, recon, parity, anti, err)


@pytest.mark.parametrize("nrhs", [2, 3, 4, 5, 8, 12, 13])
@pytest.mark.parametrize("prec,recon,tol", [("f64", 18, 1e-13), ("f32", 12, 1e-5)])
def test_dslash_multi_rhs(qx, nrhs, prec, recon, tol):
    err = _dslash_case(qx, (4, 6, 4, 8), prec, recon, nrhs, 0, True)
    assert err <= tol


SHAPES_NARROW = [(1, 1), (1, 2), (1, 4), (1, 8), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2)]
SHAPES_NL = SHAPES_NARROW + [(6, 1), (6, 2), (12, 1), (12, 2)]


@pytest.mark.parametrize("nbt,lps", SHAPES_NL)
@pytest.mark.parametrize("prec,recon,tol", [("f64", 18, 1e-13), ("f32", 12, 1e-5),
                                            ("f32", 18, 1e-5)])
def test_dslash_launch_shapes(qx, nbt, lps, prec, recon, tol):
    """Every compiled launch shape (sources per thread, wavefronts per site), with
    V/2 = 192 ragged against the 64-site tiles and a source count that leaves
    partly filled groups (5 sources: 6 and 12 per thread fill one group
    partly).  Six and twelve sources per thread exist for FP32 one-hop links
    only: FP64 rejects them."""
    dims = (6, 4, 2, 8)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=4)
    g = qx.Gauge(lat, to_dev(U), prec, recon)
    nrhs = 5
    if nbt > 4 and prec == "f64":
        with pytest.raises(qx.QXError):
            g.set_launch(nrhs, nbt, lps, 1)
        return
    g.set_launch(nrhs, nbt, lps, (nbt + lps) % 2)
    chi = synth.gauss_source(nrhs, lat.hv, 8)
    out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), 1, nrhs), nrhs, prec))
    for k in range(nrhs):
        ref = oracle.dslash_eo(dims, U, chi[k], 1, oracle.BC_T_ANTIPERIODIC)
        assert rel(out[k], ref) <= tol, (k, nbt, lps)


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("dims", [(8, 16, 4, 8), (16, 16, 6, 12), (8, 16, 8, 16)])
def test_dslash_block_orders(qx, order, dims):
    """Every block order, on lattices whose (z, t) planes hold whole 64-site
    blocks so that the tiled orders 2 and 3 are in effect (tiles cut to the
    divisors 2/3 of L2 = 6 and 6/4 of L3 = 12 on the second lattice); the slab
    orders 4 and 5 (with non-temporal output stores) are in effect where L2
    (order 4) or L3 (order 5) is a multiple of 8, and fall back to
    checkerboard order elsewhere."""
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=12)
    nrhs = 3
    chi = synth.gauss_source(nrhs, lat.hv, 13)
    refs = [oracle.dslash_eo(dims, U, chi[k], 0, oracle.BC_T_ANTIPERIODIC) for k in range(nrhs)]
    for prec, recon, tol in (("f64", 18, 1e-13), ("f32", 12, 1e-5)):
        g = qx.Gauge(lat, to_dev(U), prec, recon)
        for nbt, lps in ((1, 1), (1, 4), (2, 2), (4, 1)) + (((6, 2), (12, 1)) if prec == "f32" else ()):
            g.set_launch(nrhs, nbt, lps, order)
            out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), 0, nrhs),
                                    nrhs, prec))
            for k in range(nrhs):
                assert rel(out[k], refs[k]) <= tol, (prec, nbt, lps, order, k)


@pytest.mark.parametrize("order", [2, 3])
def test_cg_tiled_block_order(qx, order):
    """The CG engine (stencil passes, reliable updates and the per-block
    partials of the dot products) under a tiled block order."""
    dims = (8, 16, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=14)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    g32.set_launch(2, 1, 4, order)
    masses = [0.1, 0.2]
    b = synth.gauss_source(2, lat.hv, 15)
    x, st = qx.cg(g64, to_dev(b), masses, glo=g32, tol=1e-10)
    _check_solution(dims, U, masses, b, to_host(x), st)
    g32.set_launch(2, 1, 4, 1)
    x1, _ = qx.cg(g64, to_dev(b), masses, glo=g32, tol=1e-10)
    # the partials sit at the blocks' checkerboard positions: same sums, same bits
    assert np.array_equal(to_host(x), to_host(x1))


@pytest.mark.parametrize("prec,recon,tol", [("f64", 18, 1e-13), ("f32", 12, 1e-5)])
def test_tuner_and_graph_timer(qx, prec, recon, tol):
    """The autotuner settles on a compiled shape, and the graph-replayed timer
    writes the same half-Dslash as qx_dslash (checked against the oracle) and
    returns a positive time."""
    dims = (8, 8, 8, 12)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=9)
    g = qx.Gauge(lat, to_dev(U), prec, recon)
    for nrhs in (1, 3):
        nbt, lps, xcd = g.tune(nrhs)
        assert (nbt, lps) in SHAPES_NL and xcd in range(6)
        chi = synth.gauss_source(nrhs, lat.hv, 10 + nrhs)
        pin = qx.pack(lat, to_dev(chi), prec)
        out = qx.dslash(g, pin, 1, nrhs)
        out.zero_()
        t = qx.time_dslash(g, pin, 1, nrhs, out=out, reps=5)
        assert 0.0 < t < 1.0
        got = to_host(qx.unpack(lat, out, nrhs, prec))
        for k in range(nrhs):
            ref = oracle.dslash_eo(dims, U, chi[k], 1, oracle.BC_T_ANTIPERIODIC)
            assert rel(got[k], ref) <= tol, (k, nrhs)


@pytest.mark.parametrize("nbt,lps", SHAPES_NL)
def test_cg_launch_shapes(qx, nbt, lps):
    """The CG engine under every launch shape: 3 sources of different masses."""
    dims = (4, 6, 4, 4)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=5)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    g32.set_launch(3, nbt, lps, 1)
    masses = [0.1, 0.3, 0.05]
    b = synth.gauss_source(3, lat.hv, 6)
    x, st = qx.cg(g64, to_dev(b), masses, glo=g32, tol=1e-10)
    _check_solution(dims, U, masses, b, to_host(x), st)
    assert g32.launch(3) == (nbt, lps, 1)


def test_dslash_32_4_sampled(qx):
    """Full-size lattice (32^4): FP32 12-real and FP64 Dslash against the oracle."""
    dims = (32, 32, 32, 32)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    chi = synth.gauss_source(1, lat.hv, 1)
    ref = oracle.dslash_eo(dims, U, chi[0], 0)
    for prec, recon, tol in (("f64", 18, 1e-13), ("f32", 12, 1e-5)):
        g = qx.Gauge(lat, to_dev(U), prec, recon)
        out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), 0, 1), 1, prec))
        assert rel(out[0], ref) <= tol


def _pool_gauge(dims, seed):
    """SU(3) links for a large lattice, drawn (with replacement) from the
    262 144 Haar links of the 16^4 generator: every link is Haar-distributed,
    and two neighbouring links coincide with probability 4e-6, so a wrong link
    or neighbour index shows up as an error."""
    pool = gauge((16, 16, 16, 16), seed=seed).reshape(-1, 3, 3)
    V = int(np.prod(dims))
    idx = np.random.default_rng(seed + 100).integers(0, pool.shape[0], size=4 * V)
    return pool[idx].reshape(4, V, 3, 3)


def test_dslash_48_4(qx):
    """48^4 (the size of the benchmark's HBM-bound Dslash points): FP64 18-real
    under the XCD-contiguous and the tiled (z, t) block orders, FP32 12-real
    and FP16 12-real under several launch shapes, both output parities,
    against the oracle."""
    import torch

    dims = (48, 48, 48, 48)
    lat = qx.Lattice(dims)
    U = _pool_gauge(dims, 3)
    chi = synth.gauss_source(1, lat.hv, 7)
    Ud = to_dev(U)
    refs = [oracle.dslash_eo(dims, U, chi[0], p) for p in (0, 1)]
    del U
    cases = (("f64", 18, 1e-13, [(1, 1, 3), (1, 1, 1), (1, 4, 2)]),
             ("f32", 12, 1e-5, [(1, 8, 0), (1, 2, 0), (1, 1, 1)]),
             ("f16", 12, 1e-3, [(1, 1, 1), (1, 8, 0)]))
    for prec, recon, tol, shapes in cases:
        g = qx.Gauge(lat, Ud, prec, recon)
        pin = qx.pack(lat, to_dev(chi), prec)
        for shape in shapes:
            g.set_launch(1, *shape)
            for p in (0, 1):
                out = to_host(qx.unpack(lat, qx.dslash(g, pin, p, 1), 1, prec))[0]
                err = rel(out, refs[p])
                print(f"48^4 {prec}-{recon} shape {shape} parity {p}: {err:.2e}", flush=True)
                assert err <= tol, (prec, shape, p, err)
        del g, pin
        torch.cuda.empty_cache()


def test_free_field_dslash_closed_form(qx):
    """U = 1: a plane wave restricted to odd sites maps to the closed form on even sites."""
    dims = (8, 4, 6, 4)
    lat = qx.Lattice(dims)
    g = qx.Gauge(lat, to_dev(synth.unit_gauge(dims)), "f64", 18)
    V = lat.V
    lex = np.arange(V)
    x = np.stack([lex % 8, (lex // 8) % 4, (lex // 32) % 6, lex // 192], 1)
    par = x.sum(1) % 2
    p = np.array([2 * np.pi * 3 / 8, 2 * np.pi / 4, 2 * np.pi * 5 / 6, 2 * np.pi * 2 / 4])
    c = np.array([1 + 2j, -0.5j, 0.3])
    phi = np.exp(1j * x @ p)[:, None] * c[None, :]
    odd = np.zeros((lat.hv, 3), complex)
    odd[lex[par == 1] >> 1] = phi[par == 1]
    out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(odd[None])), 0, 1), 1))[0]
    eta = np.stack([np.ones(V), (-1.0) ** x[:, 0], (-1.0) ** (x[:, 0] + x[:, 1]),
                    (-1.0) ** (x[:, 0] + x[:, 1] + x[:, 2])], 1)
    fac = 1j * (eta * np.sin(p)[None, :]).sum(1)
    ev = lex[par == 0]
    np.testing.assert_allclose(out[ev >> 1], (fac[:, None] * phi)[ev], rtol=0, atol=1e-13)


# -------------------------------------------------------------- a5 operator A

@pytest.mark.parametrize("prec,recon,tol", [("f64", 18, 1e-13), ("f32", 18, 1e-5),
                                            ("f32", 12, 1e-5)])
def test_apply_A_parity(qx, prec, recon, tol):
    dims = (4, 6, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=2)
    g = qx.Gauge(lat, to_dev(U), prec, recon)
    v = synth.gauss_source(3, lat.hv, 5)
    masses = [0.1, 0.05, 0.5]
    out = to_host(qx.unpack(lat, qx.apply_A(g, qx.pack(lat, to_dev(v), prec), masses), 3, prec))
    for k in range(3):
        assert rel(out[k], oracle.apply_A(dims, U, masses[k], v[k])) <= tol


# ------------------------------------------------------------ a5-a7 solvers

def _check_solution(dims, U, masses, b, x, stats, tol=1e-10, flags=0):
    errs = []
    for k in range(b.shape[0]):
        rr = oracle.true_residual(dims, U, masses[k], b[k], x[k], flags)
        assert rr <= tol, (k, rr, stats[k])
        assert stats[k].status == 0
        assert abs(stats[k].true_rel_residual - rr) <= 1e-12
        errs.append(rr)
    return errs


def test_cg_fp64_config1(qx):
    """4^4 periodic, Haar seed 0, m = 0.1, one source: FP64 CG to 1e-10."""
    dims = (4, 4, 4, 4)
    m = 0.1
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    b = synth.gauss_source(1, lat.hv, 1)
    g64 = qx.Gauge(lat, to_dev(U), "f64")
    x, st = qx.cg(g64, to_dev(b), m, tol=1e-10)
    x = to_host(x)
    _check_solution(dims, U, [m], b, x, st)
    A = oracle.dense_A(dims, U, m)
    xd = np.linalg.solve(A, b[0].reshape(-1)).reshape(-1, 3)
    assert rel(x[0], xd) <= np.linalg.cond(A) * 1e-10


@pytest.mark.parametrize("recon", [18, 12])
def test_cg_mixed_config2(qx, recon):
    """16^4 weak field eps = 0.3, m = 0.05: FP32 inner, FP64 reliable updates."""
    dims = (16, 16, 16, 16)
    m = 0.05
    lat = qx.Lattice(dims)
    U = gauge(dims, "weak", seed=0, eps=0.3)
    b = synth.gauss_source(1, lat.hv, 1)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", recon)
    x, st = qx.cg(g64, to_dev(b), m, glo=g32, tol=1e-10)
    x = to_host(x)
    _check_solution(dims, U, [m], b, x, st)
    assert st[0].reliable_updates >= 3
    xo, sto, it, rr = oracle.cg(dims, U, m, b[0], tol=1e-12)
    assert rel(x[0], xo) <= 1e-7


def test_cg_fp64_vs_mixed_same_answer(qx):
    dims = (8, 8, 8, 8)
    m = 0.1
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, "haar", seed=3)
    b = synth.gauss_source(2, lat.hv, 4)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    x64, s64 = qx.cg(g64, to_dev(b), m, tol=1e-10)
    xmx, smx = qx.cg(g64, to_dev(b), m, glo=g32, tol=1e-10)
    _check_solution(dims, U, [m, m], b, to_host(x64), s64, flags=oracle.BC_T_ANTIPERIODIC)
    _check_solution(dims, U, [m, m], b, to_host(xmx), smx, flags=oracle.BC_T_ANTIPERIODIC)


def test_cg_multi_rhs_different_masses(qx):
    dims = (6, 4, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=6)
    masses = [0.05, 0.1, 0.2, 0.4, 1.0]
    b = synth.gauss_source(5, lat.hv, 9)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 18)
    x, st = qx.cg(g64, to_dev(b), masses, glo=g32, tol=1e-10)
    _check_solution(dims, U, masses, b, to_host(x), st)
    # heavier masses converge in fewer iterations
    assert st[4].iters < st[0].iters


def test_cg_multi_rhs_config3_32_4(qx):
    """32^4, Haar links, 12 sources, m = 0.02: FP32 12-real inner, FP64 reliable updates."""
    dims = (32, 32, 32, 32)
    m = 0.02
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    b = synth.gauss_source(12, lat.hv, 1)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    del Ud
    x, st = qx.cg(g64, to_dev(b), [m] * 12, glo=g32, tol=1e-10)
    x = to_host(x)
    for k in range(12):
        rr = oracle.true_residual(dims, U, m, b[k], x[k])
        print(f"source {k}: iters {st[k].iters}, oracle residual {rr:.2e}", flush=True)
        assert rr <= 1e-10 and st[k].status == 0, (k, rr)


@pytest.mark.parametrize("shape", [(12, 2, 4), (12, 1, 0), (6, 2, 5), (6, 1, 1), (4, 2, 4)])
def test_cg_wide_shapes_launch_engine(qx, shape):
    """Twelve sources under the launch-per-pass engine with six or twelve
    sources per thread and the slab block orders: every source solves to 1e-10
    by the oracle.  The masses differ, so the sources stop at different
    iterations and the stencils compute slots whose source no longer runs (their
    outputs are not stored).  The FP64 reliable updates take four sources per
    thread."""
    import torch

    dims = (8, 16, 8, 16)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=21)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    masses = [0.05 + 0.04 * k for k in range(12)]
    b = synth.gauss_source(12, lat.hv, 22)
    x = torch.empty_like(to_dev(b))
    B = qx.Batch([(g64, g32, to_dev(b), masses, x)], tol=1e-10, mode=qx.CG_MIXED_F32,
                 engine=qx.ENGINE_LAUNCH)
    B.set_launch(*shape)
    st = B.solve()
    _check_solution(dims, U, masses, b, to_host(x), st, flags=oracle.BC_T_ANTIPERIODIC)
    assert st[11].iters < st[0].iters
    # the same under the default shape: the same mathematics, rounding aside
    x2 = torch.empty_like(x)
    B2 = qx.Batch([(g64, g32, to_dev(b), masses, x2)], tol=1e-10, mode=qx.CG_MIXED_F32,
                  engine=qx.ENGINE_LAUNCH)
    B2.solve()
    assert rel(to_host(x), to_host(x2)) <= 1e-8


def test_uneven_batch_config4(qx):
    """8^4, 12^4, 16^4, 16^3x32, 24^4 weak fields, 4 sources each, one batch (graph replay)."""
    import torch

    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32), (24, 24, 24, 24)]
    mlist = [0.01, 0.05, 0.1]
    systems, keep = [], []
    for k, dims in enumerate(shapes):
        eps = float(np.random.Generator(np.random.PCG64(1000 + k)).uniform(0.2, 0.5))
        U = synth.weak_gauge(dims, eps, k)
        lat = qx.Lattice(dims)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64")
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        b = synth.gauss_source(4, lat.hv, 100 + k)
        masses = [mlist[(k + j) % 3] for j in range(4)]
        bd = to_dev(b)
        xd = torch.empty_like(bd)
        systems.append((g64, g32, bd, masses, xd))
        keep.append((dims, U, b, masses, xd, lat))
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    xs, all_stats = [], []
    with torch.cuda.stream(side):  # a non-default stream: the chunk is captured in a HIP graph
        batch = qx.Batch(systems, tol=1e-10, engine=qx.ENGINE_LAUNCH)
        for rep in range(2):
            all_stats.append(batch.solve())
            torch.cuda.synchronize()
            xs.append([to_host(k[4]).copy() for k in keep])
    torch.cuda.synchronize()
    # the same batch run eagerly on the default stream (no graph) gives the same bits
    all_stats.append(batch.solve())
    xs.append([to_host(k[4]).copy() for k in keep])
    for rep in (0, 1):
        for a, e in zip(xs[rep], xs[2]):
            assert np.array_equal(a, e)
    for stats in all_stats:
        j = 0
        for dims, U, b, masses, xd, lat in keep:
            x = to_host(xd)
            for s in range(4):
                rr = oracle.true_residual(dims, U, masses[s], b[s], x[s])
                assert rr <= 1e-10 and stats[j].status == 0, (dims, s, rr)
                j += 1


# ------------------------------------------------------------ failure modes

def test_cg_edge_cases(qx):
    import torch

    dims = (4, 4, 4, 4)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    g64 = qx.Gauge(lat, to_dev(U), "f64")
    g32 = qx.Gauge(lat, to_dev(U), "f32")
    b = synth.gauss_source(1, lat.hv, 1)
    # zero source: x = 0 at once
    x, st = qx.cg(g64, torch.zeros((1, lat.hv, 3), dtype=torch.complex128, device="cuda"), 0.1)
    assert st[0].status == 0 and st[0].iters == 0 and not to_host(x).any()
    # zero source with a nonzero initial guess still returns 0
    x, st = qx.cg(g64, torch.zeros((1, lat.hv, 3), dtype=torch.complex128, device="cuda"), 0.1,
                  x0=to_dev(b))
    assert st[0].status == 0 and not to_host(x).any()
    # max_iter = 1
    x, st = qx.cg(g64, to_dev(b), 0.1, max_iter=1, raise_on_fail=False)
    assert st[0].status == qx.ENOTCONVERGED and st[0].iters == 1
    # warm start from the solution: converged by the first residual check
    x1, _ = qx.cg(g64, to_dev(b), 0.1, tol=1e-10)
    x2, st = qx.cg(g64, to_dev(b), 0.1, tol=1e-10, x0=x1)
    assert st[0].status == 0 and st[0].iters == 0
    # NaN in the source
    bn = b.copy()
    bn[0, 3, 1] = np.nan
    x, st = qx.cg(g64, to_dev(bn), 0.1, raise_on_fail=False)
    assert st[0].status == qx.EBREAKDOWN
    x, st = qx.cg(g64, to_dev(bn), 0.1, glo=g32, raise_on_fail=False)
    assert st[0].status == qx.EBREAKDOWN
    # free field with m = 0 has exact zero modes: ends without converging, no hang
    gf = qx.Gauge(lat, to_dev(synth.unit_gauge(dims)), "f64")
    x, st = qx.cg(gf, to_dev(b), 0.0, max_iter=300, raise_on_fail=False)
    assert st[0].status in (qx.ENOTCONVERGED, qx.EBREAKDOWN)
    # workspace too small
    with pytest.raises(qx.QXError) as e:
        qx.cg(g64, to_dev(b), 0.1, ws=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.code in (qx.ENOMEM,)


def test_determinism(qx):
    dims = (8, 8, 8, 8)
    lat = qx.Lattice(dims)
    U = to_dev(gauge(dims, seed=2))
    g64 = qx.Gauge(lat, U, "f64")
    g32 = qx.Gauge(lat, U, "f32", 12)
    b = to_dev(synth.gauss_source(3, lat.hv, 7))
    xa, sa = qx.cg(g64, b, [0.05, 0.1, 0.2], glo=g32)
    xb, sb = qx.cg(g64, b, [0.05, 0.1, 0.2], glo=g32)
    assert np.array_equal(to_host(xa), to_host(xb))
    assert [s.iters for s in sa] == [s.iters for s in sb]


# --------------------------------------------------------------- a10 force

def test_force_config5(qx):
    """16^4 Haar, m = 0.1: GPU gradient (FP32 inner / FP64 reliable, 1e-10) against the
    oracle's FP64 gradient (CG to 1e-13)."""
    dims = (16, 16, 16, 16)
    m = 0.1
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    phi = synth.gauss_source(1, lat.hv, 1)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    S, G, x, st = qx.force(g64, to_dev(phi), m, glo=g32, tol=1e-10)
    So, Go, xo, sto = oracle.force(dims, U, m, phi[0], tol=1e-13)
    G = to_host(G)
    assert abs(S - So) <= 1e-9 * abs(So)
    assert rel(G, Go) <= 1e-7
    F = to_host(qx.force_su3(lat, Ud, to_dev(G)))
    Fo = oracle.su3_force(U, Go)
    assert rel(F, Fo) <= 1e-7


def _exp_i_T(a, e):
    """exp(i e T_a), T_a = lambda_a / 2 (Gell-Mann), by scipy's expm."""
    from scipy.linalg import expm

    return expm(1j * e * oracle.gell_mann()[a] / 2.0)


@pytest.mark.timeout(600)
def test_force_config5_finite_differences(qx):
    """Config 5's finite-difference leg at its stated size: 16^4 Haar links,
    m = 0.1, 64 links drawn without replacement (seed 5) x the 8 su(3)
    generators, central differences with h = 1e-5 along U -> exp(+-i h T_a) U.
    S(+h) - S(-h) is taken through the exact identity
    S+ - S- = x+^dag (A- - A+) x-, x+- = A+-^{-1} phi: the two solves are FP64
    GPU solves to 1e-13 warm-started from x, A+- is applied by the oracle.  The
    GPU force (FP32 12-real inner / FP64 reliable solve to 1e-10) must satisfy
    |F_FD - F| <= 1e-6 max|F| + 1e-7."""
    import torch

    dims = (16, 16, 16, 16)
    m, h = 0.1, 1e-5
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    phi = synth.gauss_source(1, lat.hv, 1)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    phid = to_dev(phi)
    S, G, x, st = qx.force(g64, phid, m, glo=g32, tol=1e-10)
    F = to_host(qx.force_su3(lat, Ud, G))
    fmax = np.abs(F).max()
    links = np.random.default_rng(5).choice(4 * lat.V, size=64, replace=False)
    worst = 0.0
    for n, l in enumerate(links):
        mu, site = divmod(int(l), lat.V)
        u0 = U[mu, site].copy()
        for a in range(8):
            up, um = _exp_i_T(a, h) @ u0, _exp_i_T(a, -h) @ u0
            xs = []
            for u in (up, um):
                Ud[mu, site] = torch.from_numpy(u).cuda()
                gp = qx.Gauge(lat, Ud, "f64")
                xs.append(to_host(qx.cg(gp, phid, m, tol=1e-13, x0=x)[0])[0])
                del gp
            Ud[mu, site] = torch.from_numpy(u0).cuda()
            U[mu, site] = um
            Am = oracle.apply_A(dims, U, m, xs[1])
            U[mu, site] = up
            Ap = oracle.apply_A(dims, U, m, xs[1])
            U[mu, site] = u0
            fd = np.vdot(xs[0], Am - Ap).real / (2 * h)
            err = abs(fd - F[mu, site, a])
            worst = max(worst, err)
            assert err <= 1e-6 * fmax + 1e-7, (mu, site, a, fd, F[mu, site, a])
        if n % 16 == 15:
            print(f"{n + 1} links done, worst |F_FD - F| = {worst:.2e} (max|F| {fmax:.2f})",
                  flush=True)


def test_force_from_fields_general(qx):
    dims = (4, 6, 4, 4)
    m = 0.3
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=8)
    g64 = qx.Gauge(lat, to_dev(U), "f64")
    x = synth.gauss_source(2, lat.hv, 1)
    lam = synth.gauss_source(2, lat.hv, 2)
    G = to_host(qx.force_from_fields(g64, to_dev(x), to_dev(lam)))
    Go = sum(oracle.force_from_fields(dims, U, x[k], lam[k], oracle.BC_T_ANTIPERIODIC)
             for k in range(2))
    assert rel(G, Go) <= 1e-13


def test_su3_force_projection(qx):
    dims = (4, 4, 4, 4)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=1)
    G = gauge(dims, seed=2) * 0.7 + 0.1j
    F = to_host(qx.force_su3(lat, to_dev(U), to_dev(G)))
    assert rel(F, oracle.su3_force(U, G)) <= 1e-14


def test_autograd_solve(qx):
    import torch

    dims = (4, 4, 4, 4)
    m = 0.2
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=3)
    b = synth.gauss_source(1, lat.hv, 4)
    w = synth.gauss_source(1, lat.hv, 5)
    Ut = to_dev(U).requires_grad_(True)
    bt = to_dev(b).requires_grad_(True)
    x = qx.StaggeredSolve.apply(Ut, bt, m, lat, 1e-12)
    loss = torch.real(torch.sum(to_dev(w).conj() * x))
    loss.backward()
    # oracle: L = Re<w, x>, so dL/dx = w, lam = A^-1 w
    xo, *_ = oracle.cg(dims, U, m, b[0], tol=1e-13)
    lo, *_ = oracle.cg(dims, U, m, w[0], tol=1e-13)
    Go = oracle.force_from_fields(dims, U, xo, lo)
    assert rel(to_host(Ut.grad), Go) <= 1e-9
    assert rel(to_host(bt.grad)[0], lo) <= 1e-9


def test_autograd_action(qx):
    dims = (4, 4, 4, 4)
    m = 0.2
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=3)
    phi = synth.gauss_source(1, lat.hv, 4)
    Ut = to_dev(U).requires_grad_(True)
    S = qx.staggered_action(Ut, to_dev(phi), m, lat, 1e-12)
    S.backward()
    So, Go, xo = oracle.force(dims, U, m, phi[0], tol=1e-13)[:3]
    assert abs(S.item() - So) <= 1e-10 * abs(So)
    assert rel(to_host(Ut.grad), Go) <= 1e-9
    # an upstream scale and the source gradient dL/dphi = 2 gS A^-1 phi
    Ut = to_dev(U).requires_grad_(True)
    pt = to_dev(phi).requires_grad_(True)
    (3.5 * qx.staggered_action(Ut, pt, m, lat, 1e-12)).backward()
    assert rel(to_host(Ut.grad), 3.5 * Go) <= 1e-9
    assert rel(to_host(pt.grad)[0], 7.0 * xo) <= 1e-9


# ------------------------------------------------------------------ engines

@pytest.mark.parametrize("dims", [(8, 4, 6, 8), (16, 16, 16, 36)])
@pytest.mark.parametrize("mixed", [False, True])
def test_engines_agree_bitwise(qx, mixed, dims):
    """The launch-per-pass engine, the fused launch sequence (reductions
    finished redundantly in every block, two state slots) and the persistent
    kernel (grid barriers) run the same reductions in the same order and
    update at the same iterations; AUTO is one of them or the two-launch
    sequence, bit for bit.  The second lattice has 1152 stencil blocks
    and 864 vector tiles per source, so the block-size-independent sums span
    several rounds of their 256 lanes, and AUTO picks the launch-per-pass
    engine there (more than 1024 blocks)."""
    dims = tuple(dims)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=9)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    glo = qx.Gauge(lat, Ud, "f32", 12) if mixed else None
    masses = [0.05, 0.2, 0.1]
    b = synth.gauss_source(3, lat.hv, 11)
    runs = [qx.cg(g64, to_dev(b), masses, glo=glo, engine=e)
            for e in (qx.ENGINE_LAUNCH, qx.ENGINE_FUSED, qx.ENGINE_PERSISTENT)]
    xa, sa = runs[0]
    for xb, sb in runs[1:]:
        assert np.array_equal(to_host(xa), to_host(xb))
        assert [s.iters for s in sa] == [s.iters for s in sb]
        assert [s.reliable_updates for s in sa] == [s.reliable_updates for s in sb]
    _check_solution(dims, U, masses, b, to_host(xa), sa, flags=oracle.BC_T_ANTIPERIODIC)
    # AUTO: the two-launch sequence for at most 3 sources while
    # 4 * sources * blocks <= 4096, the three-launch one up to 1024 blocks,
    # else launch-per-pass
    xauto, _ = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_AUTO)
    nblk = (lat.hv + 63) // 64
    if nblk <= 1024 and 4 * 3 * nblk <= 4096:
        xa = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED2)[0]
    assert np.array_equal(to_host(xauto), to_host(xa))


@pytest.mark.parametrize("engine", ["PERSISTENT", "FUSED", "LAUNCH", "FUSED2"])
def test_engine_edge_cases(qx, engine):
    """Zero source, max_iter, a non-finite source (breakdown), m = 0 on the free
    field (singular A), and a plain solve, under each engine."""
    import torch

    dims = (4, 4, 4, 4)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    g64 = qx.Gauge(lat, to_dev(U), "f64")
    g32 = qx.Gauge(lat, to_dev(U), "f32")
    b = synth.gauss_source(1, lat.hv, 1)
    P = getattr(qx, "ENGINE_" + engine)
    x, st = qx.cg(g64, torch.zeros((1, lat.hv, 3), dtype=torch.complex128, device="cuda"), 0.1,
                  engine=P)
    assert st[0].status == 0 and st[0].iters == 0 and not to_host(x).any()
    x, st = qx.cg(g64, to_dev(b), 0.1, max_iter=3, engine=P, raise_on_fail=False)
    assert st[0].status == qx.ENOTCONVERGED and st[0].iters == 3
    bn = b.copy()
    bn[0, 5, 2] = np.inf
    x, st = qx.cg(g64, to_dev(bn), 0.1, glo=g32, engine=P, raise_on_fail=False)
    assert st[0].status == qx.EBREAKDOWN
    gf = qx.Gauge(lat, to_dev(synth.unit_gauge(dims)), "f64")
    x, st = qx.cg(gf, to_dev(b), 0.0, max_iter=300, engine=P, raise_on_fail=False)
    assert st[0].status in (qx.ENOTCONVERGED, qx.EBREAKDOWN)
    x, st = qx.cg(g64, to_dev(b), 0.1, glo=g32, engine=P)
    _check_solution(dims, U, [0.1], b, to_host(x), st)


def test_engines_uneven_batch(qx):
    import torch

    shapes = [(4, 4, 4, 4), (8, 4, 4, 6), (6, 6, 6, 6), (8, 8, 8, 8)]
    systems, keep = [], []
    for k, dims in enumerate(shapes):
        U = synth.weak_gauge(dims, 0.3, 20 + k)
        lat = qx.Lattice(dims)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64")
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        nrhs = 1 + k % 3
        b = synth.gauss_source(nrhs, lat.hv, 40 + k)
        masses = [0.02 + 0.03 * j for j in range(nrhs)]
        bd = to_dev(b)
        xd = torch.empty_like(bd)
        systems.append((g64, g32, bd, masses, xd))
        keep.append((dims, U, b, masses, xd))
    for engine in (qx.ENGINE_PERSISTENT, qx.ENGINE_LAUNCH, qx.ENGINE_FUSED, qx.ENGINE_FUSED2):
        stats = qx.Batch(systems, tol=1e-10, engine=engine).solve()
        j = 0
        for dims, U, b, masses, xd in keep:
            x = to_host(xd)
            for s in range(b.shape[0]):
                rr = oracle.true_residual(dims, U, masses[s], b[s], x[s])
                assert rr <= 1e-10 and stats[j].status == 0, (engine, dims, s, rr)
                j += 1


@pytest.mark.parametrize("dims", [(8, 4, 6, 8), (16, 16, 16, 16)])
@pytest.mark.parametrize("mixed", [False, True])
def test_fused2_solves(qx, mixed, dims):
    """The two-launch sequence (|r|^2 from Re<r, Ap> and |Ap|^2): solutions to
    1e-10 measured by the oracle, iteration counts next to the three-launch
    sequence's, bitwise reproducible, and independent of the block order
    (partial sums stored at checkerboard-block positions)."""
    dims = tuple(dims)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=9)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    glo = qx.Gauge(lat, Ud, "f32", 12) if mixed else None
    masses = [0.05, 0.2, 0.1]
    b = synth.gauss_source(3, lat.hv, 11)
    x2, s2 = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED2)
    _check_solution(dims, U, masses, b, to_host(x2), s2, flags=oracle.BC_T_ANTIPERIODIC)
    x1, s1 = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED)
    for a, c in zip(s2, s1):
        assert abs(a.iters - c.iters) <= max(3, c.iters // 20), (a.iters, c.iters)
    x2b, _ = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED2)
    assert np.array_equal(to_host(x2), to_host(x2b))
    if glo is not None:
        glo.set_launch(3, 1, 4, 2)
        x2c, _ = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED2)
        glo.set_launch(3, 1, 4, 1)
        x2d, _ = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED2)
        assert np.array_equal(to_host(x2c), to_host(x2d))


def test_fused2_naik(qx):
    """The two-launch sequence on the improved operator, mixed and FP64."""
    dims = (8, 4, 6, 8)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    flags = oracle.NAIK | oracle.BC_T_ANTIPERIODIC
    U = gauge(dims, seed=35)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64", qx.RECON_NAIK)
    g32 = qx.Gauge(lat, Ud, "f32", qx.RECON_NAIK)
    masses = [0.05, 0.2, 0.1]
    b = synth.gauss_source(3, lat.hv, 36)
    for glo in (None, g32):
        x, st = qx.cg(g64, to_dev(b), masses, glo=glo, engine=qx.ENGINE_FUSED2)
        _check_solution(dims, U, masses, b, to_host(x), st, flags=flags)


# ------------------------------------------------------------ Naik term (f1)

NAIK_SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 8), (6, 4, 2, 8), (8, 8, 8, 12)]


@pytest.mark.parametrize("dims", NAIK_SHAPES)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_naik_dslash_parity(qx, dims, prec, tol):
    """Improved operator (one-hop x 9/8 and three-hop x -1/24) against the oracle, both
    parities and boundary conditions; extents 2 and 4 wrap the three-hop neighbours."""
    for anti in (False, True):
        lat = qx.Lattice(dims, antiperiodic_t=anti)
        flags = oracle.NAIK | (oracle.BC_T_ANTIPERIODIC if anti else 0)
        U = gauge(dims, seed=31)
        g = qx.Gauge(lat, to_dev(U), prec, qx.RECON_NAIK)
        for pout in (0, 1):
            chi = synth.gauss_source(2, lat.hv, 32 + pout)
            out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), pout, 2), 2,
                                    prec))
            for k in range(2):
                ref = oracle.dslash_eo(dims, U, chi[k], pout, flags)
                assert rel(out[k], ref) <= tol, (anti, pout, k)


@pytest.mark.parametrize("nbt,lps", SHAPES_NARROW)
def test_naik_launch_shapes(qx, nbt, lps):
    dims = (6, 4, 2, 8)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=33)
    nrhs = 5
    chi = synth.gauss_source(nrhs, lat.hv, 34)
    for prec, tol in (("f64", 1e-13), ("f32", 1e-5)):
        g = qx.Gauge(lat, to_dev(U), prec, qx.RECON_NAIK)
        g.set_launch(nrhs, nbt, lps, (nbt + lps) % 4)
        out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), 1, nrhs), nrhs,
                                prec))
        for k in range(nrhs):
            ref = oracle.dslash_eo(dims, U, chi[k], 1, oracle.NAIK | oracle.BC_T_ANTIPERIODIC)
            assert rel(out[k], ref) <= tol, (prec, nbt, lps, k)


def test_naik_dslash_32_4(qx):
    """Full-size lattice: FP64 and FP32 improved operator against the oracle."""
    dims = (32, 32, 32, 32)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    chi = synth.gauss_source(1, lat.hv, 1)
    ref = oracle.dslash_eo(dims, U, chi[0], 0, oracle.NAIK)
    for prec, tol in (("f64", 1e-13), ("f32", 1e-5)):
        g = qx.Gauge(lat, to_dev(U), prec, qx.RECON_NAIK)
        out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), 0, 1), 1, prec))
        assert rel(out[0], ref) <= tol


@pytest.mark.parametrize("mixed", [False, True])
def test_naik_cg_engines(qx, mixed):
    """CG on the improved operator to 1e-10 (oracle-measured), under every engine, with
    bitwise-identical results; three sources with different masses."""
    dims = (8, 4, 6, 8)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    flags = oracle.NAIK | oracle.BC_T_ANTIPERIODIC
    U = gauge(dims, seed=35)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64", qx.RECON_NAIK)
    glo = qx.Gauge(lat, Ud, "f32", qx.RECON_NAIK) if mixed else None
    masses = [0.05, 0.2, 0.1]
    b = synth.gauss_source(3, lat.hv, 36)
    runs = [qx.cg(g64, to_dev(b), masses, glo=glo, engine=e)
            for e in (qx.ENGINE_LAUNCH, qx.ENGINE_FUSED, qx.ENGINE_PERSISTENT)]
    xa, sa = runs[0]
    for xb, sb in runs[1:]:
        assert np.array_equal(to_host(xa), to_host(xb))
        assert [s.iters for s in sa] == [s.iters for s in sb]
    _check_solution(dims, U, masses, b, to_host(xa), sa, flags=flags)


def test_naik_apply_A_and_rejections(qx):
    dims = (4, 6, 4, 4)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=37)
    Ud = to_dev(U)
    gn = qx.Gauge(lat, Ud, "f64", qx.RECON_NAIK)
    v = synth.gauss_source(2, lat.hv, 38)
    out = to_host(qx.unpack(lat, qx.apply_A(gn, qx.pack(lat, to_dev(v), "f64"), [0.1, 0.3]), 2,
                            "f64"))
    for k, m in enumerate((0.1, 0.3)):
        assert rel(out[k], oracle.apply_A(dims, U, m, v[k], oracle.NAIK)) <= 1e-13
    # the force is implemented for the one-hop operator only
    with pytest.raises(qx.QXError):
        qx.force(gn, to_dev(v[:1]), 0.1)
    # mixed solves need both handles of the same operator
    g32 = qx.Gauge(lat, Ud, "f32", 18)
    with pytest.raises(qx.QXError):
        qx.cg(gn, to_dev(v[:1]), [0.1], glo=g32)


# ------------------------------------------------- HMC molecular dynamics (f3)

def _md_start(dims, seed):
    from oracle import hmc  # noqa: F401  (oracle package imported by the tests only)
    U = synth.weak_gauge(dims, 0.3, seed)
    p = np.random.default_rng(seed + 1).standard_normal((4, U.shape[1], 8))
    return U, p


def test_gauge_action_and_force_parity(qx):
    from oracle import hmc
    dims = (6, 4, 4, 8)
    lat = qx.Lattice(dims)
    U = synth.haar_gauge(dims, 41)
    beta = 5.6
    S = qx.gauge_action(lat, to_dev(U), beta)
    ref = hmc.gauge_action(dims, U, beta)
    assert abs(S - ref) <= 1e-13 * abs(ref)
    G = to_host(qx.gauge_force(lat, to_dev(U), beta))
    Gr = hmc.gauge_grad(dims, U, beta)
    assert np.abs(G - Gr).max() <= 1e-13 * np.abs(Gr).max()
    # accumulate onto a given gradient
    G0 = synth.haar_gauge(dims, 42)
    Ga = to_host(qx.gauge_force(lat, to_dev(U), beta, G=to_dev(G0), accumulate=True))
    assert np.abs(Ga - (G0 + Gr)).max() <= 1e-13 * np.abs(Gr).max()


def test_md_updates_parity(qx):
    from oracle import hmc
    dims = (4, 4, 6, 4)
    lat = qx.Lattice(dims)
    U, p = _md_start(dims, 43)
    G = synth.haar_gauge(dims, 44)
    pd = to_dev(p)
    qx.md_update_momenta(lat, to_dev(U), to_dev(G), 0.07, pd)
    assert np.abs(to_host(pd) - (p - 0.07 * oracle.su3_force(U, G))).max() <= 1e-13
    Ud = to_dev(U)
    big = 3.0 * p  # large steps exercise the scaling and squaring
    for eps in (0.05, 0.9):
        Ud = to_dev(U)
        qx.md_update_links(lat, to_dev(big), eps, Ud)
        assert np.abs(to_host(Ud) - hmc.link_update(U, big, eps)).max() <= 1e-13
    assert abs(qx.md_kinetic(lat, to_dev(p)) - hmc.kinetic(p)) <= 1e-12 * hmc.kinetic(p)


@pytest.mark.parametrize("fermions", [False, True])
def test_md_trajectory_parity(qx, fermions):
    """Four leapfrog steps (beta 5.5, m 0.2, eps 0.05) against the oracle trajectory:
    links, momenta and the energy change."""
    from oracle import hmc
    dims = (4, 4, 4, 8)
    lat = qx.Lattice(dims)
    U, p = _md_start(dims, 45)
    phi = synth.gauss_source(1, lat.hv, 46)[0] if fermions else None
    Ur, pr, H0r, H1r = hmc.md_trajectory(dims, U, p, phi, 5.5, 0.2, 0.05, 4, tol=1e-13)
    Ud, pd = to_dev(U), to_dev(p)
    g64 = qx.Gauge(lat, Ud, "f64")
    H0, H1, iters = qx.md_trajectory(g64, Ud, pd, 5.5, 0.05, 4,
                                     phi=to_dev(phi) if fermions else None, mass=0.2, tol=1e-12)
    assert abs(H0 - H0r) <= 1e-10 * abs(H0r)
    assert abs((H1 - H0) - (H1r - H0r)) <= 1e-7, (H1 - H0, H1r - H0r)
    assert np.abs(to_host(Ud) - Ur).max() <= 1e-10
    assert np.abs(to_host(pd) - pr).max() <= 1e-9
    assert (iters > 0) == fermions


def test_md_trajectory_mixed_reversible(qx):
    """Mixed-precision force solves: the same trajectory as with FP64 solves (both to
    1e-12), and run back with -p it returns to the start."""
    dims = (4, 4, 4, 8)
    lat = qx.Lattice(dims)
    U, p = _md_start(dims, 47)
    phi = to_dev(synth.gauss_source(1, lat.hv, 48)[0])
    Uf, pf = to_dev(U), to_dev(p)
    g64f = qx.Gauge(lat, Uf, "f64")
    F0, F1, _ = qx.md_trajectory(g64f, Uf, pf, 5.5, 0.05, 6, phi=phi, mass=0.2, tol=1e-12)
    Ud, pd = to_dev(U), to_dev(p)
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    H0, H1, _ = qx.md_trajectory(g64, Ud, pd, 5.5, 0.05, 6, phi=phi, mass=0.2, glo=g32, tol=1e-12)
    assert abs(H0 - F0) <= 1e-10 * abs(F0) and abs((H1 - H0) - (F1 - F0)) <= 1e-7
    assert np.abs(to_host(Ud) - to_host(Uf)).max() <= 1e-10
    pd.neg_()
    H2, H3, _ = qx.md_trajectory(g64, Ud, pd, 5.5, 0.05, 6, phi=phi, mass=0.2, glo=g32, tol=1e-12)
    assert np.abs(to_host(Ud) - U).max() <= 1e-9
    assert np.abs(-to_host(pd) - p).max() <= 1e-8
    assert abs(H3 - H0) <= 1e-9 * abs(H0)


# ------------------------------------------------------- meson correlators (f4)

@pytest.mark.parametrize("mixed", [False, True])
def test_meson_correlators_parity(qx, mixed):
    """Point-source correlators of six direction masks against the oracle."""
    from oracle import meson
    dims = (4, 6, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=61)
    src = (2, 1, 3, 2)
    masks = [0, 1, 2, 4, 8, 7, 15]
    ref = meson.correlators(dims, meson.point_propagator(dims, U, 0.15, src), src, masks)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    glo = qx.Gauge(lat, Ud, "f32", 12) if mixed else None
    C, st = qx.meson_correlators(g64, 0.15, src, masks, glo=glo, tol=1e-12)
    assert all(s.status == 0 for s in st)
    scale = np.abs(ref).max()
    assert np.abs(C - ref).max() <= 1e-9 * scale, np.abs(C - ref).max() / scale


def test_meson_rejects_odd_source(qx):
    dims = (4, 4, 4, 4)
    lat = qx.Lattice(dims)
    g64 = qx.Gauge(lat, to_dev(gauge(dims, seed=62)), "f64")
    with pytest.raises(qx.QXError):
        qx.meson_correlators(g64, 0.1, (1, 0, 0, 0))


def test_naik_uneven_batch(qx):
    """Improved-operator systems of different lattice sizes in one batch (mixed), to 1e-10."""
    import torch

    shapes = [(4, 4, 4, 4), (8, 4, 4, 6), (6, 6, 6, 6)]
    systems, keep = [], []
    for k, dims in enumerate(shapes):
        U = synth.weak_gauge(dims, 0.3, 70 + k)
        lat = qx.Lattice(dims)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64", qx.RECON_NAIK)
        g32 = qx.Gauge(lat, Ud, "f32", qx.RECON_NAIK)
        nrhs = 1 + k % 2
        b = synth.gauss_source(nrhs, lat.hv, 80 + k)
        masses = [0.05 + 0.04 * j for j in range(nrhs)]
        bd = to_dev(b)
        xd = torch.empty_like(bd)
        systems.append((g64, g32, bd, masses, xd))
        keep.append((dims, U, b, masses, xd))
    stats = qx.Batch(systems, tol=1e-10).solve()
    j = 0
    for dims, U, b, masses, xd in keep:
        x = to_host(xd)
        for s in range(b.shape[0]):
            rr = oracle.true_residual(dims, U, masses[s], b[s], x[s], oracle.NAIK)
            assert rr <= 1e-10 and stats[j].status == 0, (dims, s, rr)
            j += 1


def test_naik_meson_correlators(qx):
    from oracle import meson
    dims = (4, 4, 6, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=63)
    src = (0, 2, 2, 4)
    masks = [0, 8, 7]
    ref = meson.correlators(dims, meson.point_propagator(dims, U, 0.2, src, flags=oracle.NAIK), src,
                            masks)
    g64 = qx.Gauge(lat, to_dev(U), "f64", qx.RECON_NAIK)
    C, _ = qx.meson_correlators(g64, 0.2, src, masks, tol=1e-12)
    assert np.abs(C - ref).max() <= 1e-9 * np.abs(ref).max()
