"""Mixed solves whose inner iterations load FP16 links (binary16, converted to
FP32 as loaded; vectors and arithmetic FP32; FP64 reliable updates and final
residual), against the FP64 oracle.

Bar: the oracle's FP64 true relative residual of the returned x at most the
requested 1e-10, as for every mixed solve: the FP64 reliable updates correct
what the coarser inner operator (about 5e-4 relative per link element) leaves,
so only the iteration count may differ from the FP32-link solve.  The engines
run the same reductions in the same order whatever the link storage, so the
launch-per-pass, three-launch fused and persistent engines agree bit for bit
here too.
"""
import numpy as np
import pytest

import oracle
from gpu_util import gauge, rel, to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu

ENGINES = ["LAUNCH", "FUSED", "FUSED2", "PERSISTENT", "AUTO"]


def _check(dims, U, masses, b, x, stats, flags=0, tol=1e-10):
    for k in range(b.shape[0]):
        rr = oracle.true_residual(dims, U, masses[k], b[k], x[k], flags)
        assert rr <= tol, (k, rr, stats[k])
        assert stats[k].status == 0
        assert abs(stats[k].true_rel_residual - rr) <= 1e-12
        assert stats[k].reliable_updates >= 1


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("recon", [18, 12, 36])
def test_cg_f16_links_engines(qx, engine, recon):
    """Three sources of different masses on a ragged antiperiodic lattice
    (V/2 = 384: six stencil blocks, the last one full; 18 vector tiles)."""
    dims = (8, 4, 6, 4)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    naik = recon == 36
    U = gauge(dims, "weak" if naik else "haar", seed=70)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64", 36 if naik else 18)
    g16 = qx.Gauge(lat, Ud, "f16", recon)
    masses = [0.05, 0.2, 0.1]
    b = synth.gauss_source(3, lat.hv, 71)
    x, st = qx.cg(g64, to_dev(b), masses, glo=g16, engine=getattr(qx, "ENGINE_" + engine))
    flags = oracle.BC_T_ANTIPERIODIC | (oracle.NAIK if naik else 0)
    _check(dims, U, masses, b, to_host(x), st, flags)


def _round16(U):
    """The values an FP16 link holds: each real and imaginary part rounded once
    from FP64 to binary16, to nearest with ties to even (numpy's conversion)."""
    h = lambda a: a.astype(np.float16).astype(np.float64)
    return h(U.real) + 1j * h(U.imag)


@pytest.mark.parametrize("engine", ["LAUNCH", "FUSED2", "PERSISTENT"])
def test_f16_links_equal_fp32_links_of_rounded_field(qx, engine):
    """A solve with FP16 18-real inner links is, bit for bit, the solve with
    FP32 inner links packed from the binary16-rounded field (same launch
    shape): the links are converted exactly to FP32 as they are loaded and
    every later step is shared.  What FP16 links change is the inner operator
    itself, not the solver."""
    dims = (8, 4, 6, 4)
    lat = qx.Lattice(dims, antiperiodic_t=True)
    U = gauge(dims, seed=80)
    g64 = qx.Gauge(lat, to_dev(U), "f64")
    g16 = qx.Gauge(lat, to_dev(U), "f16", 18)
    g32r = qx.Gauge(lat, to_dev(_round16(U)), "f32", 18)
    for g in (g16, g32r):
        g.set_launch(3, 1, 2, 1)
    masses = [0.05, 0.2, 0.1]
    b = synth.gauss_source(3, lat.hv, 81)
    e = getattr(qx, "ENGINE_" + engine)
    xa, sa = qx.cg(g64, to_dev(b), masses, glo=g16, engine=e)
    xb, sb = qx.cg(g64, to_dev(b), masses, glo=g32r, engine=e)
    assert np.array_equal(to_host(xa), to_host(xb))
    assert [(s.iters, s.reliable_updates) for s in sa] == [(s.iters, s.reliable_updates) for s in sb]
    _check(dims, U, masses, b, to_host(xa), sa, oracle.BC_T_ANTIPERIODIC)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 2, 10)])
def test_cg_f16_links_engines_bitwise(qx, dims):
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=72)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    masses = [0.1, 0.03]
    b = synth.gauss_source(2, lat.hv, 73)
    runs = [qx.cg(g64, to_dev(b), masses, glo=g16, engine=e)
            for e in (qx.ENGINE_LAUNCH, qx.ENGINE_FUSED, qx.ENGINE_PERSISTENT)]
    xa, sa = runs[0]
    for xb, sb in runs[1:]:
        assert np.array_equal(to_host(xa), to_host(xb))
        assert [s.iters for s in sa] == [s.iters for s in sb]
        assert [s.reliable_updates for s in sa] == [s.reliable_updates for s in sb]
    _check(dims, U, masses, b, to_host(xa), sa)


def test_cg_f16_links_16_4(qx):
    """16^4 Haar links, m = 0.1, one source, AUTO engine: converges to 1e-10
    in at most 1.5 times the FP32-link iterations."""
    dims = (16, 16, 16, 16)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=0)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    b = synth.gauss_source(1, lat.hv, 1)
    x16, s16 = qx.cg(g64, to_dev(b), [0.1], glo=qx.Gauge(lat, Ud, "f16", 12))
    x32, s32 = qx.cg(g64, to_dev(b), [0.1], glo=qx.Gauge(lat, Ud, "f32", 12))
    _check(dims, U, [0.1], b, to_host(x16), s16)
    assert s16[0].iters <= 1.5 * s32[0].iters, (s16[0].iters, s32[0].iters)
    # both are solutions of the same system to 1e-10
    assert rel(to_host(x16), to_host(x32)) <= 1e-8


def test_batch_f16_links_uneven(qx):
    """Two lattices of different size in one batch, FP16 inner links; a batch
    that mixes FP16 and FP32 inner links is rejected."""
    import torch

    systems, keep = [], []
    for k, dims in enumerate([(4, 4, 4, 4), (8, 4, 6, 8)]):
        lat = qx.Lattice(dims)
        U = gauge(dims, seed=74 + k)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64")
        g16 = qx.Gauge(lat, Ud, "f16", 12)
        b = synth.gauss_source(2, lat.hv, 76 + k)
        masses = [0.1, 0.05]
        xd = torch.empty_like(to_dev(b))
        systems.append((g64, g16, to_dev(b), masses, xd))
        keep.append((dims, U, b, masses, xd, lat, Ud))
    for engine in ("LAUNCH", "FUSED", "FUSED2"):
        batch = qx.Batch(systems, tol=1e-10, engine=getattr(qx, "ENGINE_" + engine))
        stats = batch.solve()
        j = 0
        for dims, U, b, masses, xd, _, _ in keep:
            _check(dims, U, masses, b, to_host(xd), stats[j:j + 2])
            j += 2
    dims, U, b, masses, xd, lat, Ud = keep[1]
    mixed = [systems[0], (systems[1][0], qx.Gauge(lat, Ud, "f32", 12)) + systems[1][2:]]
    with pytest.raises(qx.QXError) as e:
        qx.Batch(mixed, tol=1e-10)
    assert e.value.code == qx.EINVAL


def test_force_f16_links(qx):
    """The fermion force with FP16 inner links against the oracle's FP64 force."""
    dims = (4, 6, 4, 8)
    m = 0.1
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=78)
    phi = synth.gauss_source(1, lat.hv, 79)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    S, G, x, st = qx.force(g64, to_dev(phi), m, glo=qx.Gauge(lat, Ud, "f16", 12), tol=1e-10)
    So, Go, xo, sto = oracle.force(dims, U, m, phi[0], tol=1e-13)
    assert abs(S - So) <= 1e-9 * abs(So)
    assert rel(to_host(G), Go) <= 1e-7


def test_mesons_f16_links(qx):
    from oracle import meson

    dims = (4, 6, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, seed=61)
    src = (2, 1, 3, 2)
    masks = [0, 1, 2, 4, 8, 7, 15]
    ref = meson.correlators(dims, meson.point_propagator(dims, U, 0.15, src), src, masks)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64")
    C, st = qx.meson_correlators(g64, 0.15, src, masks, glo=qx.Gauge(lat, Ud, "f16", 12),
                                 tol=1e-12)
    assert all(s.status == 0 for s in st)
    scale = np.abs(ref).max()
    assert np.abs(C - ref).max() <= 1e-9 * scale


def test_md_trajectory_f16_links(qx):
    """Molecular dynamics with FP16 inner links in the force solves (the FP16
    handle repacked from U after every link update): the trajectory of FP64
    force solves (both to 1e-12), and back to the start under -p."""
    dims = (4, 4, 4, 8)
    lat = qx.Lattice(dims)
    U = gauge(dims, "weak", seed=82, eps=0.2)
    rng = np.random.default_rng(83)
    p = rng.standard_normal((4, lat.V, 8))
    phi = to_dev(synth.gauss_source(1, lat.hv, 84)[0])
    Uf, pf = to_dev(U), to_dev(p)
    F0, F1, _ = qx.md_trajectory(qx.Gauge(lat, Uf, "f64"), Uf, pf, 5.5, 0.05, 6, phi=phi,
                                 mass=0.2, tol=1e-12)
    Ud, pd = to_dev(U), to_dev(p)
    g64 = qx.Gauge(lat, Ud, "f64")
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    H0, H1, iters = qx.md_trajectory(g64, Ud, pd, 5.5, 0.05, 6, phi=phi, mass=0.2, glo=g16,
                                     tol=1e-12)
    assert iters > 0
    assert abs(H0 - F0) <= 1e-10 * abs(F0) and abs((H1 - H0) - (F1 - F0)) <= 1e-7
    assert np.abs(to_host(Ud) - to_host(Uf)).max() <= 1e-10
    pd.neg_()
    H2, H3, _ = qx.md_trajectory(g64, Ud, pd, 5.5, 0.05, 6, phi=phi, mass=0.2, glo=g16, tol=1e-12)
    assert np.abs(to_host(Ud) - U).max() <= 1e-9
    assert np.abs(-to_host(pd) - p).max() <= 1e-8
    assert abs(H3 - H0) <= 1e-9 * abs(H0)
