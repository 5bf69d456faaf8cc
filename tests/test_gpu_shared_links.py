"""Links shared through LDS by the source groups of a block (one wavefront
per site and two or more groups of sources per block): the staged links are
the same values as the ones a wavefront loads itself, so

  * the standalone half-Dslash gives each of several sources the bits that
    source gets alone (one group, links loaded by the wavefront), and the
    oracle's values within the precision's bound;
  * the launch-per-pass engine, whose D_oe and D_eo passes share the links,
    agrees bit for bit with the fused and persistent engines, whose passes do
    not, under the same launch shape, and solves to the oracle's 1e-10.

The lattices leave a ragged last tile (V/2 = 288: lanes past the lattice
take part in staging with a clamped site)."""
import numpy as np
import pytest

import oracle
from gpu_util import gauge, rel, to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 4, 6)


# FP32-12 (24 KB per tile), FP32-18 (40 KB), FP64-12 (48 KB); FP64-18 (72 KB)
# is not staged and is the control
@pytest.mark.parametrize("prec,recon,tol", [("f32", 12, 1e-5), ("f32", 18, 1e-5),
                                            ("f64", 12, 1e-13), ("f64", 18, 1e-13)])
@pytest.mark.parametrize("nbt", [1, 2])
def test_dslash_shared_links_bitwise(qx, prec, recon, tol, nbt):
    lat = qx.Lattice(DIMS, antiperiodic_t=True)
    U = gauge(DIMS, seed=31)
    g = qx.Gauge(lat, to_dev(U), prec, recon)
    n = 5  # five or three groups, the last one partly filled
    chi = synth.gauss_source(n, lat.hv, 32)
    g.set_launch(n, nbt, 1, 0)
    g.set_launch(1, 1, 1, 0)
    for parity in (0, 1):
        out = to_host(qx.unpack(lat, qx.dslash(g, qx.pack(lat, to_dev(chi), prec), parity, n), n,
                                prec))
        for k in range(n):
            one = qx.pack(lat, to_dev(chi[k:k + 1]), prec)
            alone = to_host(qx.unpack(lat, qx.dslash(g, one, parity, 1), 1, prec))[0]
            assert np.array_equal(out[k], alone), (parity, k)
        ref = oracle.dslash_eo(DIMS, U, chi[n - 1], parity, oracle.BC_T_ANTIPERIODIC)
        assert rel(out[n - 1], ref) <= tol


@pytest.mark.parametrize("inner", ["f32", "f16", None])
def test_engines_shared_links_bitwise(qx, inner):
    """Six sources under (2, 1, 0): three groups of two sources per block.
    FP64 links in 12 reals (staged) for the FP64 solve and the reliable
    updates; FP32 or FP16 12-real inner links."""
    lat = qx.Lattice(DIMS, antiperiodic_t=True)
    U = gauge(DIMS, seed=41)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64", 12)
    glo = qx.Gauge(lat, Ud, inner, 12) if inner else None
    n = 6
    masses = [0.05, 0.1, 0.2, 0.05, 0.3, 0.15]
    b = synth.gauss_source(n, lat.hv, 42)
    (glo if glo is not None else g64).set_launch(n, 2, 1, 0)
    runs = [qx.cg(g64, to_dev(b), masses, glo=glo, engine=e)
            for e in (qx.ENGINE_LAUNCH, qx.ENGINE_FUSED, qx.ENGINE_PERSISTENT)]
    xa, sa = runs[0]
    for xb, sb in runs[1:]:
        assert np.array_equal(to_host(xa), to_host(xb))
        assert [s.iters for s in sa] == [s.iters for s in sb]
        assert [s.reliable_updates for s in sa] == [s.reliable_updates for s in sb]
    x = to_host(xa)
    for k in range(n):
        rr = oracle.true_residual(DIMS, U, masses[k], b[k], x[k], oracle.BC_T_ANTIPERIODIC)
        assert rr <= 1e-10 and sa[k].status == 0, (k, rr)


def test_uneven_batch_shared_links_bitwise(qx):
    """Two lattices of 5 and 2 sources in one batch under (2, 1, 0): every
    block has three source groups, so in the smaller system's blocks two
    groups have no source and still stage their share of the links.  The
    launch-per-pass engine (shared links) and the persistent engine (not
    shared) give the same bits, and every source meets the oracle's 1e-10."""
    import torch

    specs = [((6, 4, 4, 6), 5), ((4, 4, 4, 6), 2)]
    systems, keep = [], []
    for k, (dims, n) in enumerate(specs):
        lat = qx.Lattice(dims, antiperiodic_t=True)
        U = gauge(dims, seed=51 + k)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64", 12)
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        b = synth.gauss_source(n, lat.hv, 61 + k)
        masses = [0.05 + 0.04 * j for j in range(n)]
        systems.append([g64, g32, to_dev(b), masses, None])
        keep.append((dims, U, b, masses))
    # the batch takes its shape from the first system's inner links
    systems[0][1].set_launch(5, 2, 1, 0)
    runs = []
    for engine in (qx.ENGINE_LAUNCH, qx.ENGINE_PERSISTENT):
        for s in systems:
            s[4] = torch.zeros_like(s[2])
        B = qx.Batch([tuple(s) for s in systems], tol=1e-10, engine=engine)
        assert B.launch()[0][:2] == (2, 1)
        st = B.solve()
        torch.cuda.synchronize()
        runs.append(([to_host(s[4]) for s in systems], st))
    (xa, sa), (xb, sb) = runs
    for a, b in zip(xa, xb):
        assert np.array_equal(a, b)
    assert [s.iters for s in sa] == [s.iters for s in sb]
    j = 0
    for (dims, U, b, masses), x in zip(keep, xa):
        for k in range(b.shape[0]):
            rr = oracle.true_residual(dims, U, masses[k], b[k], x[k], oracle.BC_T_ANTIPERIODIC)
            assert rr <= 1e-10 and sa[j].status == 0, (dims, k, rr)
            j += 1
