"""The batch launch-shape tuner: it times chunks of the solve under every
admissible shape, keeps the fastest, leaves the systems' x untouched, and the
tuned batch solves to 1e-10 (oracle) with the same bits as a batch planned
with that shape from the handle."""
import numpy as np
import pytest

import oracle
from gpu_util import gauge, to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu


def _systems(qx, torch, specs):
    systems, keep = [], []
    for k, (dims, nsrc) in enumerate(specs):
        lat = qx.Lattice(dims, antiperiodic_t=True)
        U = gauge(dims, seed=90 + k)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64")
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        b = synth.gauss_source(nsrc, lat.hv, 95 + k)
        masses = [0.05 + 0.05 * j for j in range(nsrc)]
        xd = torch.zeros_like(to_dev(b))
        systems.append((g64, g32, to_dev(b), masses, xd))
        keep.append((dims, U, b, masses, xd))
    return systems, keep


def _check(keep, stats):
    j = 0
    for dims, U, b, masses, xd in keep:
        x = to_host(xd)
        for k in range(b.shape[0]):
            rr = oracle.true_residual(dims, U, masses[k], b[k], x[k], oracle.BC_T_ANTIPERIODIC)
            assert rr <= 1e-10 and stats[j].status == 0, (dims, k, rr)
            j += 1


@pytest.mark.parametrize("engine,stream", [("AUTO", True), ("LAUNCH", False), ("FUSED2", True)])
def test_batch_tune(qx, engine, stream):
    import torch

    specs = [((8, 8, 8, 8), 2), ((6, 4, 4, 8), 3)]
    systems, keep = _systems(qx, torch, specs)
    side = torch.cuda.Stream() if stream else torch.cuda.current_stream()
    with torch.cuda.stream(side):
        B = qx.Batch(systems, tol=1e-10, engine=getattr(qx, "ENGINE_" + engine))
        nbt, lps, order = B.tune(2)
        torch.cuda.synchronize()
        # small systems run the fused sequences, which take at most four sources per thread
        assert nbt in (1, 2, 4) and lps in (1, 2, 4, 8) and order in range(6)
        assert lps > 1  # batches of at most 1024 blocks per system split the hops
        shape, deo = B.launch()
        assert shape == (nbt, lps, order)
        # only the launch-per-pass engine runs its D_eo pass under a shape of its own
        if engine != "LAUNCH":
            assert deo == (nbt, lps)
        assert deo[0] in (1, 2, 4) and deo[1] > 1
        for k in keep:
            assert not to_host(k[4]).any()  # tuning writes no solution
        st = B.solve()
        torch.cuda.synchronize()
        _check(keep, st)
        tuned = [to_host(k[4]).copy() for k in keep]
        # the same shape set on the first system's handle gives the same bits
        systems[0][1].set_launch(3, nbt, lps, order)
        for k in keep:
            k[4].zero_()
        B2 = qx.Batch(systems, tol=1e-10, engine=getattr(qx, "ENGINE_" + engine))
        if deo != (nbt, lps):
            B2.set_deo_launch(*deo)
        # (the plan may take another block order, which changes no bits)
        assert B2.launch()[0][:2] == shape[:2] and B2.launch()[1] == deo
        st2 = B2.solve()
        torch.cuda.synchronize()
    for k, t in zip(keep, tuned):
        assert np.array_equal(to_host(k[4]), t)
    assert [s.iters for s in st] == [s.iters for s in st2]


def test_batch_deo_launch(qx):
    """qx_batch_set_deo_launch: the launch-per-pass engine's D_eo pass under a
    shape of its own solves to the oracle's 1e-10, qx_batch_get_launch reports
    it, qx_batch_set_launch resets it; other engines and unavailable shapes
    are refused."""
    import torch

    systems, keep = _systems(qx, torch, [((8, 4, 6, 8), 3)])
    B = qx.Batch(systems, tol=1e-10, mode=qx.CG_MIXED_F32, engine=qx.ENGINE_LAUNCH)
    B.set_launch(1, 2, 1)
    B.set_deo_launch(4, 1)
    assert B.launch() == ((1, 2, 1), (4, 1))
    st = B.solve()
    torch.cuda.synchronize()
    _check(keep, st)
    B.set_launch(2, 2, 0)
    assert B.launch() == ((2, 2, 0), (2, 2))
    with pytest.raises(qx.QXError) as e:
        B.set_deo_launch(3, 1)
    assert e.value.code == qx.EINVAL
    F = qx.Batch(systems, tol=1e-10, engine=qx.ENGINE_FUSED2)
    with pytest.raises(qx.QXError) as e:
        F.set_deo_launch(1, 2)
    assert e.value.code == qx.EINVAL
    L = qx.load()
    assert L.qx_batch_get_launch(None, None, None, None, None, None) == qx.EINVAL
    assert L.qx_batch_set_deo_launch(None, 1, 2, None) == qx.EINVAL


def test_batch_tune_rejects(qx):
    import torch

    systems, _ = _systems(qx, torch, [((4, 4, 4, 4), 1)])
    B = qx.Batch(systems, tol=1e-10)
    for n in (0, 65):
        with pytest.raises(qx.QXError) as e:
            B.tune(n)
        assert e.value.code == qx.EINVAL
    P = qx.Batch(systems, tol=1e-10, engine=qx.ENGINE_PERSISTENT)
    with pytest.raises(qx.QXError) as e:
        P.tune(1)
    assert e.value.code == qx.EINVAL
    L = qx.load()
    assert L.qx_batch_tune(None, 1, None, None, None, None) == qx.EINVAL
    # the batch still solves after a rejected call
    st = B.solve()
    assert st[0].status == 0


@pytest.mark.parametrize("engine_name", ["ENGINE_LAUNCH", "ENGINE_FUSED", "ENGINE_FUSED2"])
def test_batch_profile_and_set_launch(qx, engine_name):
    """qx_batch_profile: event-timed chunks of the solve, pass by pass.  Every
    iteration slot launches one D_oe and one D_eo pass; under the
    launch-per-pass engine each source served by a D_eo launch is one
    iteration of that source, so the served-source count equals the summed
    iteration counts; the profile leaves x untouched.  qx_batch_set_launch
    then fixes a shape and the solve stays oracle-correct."""
    import torch

    systems, keep = _systems(qx, torch, [((8, 4, 6, 8), 3)])
    engine = getattr(qx, engine_name)
    B = qx.Batch(systems, tol=1e-10, mode=qx.CG_MIXED_F32, engine=engine)
    chunk = B.chunk()
    passes, st = B.profile(2)
    assert passes["doe"]["launches"] == 2 * chunk
    assert passes["deo"]["launches"] == 2 * chunk
    for name, q in passes.items():
        assert 0 <= q["active_launches"] <= q["launches"]
        assert q["ms"] >= q["active_ms"] >= 0.0
        if q["active_launches"]:
            assert q["active_ms"] > 0.0
    if engine_name == "ENGINE_LAUNCH":
        assert passes["deo"]["source_launches"] == sum(s.iters for s in st)
        assert passes["p"]["launches"] == 2 * chunk and passes["xr"]["launches"] == 2 * chunk
    assert all(s.iters > 0 for s in st)
    assert not to_host(systems[0][4]).any()  # x untouched
    B.set_launch(2, 2, 1)
    st = B.solve()
    _check(keep, st)
    with pytest.raises(qx.QXError):
        B.set_launch(3, 2, 1)
