"""The asynchronous batch solve (no host synchronisation, statistics written to
device memory) against the synchronous one: the same kernels in the same order,
so the same solutions bit for bit once enough chunks are enqueued; too few
chunks leave the sources reported as not converged."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu


def _systems(qx, torch):
    systems, keep = [], []
    for k, dims in enumerate([(8, 8, 8, 8), (8, 4, 6, 8)]):
        U = synth.weak_gauge(dims, 0.3, 60 + k)
        lat = qx.Lattice(dims)
        Ud = to_dev(U)
        g64 = qx.Gauge(lat, Ud, "f64")
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        b = synth.gauss_source(3, lat.hv, 62 + k)
        masses = [0.05, 0.1, 0.2]
        bd = to_dev(b)
        xd = torch.empty_like(bd)
        systems.append((g64, g32, bd, masses, xd))
        keep.append((dims, U, b, masses, xd))
    return systems, keep


@pytest.mark.parametrize("engine", ["FUSED", "LAUNCH", "PERSISTENT", "FUSED2"])
def test_batch_solve_async_matches_sync(qx, engine):
    import torch

    systems, keep = _systems(qx, torch)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        batch = qx.Batch(systems, tol=1e-10, engine=getattr(qx, "ENGINE_" + engine))
        ref_stats = batch.solve()
        torch.cuda.synchronize()
        ref_x = [to_host(k[4]).copy() for k in keep]
        chunk = batch.chunk()
        assert chunk >= 1
        if engine == "PERSISTENT":
            # a chunk of the persistent kernel also ends at every reliable update
            n_ok = sum(s.reliable_updates + 1 for s in ref_stats) + 3
        else:
            slots = max(s.iters for s in ref_stats) + 4 * max(s.reliable_updates for s in ref_stats)
            n_ok = slots // chunk + 3
        for k in keep:
            k[4].zero_()
        # two solves enqueued back to back, the first with too few chunks
        d_short = batch.solve_async(1)
        x_short = [k[4].clone() for k in keep]
        d_full = batch.solve_async(n_ok)
        torch.cuda.synchronize()
    short = batch.stats_from_device(d_short)
    full = batch.stats_from_device(d_full)
    if ref_stats[0].iters > chunk:
        assert all(s.status == qx.ENOTCONVERGED for s in short)
    for a in x_short:
        assert np.isfinite(to_host(a)).all()
    for k, r in zip(keep, ref_x):
        assert np.array_equal(to_host(k[4]), r)
    for a, b in zip(full, ref_stats):
        assert (a.status, a.iters, a.reliable_updates) == (b.status, b.iters, b.reliable_updates)
        assert a.true_rel_residual == b.true_rel_residual and a.seconds == 0.0
    j = 0
    for dims, U, b, masses, xd in keep:
        x = to_host(xd)
        for s in range(3):
            assert oracle.true_residual(dims, U, masses[s], b[s], x[s]) <= 1e-10
            assert full[j].status == qx.OK
            j += 1


def test_batch_solve_async_rejects(qx):
    import torch

    systems, _ = _systems(qx, torch)
    batch = qx.Batch(systems, tol=1e-10)
    with pytest.raises(qx.QXError):
        batch.solve_async(0)
    L = qx.load()
    assert L.qx_batch_solve_async(batch._h, 1, None, None) == qx.EINVAL
