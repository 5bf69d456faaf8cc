"""A seeded sweep over small ragged problems: lattice extents from {2, 4, 6, 8}
(V/2 from 8 to 2048, ragged against the 64-site tiles), 1 to 4 sources with
their own masses, every engine, FP64 and mixed solves (the mixed ones of
seeds 30 to 39 with FP16 inner links), 12-real, 18-real and
improved-operator links, periodic and antiperiodic time.  Every solution must
reach a true relative residual of 1e-10 measured by the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import to_dev, to_host
from paper_1612_02750_amd import synth

pytestmark = pytest.mark.gpu

ENGINES = ["AUTO", "LAUNCH", "FUSED", "FUSED2", "PERSISTENT"]


def _case(seed):
    rng = np.random.Generator(np.random.PCG64(500 + seed))
    dims = tuple(int(v) for v in rng.choice([2, 4, 6, 8], size=4))
    nsrc = int(rng.integers(1, 5))
    masses = [float(v) for v in rng.uniform(0.05, 0.5, size=nsrc)]
    engine = ENGINES[seed % len(ENGINES)]
    mixed = bool(seed % 2)
    recon = [12, 18, 36][seed % 3] if mixed else [18, 36][(seed // 3) % 2]
    anti = bool((seed // 2) % 2)
    lo = "f16" if seed >= 30 else "f32"
    return dims, nsrc, masses, engine, mixed, recon, anti, lo


@pytest.mark.parametrize("seed", range(40))
def test_sweep(qx, seed):
    dims, nsrc, masses, engine, mixed, recon, anti, lo = _case(seed)
    lat = qx.Lattice(dims, antiperiodic_t=anti)
    flags = (oracle.BC_T_ANTIPERIODIC if anti else 0) | (oracle.NAIK if recon == 36 else 0)
    U = synth.haar_gauge(dims, 600 + seed)
    Ud = to_dev(U)
    g64 = qx.Gauge(lat, Ud, "f64", 36 if recon == 36 else 18)
    glo = qx.Gauge(lat, Ud, lo, recon) if mixed else None
    b = synth.gauss_source(nsrc, lat.hv, 700 + seed)
    x, st = qx.cg(g64, to_dev(b), masses, glo=glo, tol=1e-10,
                  engine=getattr(qx, "ENGINE_" + engine))
    x = to_host(x)
    for k in range(nsrc):
        rr = oracle.true_residual(dims, U, masses[k], b[k], x[k], flags)
        assert st[k].status == qx.OK and rr <= 1e-10, (dims, nsrc, engine, mixed, recon, anti, lo,
                                                       k, rr)
