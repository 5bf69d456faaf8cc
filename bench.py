"""Benchmark: staggered Dslash + even-odd CG on one MI355X.

Workload (one step): a full mixed-precision solve of (m^2 - D_eo D_oe) x = b to
a true FP64 relative residual of 1e-10 on a 16^4 lattice with weak-field links
U = exp(0.3 i H) (seed 0), one Gaussian source (seed 1), m = 0.05, FP32 inner
iteration on 12-real links, FP64 reliable updates when |r| drops below
0.1 max|r|.  Inputs are resident in HBM before the timed region; the step
includes packing b, every inner iteration and reliable update, and unpacking x.

Reported beside it (same run):
  * the same solve in plain FP64 (time-to-solution, mixed vs FP64);
  * the dominant kernel (the FP32 half-Dslash) timed alone, launches replayed
    from a HIP graph between HIP events on their stream, against the HBM
    roofline;
  * the half-Dslash on 32^4 (the size where links no longer fit the 256 MB
    Infinity Cache) and 48^4 in FP32-12, FP64-18 and FP16-12 (per-site
    scaled vectors), one and twelve sources;
  * the measured bandwidth of a plain copy kernel;
  * 32^4 with twelve sources (Haar links, m = 0.02): one mixed batch against
    plain FP64 solves one after another and an FP64 batch, the same batch with
    FP16 inner links, and its first source alone with FP32 and FP16 inner
    links; a 32^4 weak-field solve with FP32 and FP16 inner links; the 16^4
    step with FP16 inner links;
  * the improved operator (Naik term): Dslash at 32^4 / 48^4 and a 16^4 CG;
  * one HMC molecular-dynamics trajectory on 16^4 and point-source meson
    correlators on 16^3 x 32;
  * the uneven batch (8^4 ... 24^4, four sources each) replayed as one graph
    against its systems solved one at a time, and the 16^4 fermion force;
  * the CPU oracle (FP64 CG on the host cores) on the same system, whole
    solves repeated for about 10 s.

Flop convention: 570 flops per output site per half-Dslash; one CG iteration
costs 606 V (two half-Dslash + BLAS-1), one reliable update 570 V + 12 V.

    python bench.py [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FLOPS_SITE = 570
FLOPS_SITE_NAIK = 1146  # 16 SU(3) x colour-vector products + 15 vector sums


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the 32^4 twelve-source comparison")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the dominant-kernel timing and the copy probe (for counter runs)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_kernel(torch, fn, reps):
    """Average duration of fn() (one launch) from HIP events on the current stream."""
    s = torch.cuda.current_stream()
    for _ in range(5):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3  # seconds per launch


BYTES_SITE_F32_12 = 432  # 8 FP32 12-real links + one input and one output colour vector

# HBM-side bytes per launch of the dominant kernel from two rocprofv3 counter
# runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the same
# counters read for the library's copy kernel on 1 GiB (FETCH x 2.000, WRITE
# x 1.000).  Reported only while the kernel sources and the launch shape are
# the ones the counters were taken with.
# From profiles/dslash_16x16x16x16_to_48x48x48x48_counters.md; keyed by
# launch shape "nbt,lps,order".
TRAFFIC = {
    "sha": "35f119f62d191bfe",
    "bytes": {
        "1,1,0": 16248832,
        "1,1,1": 15069184,
        "1,1,2": 14880768,
        "1,1,3": 14880768,
        "1,2,0": 16277504,
        "1,2,1": 15097856,
        "1,2,2": 14901248,
        "1,2,3": 14901248,
        "1,4,0": 16254976,
        "1,4,1": 15075328,
        "1,4,2": 14886912,
        "1,4,3": 14886912,
        "1,8,0": 16287744,
        "1,8,1": 15108096,
        "1,8,2": 14911488,
        "1,8,3": 14911488
    },
}
KERNEL_SOURCES = ("qx_dslash.hip", "qx_device.h", "qx_internal.h", "qx_launch.h", "qx_dispatch.h")


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1612_02750_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def dominant_kernel(torch, qx, lat, g32, bd, reps, plain=False):
    """The FP32 12-real half-Dslash on the workload lattice, timed alone
    (plain=True: a few ordinary launches for a counter run, not timed)."""
    p32 = qx.pack(lat, bd, "f32")
    o32 = qx.dslash(g32, p32, 0, 1)
    if plain:
        for _ in range(reps):
            qx.dslash(g32, p32, 0, 1, out=o32)
        torch.cuda.synchronize()
        return None, None
    t_k = qx.time_dslash(g32, p32, 0, 1, out=o32, reps=reps)
    achieved = BYTES_SITE_F32_12 * lat.hv / t_k / 1e9
    log(f"dominant kernel (FP32-12 half-Dslash, {lat.dims}): {t_k * 1e6:.2f} us, "
        f"{achieved:.0f} GB/s algorithmic, {FLOPS_SITE * lat.hv / t_k / 1e9:.0f} GFLOP/s")
    return t_k, achieved


def launch_floor(torch, qx, synth, reps):
    """Per-launch time of the same kernel on a 2^4 lattice (8 output sites,
    one block) with the same graph-replayed timer: the dispatch-to-dispatch
    floor that every launch pays, whatever its work."""
    dims = (2, 2, 2, 2)
    lat = qx.Lattice(dims)
    g = qx.Gauge(lat, torch.from_numpy(synth.haar_gauge(dims, 0)).cuda(), "f32", 12)
    pin = qx.pack(lat, torch.from_numpy(synth.gauss_source(1, lat.hv, 1)).cuda(), "f32")
    out = qx.dslash(g, pin, 0, 1)
    t = qx.time_dslash(g, pin, 0, 1, out=out, reps=reps)
    log(f"launch floor (2^4 half-Dslash, graph-replayed): {t * 1e6:.2f} us")
    return t


def _dslash_point(torch, qx, g, lat, nrhs, seed, link_b, vec_b, reps, plain, key, out,
                  flops_site=FLOPS_SITE):
    from paper_1612_02750_amd import synth

    src = torch.from_numpy(synth.gauss_source(nrhs, lat.hv, seed)).cuda()
    pin = qx.pack(lat, src, g.prec)
    pout = qx.dslash(g, pin, 0, nrhs)
    if plain:
        for _ in range(5):
            qx.dslash(g, pin, 0, nrhs, out=pout)
        torch.cuda.synchronize()
        return
    # median of three timings of `reps` graph-replayed launches each
    t = sorted(qx.time_dslash(g, pin, 0, nrhs, out=pout, reps=reps) for _ in range(3))[1]
    by = (link_b + 2 * vec_b * nrhs) * lat.hv
    out[key] = {
        "us": round(t * 1e6, 2),
        "gflops": round(flops_site * nrhs * lat.hv / t / 1e9, 1),
        "gbs_algorithmic": round(by / t / 1e9, 1),
        "frac_hbm_peak": round(by / t / 1e9 / HBM_PEAK_GBS, 3),
        "shape": list(g.launch(nrhs)),
    }
    log(f"{key}: {out[key]}")


def dslash_sweep(torch, qx, tune=True, plain=False):
    """Half-Dslash at 32^4 (Haar links; FP32 12-real links fit the 256 MB
    Infinity Cache, FP64 18-real ones do not) with one and twelve sources, and
    at 48^4 (every operand far beyond the cache) with one source.  Compulsory
    bytes per output site: 8 links + one input and one output colour vector
    per source.  The improved operator (Naik term, link storage 36) is
    measured beside it: 16 links per site, 1146 flops per output site.
    tune=False keeps the shapes already known (the tuning cache of an earlier
    run); plain=True only launches (for counter runs)."""
    from paper_1612_02750_amd import synth

    res = {}
    # (precision, link storage, link bytes and colour-vector bytes per site);
    # an FP16 vector is 12 bytes of pairs and a 4-byte scale
    variants = (("f32", 12, 384, 24), ("f64", 18, 1152, 48), ("f16", 12, 192, 16))
    naik = (("f32", 1152, 24), ("f64", 2304, 48), ("f16", 576, 16))
    dims32 = (32, 32, 32, 32)
    lat32 = qx.Lattice(dims32)
    U32 = torch.from_numpy(synth.haar_gauge(dims32, 0)).cuda()
    for prec, recon, link_b, vec_b in variants:
        g = qx.Gauge(lat32, U32, prec, recon)
        for nrhs in (1, 12):
            if tune:
                g.tune(nrhs)
            _dslash_point(torch, qx, g, lat32, nrhs, 2, link_b, vec_b, 50, plain,
                          f"32^4-{prec}-{recon}-nrhs{nrhs}", res)
        del g
    for prec, link_b, vec_b in naik:
        g = qx.Gauge(lat32, U32, prec, qx.RECON_NAIK)
        if tune:
            g.tune(1)
        _dslash_point(torch, qx, g, lat32, 1, 2, link_b, vec_b, 50, plain,
                      f"32^4-{prec}-naik-nrhs1", res, flops_site=FLOPS_SITE_NAIK)
        del g
    del U32
    # link values do not change the traffic: a unit gauge field built on the device
    dims48 = (48, 48, 48, 48)
    lat48 = qx.Lattice(dims48)
    U48 = torch.zeros((4, lat48.V, 3, 3), dtype=torch.complex128, device="cuda")
    U48[..., 0, 0] = U48[..., 1, 1] = U48[..., 2, 2] = 1.0
    for prec, recon, link_b, vec_b in variants:
        g = qx.Gauge(lat48, U48, prec, recon)
        if tune:
            g.tune(1)
        _dslash_point(torch, qx, g, lat48, 1, 3, link_b, vec_b, 30, plain,
                      f"48^4-{prec}-{recon}-nrhs1", res)
        del g
    for prec, link_b, vec_b in naik:
        g = qx.Gauge(lat48, U48, prec, qx.RECON_NAIK)
        if tune:
            g.tune(1)
        _dslash_point(torch, qx, g, lat48, 1, 3, link_b, vec_b, 20, plain,
                      f"48^4-{prec}-naik-nrhs1", res, flops_site=FLOPS_SITE_NAIK)
        del g
    del U48
    return res


def copy_probe(torch, qx, nb=1 << 30, timed=True):
    """Plain copy of nb bytes: measured bandwidth (read + write) and counter calibration."""
    a = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    c = torch.empty(nb, dtype=torch.uint8, device="cuda")
    if not timed:
        scratch = torch.zeros(8192, dtype=torch.int32, device="cuda")
        for _ in range(3):
            qx.probe_copy(c, a, nb)
            qx.probe_read(a, nb, scratch)
        torch.cuda.synchronize()
        return None, None
    t_copy = time_kernel(torch, lambda: qx.probe_copy(c, a, nb), 20)
    copy_gbs = 2 * nb / t_copy / 1e9
    scratch = torch.zeros(8192, dtype=torch.int32, device="cuda")
    t_read = time_kernel(torch, lambda: qx.probe_read(a, nb, scratch), 20)
    read_gbs = nb / t_read / 1e9
    log(f"copy probe: {nb} bytes, {t_copy * 1e6:.1f} us, {copy_gbs:.0f} GB/s (read + write); "
        f"read probe: {t_read * 1e6:.1f} us, {read_gbs:.0f} GB/s")
    return copy_gbs, read_gbs


def naik_cg(torch, qx, synth):
    """The improved operator (Naik term) on the step's 16^4 system: mixed and
    FP64 time-to-solution to 1e-10."""
    dims, m, eps, tol = (16, 16, 16, 16), 0.05, 0.3, 1e-10
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.weak_gauge(dims, eps, 0)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", qx.RECON_NAIK)
    g32 = qx.Gauge(lat, Ud, "f32", qx.RECON_NAIK)
    g64.tune(1)
    g32.tune(1)
    bd = torch.from_numpy(synth.gauss_source(1, lat.hv, 1)).cuda()
    out = {"workload": "16^4 weak-field links eps=0.3, improved operator (Naik), m=0.05, tol 1e-10"}
    for name, glo, mode in (("mixed", g32, qx.CG_MIXED_F32), ("fp64", None, qx.CG_FP64)):
        x = torch.empty_like(bd)
        B = qx.Batch([(g64, glo, bd, [m], x)], tol=tol, mode=mode)
        out[f"{name}_solver_launch_shape"] = list(B.tune(2))
        B.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            st = B.solve()
        torch.cuda.synchronize()
        out[f"{name}_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
        out[f"{name}_iters"] = st[0].iters
        out[f"{name}_true_rel_residual"] = st[0].true_rel_residual
    out["speedup_mixed_vs_fp64"] = round(out["fp64_ms"] / out["mixed_ms"], 3)
    log(f"16^4 Naik CG: {out}")
    return out


def hmc_md(torch, qx, synth):
    """One HMC molecular-dynamics trajectory on 16^4 (weak-field start eps=0.3,
    Gaussian momenta and pseudofermion, beta 5.5, m 0.1): ten leapfrog steps
    of 0.02 with mixed-precision force solves to 1e-10."""
    dims, beta, m, eps, nsteps = (16, 16, 16, 16), 5.5, 0.1, 0.02, 10
    lat = qx.Lattice(dims)
    U0 = torch.from_numpy(synth.weak_gauge(dims, 0.3, 0)).cuda()
    p0 = torch.from_numpy(np.random.default_rng(5).standard_normal((4, lat.V, 8))).cuda()
    phi = torch.from_numpy(synth.gauss_source(1, lat.hv, 6)[0]).cuda()
    U = U0.clone()
    g64 = qx.Gauge(lat, U, "f64")
    g32 = qx.Gauge(lat, U, "f32", 12)
    g32.tune(1)
    out = {"workload": "16^4 HMC trajectory: beta 5.5, m 0.1, 10 leapfrog steps of 0.02, "
                       "mixed force solves to 1e-10"}
    for rep in range(2):  # the first run warms up
        U.copy_(U0)
        p = p0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H0, H1, it = qx.md_trajectory(g64, U, p, beta, eps, nsteps, phi=phi, mass=m, glo=g32,
                                      tol=1e-10)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
    out.update({"trajectory_ms": round(t * 1e3, 2), "ms_per_step": round(t * 1e3 / nsteps, 3),
                "cg_iters_per_force": round(it / (nsteps + 1), 1), "dH": H1 - H0, "H_start": H0})
    log(f"16^4 HMC: {out}")
    return out


def mesons(torch, qx, synth):
    """Point-source staggered meson correlators on 16^3 x 32 (weak field eps=0.3,
    m=0.05, seven direction masks), the three colour sources solved together
    in mixed precision to 1e-10."""
    dims, m = (16, 16, 16, 32), 0.05
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.weak_gauge(dims, 0.3, 0)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64")
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    g32.tune(3)
    masks = [0, 1, 2, 4, 8, 7, 15]
    qx.meson_correlators(g64, m, (0, 0, 0, 0), masks, glo=g32, tol=1e-10)
    t0 = time.perf_counter()
    C, st = qx.meson_correlators(g64, m, (0, 0, 0, 0), masks, glo=g32, tol=1e-10)
    t = time.perf_counter() - t0
    out = {"workload": "16^3x32 weak-field links, point source, m=0.05, 7 channels, mixed to 1e-10",
           "ms": round(t * 1e3, 2), "cg_iters": max(s.iters for s in st),
           "pion_C_t0_t1_t2": [float(v) for v in C[0, :3]]}
    log(f"mesons 16^3x32: {out}")
    return out


def multi_rhs(torch, qx, synth):
    """32^4 Haar links, 12 Gaussian sources, m = 0.02, tol 1e-10: the twelve
    sources solved together (FP32 12-real inner iteration, FP64 reliable
    updates, one batch) against plain FP64 CG solving them one after another;
    the same batch with FP16 12-real inner links, and the first source alone
    with FP32 and with FP16 inner links."""
    dims, m, nsrc = (32, 32, 32, 32), 0.02, 12
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.haar_gauge(dims, 0)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", 18)
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    del Ud
    shape12 = g32.tune(nsrc)
    shape1 = g64.tune(1)
    # FP16 inner links run the FP32-vector engine: the FP32 handle's shapes
    g16.set_launch(nsrc, *shape12)
    g16.set_launch(1, *g32.tune(1))
    bd = torch.from_numpy(synth.gauss_source(nsrc, lat.hv, 1)).cuda()
    x_mx = torch.empty_like(bd)
    mixed = qx.Batch([(g64, g32, bd, [m] * nsrc, x_mx)], tol=1e-10, mode=qx.CG_MIXED_F32)
    tuned = {"mixed_batch_12": list(mixed.tune(2))}
    mixed.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = mixed.solve()
    torch.cuda.synchronize()
    t_mx = time.perf_counter() - t0
    x_16 = torch.empty_like(bd)
    mixed16 = qx.Batch([(g64, g16, bd, [m] * nsrc, x_16)], tol=1e-10, mode=qx.CG_MIXED_F32)
    tuned["mixed_f16_links_batch_12"] = list(mixed16.tune(2))
    mixed16.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st16 = mixed16.solve()
    torch.cuda.synchronize()
    t_16 = time.perf_counter() - t0
    del mixed16, x_16
    # one source of the same system: FP32 and FP16 inner links
    one = {}
    for name, glo in (("f32_links", g32), ("f16_links", g16)):
        x1 = torch.empty_like(bd[:1])
        b1 = qx.Batch([(g64, glo, bd[:1], [m], x1)], tol=1e-10, mode=qx.CG_MIXED_F32)
        tuned[f"one_source_{name}"] = list(b1.tune(2))
        b1.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            s1 = b1.solve()
        torch.cuda.synchronize()
        one[name] = {"ms": round((time.perf_counter() - t0) / 2 * 1e3, 2), "iters": s1[0].iters,
                     "true_rel_residual": s1[0].true_rel_residual}
        del b1, x1
    x_b64 = torch.empty_like(bd)
    batch64 = qx.Batch([(g64, None, bd, [m] * nsrc, x_b64)], tol=1e-10, mode=qx.CG_FP64)
    tuned["fp64_batch_12"] = list(batch64.tune(2))
    batch64.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stb = batch64.solve()
    torch.cuda.synchronize()
    t_b64 = time.perf_counter() - t0
    del batch64, x_b64
    x_64 = torch.empty_like(bd)
    plains = [qx.Batch([(g64, None, bd[k:k + 1], [m], x_64[k:k + 1])], tol=1e-10, mode=qx.CG_FP64)
              for k in range(nsrc)]
    tuned["fp64_sequential"] = [list(p.tune(1)) for p in plains][0]
    plains[0].solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st64 = [p.solve()[0] for p in plains]
    torch.cuda.synchronize()
    t_64 = time.perf_counter() - t0
    out = {
        "workload": "32^4 Haar links, 12 Gaussian sources, m=0.02, tol 1e-10",
        "mixed_batch_12_ms": round(t_mx * 1e3, 2),
        "fp64_sequential_12_ms": round(t_64 * 1e3, 2),
        "speedup": round(t_64 / t_mx, 3),
        "fp64_batch_12_ms": round(t_b64 * 1e3, 2),
        "speedup_vs_fp64_batch": round(t_b64 / t_mx, 3),
        "mixed_iters_max": max(s.iters for s in st),
        "fp64_iters_max": max(s.iters for s in st64),
        "mixed_f16_links_batch_12_ms": round(t_16 * 1e3, 2),
        "mixed_f16_links_iters_max": max(s.iters for s in st16),
        "speedup_f16_links": round(t_64 / t_16, 3),
        "one_source_mixed": one,
        "max_true_rel_residual": max(max(s.true_rel_residual for s in st),
                                     max(s.true_rel_residual for s in st64),
                                     max(s.true_rel_residual for s in stb),
                                     max(s.true_rel_residual for s in st16)),
        "launch_shape_f32_12src": list(shape12),
        "launch_shape_f64_1src": list(shape1),
        "solver_launch_shapes": tuned,
    }
    log(f"32^4 x 12 sources: {out}")
    return out


def f16_links_weak32(torch, qx, synth):
    """32^4 weak-field links (eps 0.3), one source, m = 0.05, tol 1e-10: the
    mixed solve with FP32 and with FP16 12-real inner links (the FP32
    handle's tuned launch shape for both)."""
    dims, m = (32, 32, 32, 32), 0.05
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.weak_gauge(dims, 0.3, 0)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", 18)
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    del Ud
    g16.set_launch(1, *g32.tune(1))
    bd = torch.from_numpy(synth.gauss_source(1, lat.hv, 1)).cuda()
    out = {"workload": "32^4 weak-field links eps=0.3, one source, m=0.05, mixed to 1e-10"}
    for name, glo in (("f32_links", g32), ("f16_links", g16)):
        x = torch.empty_like(bd)
        B = qx.Batch([(g64, glo, bd, [m], x)], tol=1e-10, mode=qx.CG_MIXED_F32)
        shape = list(B.tune(2))
        B.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            st = B.solve()
        torch.cuda.synchronize()
        out[name] = {"ms": round((time.perf_counter() - t0) / 3 * 1e3, 2), "iters": st[0].iters,
                     "true_rel_residual": st[0].true_rel_residual, "solver_launch_shape": shape}
        del B, x
    out["speedup_f16_links"] = round(out["f32_links"]["ms"] / out["f16_links"]["ms"], 3)
    log(f"32^4 weak field, FP16 inner links: {out}")
    return out


def cg_kernels_sample(torch, qx, synth):
    """A few CG iterations for counter runs: the step's 16^4 mixed solve (the
    AUTO engine) cut at 32 iterations, and the 32^4 twelve-source mixed solve
    (launch-per-pass engine) cut at 6."""
    for dims, seed_kind, nsrc, m, iters in (((16, 16, 16, 16), "weak", 1, 0.05, 32),
                                            ((32, 32, 32, 32), "haar", 12, 0.02, 6)):
        lat = qx.Lattice(dims)
        U = synth.weak_gauge(dims, 0.3, 0) if seed_kind == "weak" else synth.haar_gauge(dims, 0)
        Ud = torch.from_numpy(U).cuda()
        g64 = qx.Gauge(lat, Ud, "f64", 18)
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        del Ud
        bd = torch.from_numpy(synth.gauss_source(nsrc, lat.hv, 1)).cuda()
        qx.cg(g64, bd, [m] * nsrc, glo=g32, tol=1e-10, max_iter=iters, raise_on_fail=False)
        torch.cuda.synchronize()
        del g64, g32, bd


def uneven_batch(torch, qx, synth):
    """Lattices 8^4, 12^4, 16^4, 16^3 x 32 and 24^4 with weak-field links
    (eps in [0.2, 0.5] by seed), four Gaussian sources each, masses from
    {0.01, 0.05, 0.1}, FP32 12-real inner / FP64 reliable updates to 1e-10:
    the whole batch replayed from its HIP graph against the same systems
    solved one after another (each as its own batch)."""
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32), (24, 24, 24, 24)]
    mlist = [0.01, 0.05, 0.1]
    systems = []
    for k, dims in enumerate(shapes):
        eps = float(np.random.Generator(np.random.PCG64(1000 + k)).uniform(0.2, 0.5))
        lat = qx.Lattice(dims)
        Ud = torch.from_numpy(synth.weak_gauge(dims, eps, k)).cuda()
        g64 = qx.Gauge(lat, Ud, "f64", 18)
        g32 = qx.Gauge(lat, Ud, "f32", 12)
        g32.tune(4)
        bd = torch.from_numpy(synth.gauss_source(4, lat.hv, 100 + k)).cuda()
        systems.append((g64, g32, bd, [mlist[(k + j) % 3] for j in range(4)], torch.empty_like(bd)))
    batch = qx.Batch(systems, tol=1e-10, mode=qx.CG_MIXED_F32)
    singles = [qx.Batch([s], tol=1e-10, mode=qx.CG_MIXED_F32) for s in systems]
    # the solver's launch-shape tuner on the batch and on each single system
    tuned = {"batch": list(batch.tune(2)), "singles": [list(b.tune(2)) for b in singles]}
    batch.solve()
    for b in singles:
        b.solve()
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st = batch.solve()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        st1 = [x for b in singles for x in b.solve()]
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    out = {
        "workload": "8^4, 12^4, 16^4, 16^3x32, 24^4 weak fields, 4 sources each, mixed to 1e-10",
        "batch_ms": round(t_batch * 1e3, 3),
        "one_system_at_a_time_ms": round(t_single * 1e3, 3),
        "speedup": round(t_single / t_batch, 3),
        "iters_max": max(x.iters for x in st),
        "max_true_rel_residual": max(max(x.true_rel_residual for x in st),
                                     max(x.true_rel_residual for x in st1)),
        "all_converged": all(x.status == qx.OK for x in st + st1),
        "solver_launch_shapes": tuned,
    }
    log(f"uneven batch: {out}")
    return out


def force_16(torch, qx, synth):
    """Fermion force of S = phi^dag A^-1 phi on 16^4 Haar links, m = 0.1: the
    solve (FP32 12-real inner, FP64 reliable updates, to 1e-10), D_oe of the
    solution and the per-link outer products, as one call."""
    dims, m = (16, 16, 16, 16), 0.1
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.haar_gauge(dims, 0)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", 18)
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    g32.tune(1)
    phi = torch.from_numpy(synth.gauss_source(1, lat.hv, 1)).cuda()
    qx.force(g64, phi, m, glo=g32)
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        S, G, x, st = qx.force(g64, phi, m, glo=g32)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    out = {
        "workload": "16^4 Haar links, Gaussian phi, m=0.1, mixed solve to 1e-10 + force",
        "ms": round(t * 1e3, 3),
        "cg_iters": st[0].iters,
        "true_rel_residual": st[0].true_rel_residual,
        "action": float(S),
    }
    log(f"16^4 force: {out}")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch

    import paper_1612_02750_amd as qx
    from paper_1612_02750_amd import synth

    qx.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    # ------------------------------------------------------------- workload
    dims = (16, 16, 16, 16)
    m, eps, tol, delta = 0.05, 0.3, 1e-10, 0.1
    lat = qx.Lattice(dims)
    V, hv = lat.V, lat.hv
    U = synth.weak_gauge(dims, eps, 0)
    b = synth.gauss_source(1, hv, 1)
    Ud = torch.from_numpy(U).cuda()
    bd = torch.from_numpy(b).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", 18)
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    if args.kernels_only:
        # counter runs: the kernels of the timed run with its launch shapes
        # (read from the tuning cache that run wrote), a few plain launches each
        # the dominant kernel under every one-source launch shape, three
        # dispatches each in this order (the counter summaries map dispatches
        # to shapes by their order)
        order = []
        for lps in (1, 2, 4, 8):
            for xo in (0, 1, 2, 3):
                g32.set_launch(1, 1, lps, xo)
                dominant_kernel(torch, qx, lat, g32, bd, 3, plain=True)
                order.append([1, lps, xo])
        dslash_sweep(torch, qx, tune=False, plain=True)
        copy_probe(torch, qx, timed=False)
        cg_kernels_sample(torch, qx, synth)
        print(json.dumps({"kernels_only": True, "dominant_shapes_in_order": order}))
        return
    shape32 = g32.tune(1)
    shape64 = g64.tune(1)
    log(f"tuned launch shapes: f32-12 {shape32}, f64-18 {shape64}")
    x_mx = torch.empty_like(bd)
    x_64 = torch.empty_like(bd)
    mixed = qx.Batch([(g64, g32, bd, [m], x_mx)], tol=tol, mode=qx.CG_MIXED_F32, delta=delta)
    plain = qx.Batch([(g64, None, bd, [m], x_64)], tol=tol, mode=qx.CG_FP64)

    # the solver's own launch-shape tuner, for both solves (outside the timed region)
    solver_shapes = {"mixed": list(mixed.tune(2)), "fp64": list(plain.tune(2))}
    log(f"solver launch shapes: {solver_shapes}")
    for _ in range(args.warmup):
        mixed.solve()
    plain.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = mixed.solve()
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    s_mx = st[0]
    log(f"mixed: {t_mixed * 1e3:.3f} ms/solve, iters {s_mx.iters}, updates {s_mx.reliable_updates}, "
        f"residual {s_mx.true_rel_residual:.2e}")

    reps64 = max(3, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps64):
        st64 = plain.solve()
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0) / reps64
    s_64 = st64[0]
    log(f"fp64:  {t_fp64 * 1e3:.3f} ms/solve, iters {s_64.iters}, residual {s_64.true_rel_residual:.2e}")

    # the same mixed solve under each CG engine
    engines = {}
    for name, eng in (("launch", qx.ENGINE_LAUNCH), ("persistent", qx.ENGINE_PERSISTENT)):
        xe = torch.empty_like(bd)
        be = qx.Batch([(g64, g32, bd, [m], xe)], tol=tol, mode=qx.CG_MIXED_F32, delta=delta,
                      engine=eng)
        be.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            se = be.solve()
        torch.cuda.synchronize()
        engines[name] = {"ms": round((time.perf_counter() - t0) / 3 * 1e3, 3), "iters": se[0].iters}
        del be
    log(f"engines (mixed 16^4): {engines}")
    # the same mixed solve with FP16 inner links (FP32 vectors), FP32 handle's shape
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    g16.set_launch(1, *shape32)
    x16 = torch.empty_like(bd)
    b16 = qx.Batch([(g64, g16, bd, [m], x16)], tol=tol, mode=qx.CG_MIXED_F32, delta=delta)
    b16.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        s16 = b16.solve()
    torch.cuda.synchronize()
    t_f16 = (time.perf_counter() - t0) / 3
    log(f"mixed, FP16 inner links: {t_f16 * 1e3:.3f} ms/solve, iters {s16[0].iters}, "
        f"residual {s16[0].true_rel_residual:.2e}")
    del b16, x16

    flops_mixed = (s_mx.iters * 606 + s_mx.reliable_updates * 582) * V
    value = flops_mixed / t_mixed / 1e9

    # ---------------------------------------------- dominant kernel vs roofline
    t_k, achieved = dominant_kernel(torch, qx, lat, g32, bd, args.kernel_reps)
    t_floor = launch_floor(torch, qx, synth, args.kernel_reps)
    sha = kernel_sha()
    traffic = None
    if TRAFFIC and TRAFFIC["sha"] == sha:
        traffic = TRAFFIC["bytes"].get(",".join(str(v) for v in shape32))

    # ------------------------------------------- 32^4 and 48^4 Dslash (HBM size)
    d32 = dslash_sweep(torch, qx)

    copy_gbs, read_gbs = copy_probe(torch, qx)

    multi = None if args.no_multi else multi_rhs(torch, qx, synth)
    f16w = None if args.no_multi else f16_links_weak32(torch, qx, synth)
    naik = naik_cg(torch, qx, synth)
    md = hmc_md(torch, qx, synth)
    mes = mesons(torch, qx, synth)
    uneven = uneven_batch(torch, qx, synth)
    frc = force_16(torch, qx, synth)


    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu:
        import oracle

        threads = oracle.threads()
        # whole FP64 solves of the step's system, repeated until 10 s of host time
        t0 = time.perf_counter()
        solves, iters = 0, 0
        while True:
            xo, sto, it_o, rr_o = oracle.cg(dims, U, m, b[0], tol=tol)
            solves += 1
            iters += it_o
            t_cpu = time.perf_counter() - t0
            if t_cpu >= 10.0:
                break
        cpu = {
            "value": round(iters * 606 * V / t_cpu / 1e9, 3),
            "unit": "GFLOP/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{solves} full FP64 CG solves of the same 16^4 system to 1e-10 "
                      f"({it_o} iterations each, {t_cpu:.1f} s in all, true residual {rr_o:.1e}), "
                      f"{threads} OpenMP threads",
        }
        # parity of the benchmarked solution against the oracle
        rr_gpu = oracle.true_residual(dims, U, m, b[0], x_mx.cpu().numpy()[0])
        log(f"cpu oracle: {cpu}; oracle residual of the GPU solution {rr_gpu:.2e}")

    out = {
        "metric": "Dslash GFLOP/s + % HBM roofline; CG time-to-solution @1e-10, mixed vs FP64",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 reliable updates",
        "data": "synthetic",
        "config": {
            "workload": "mixed-precision even-odd CG, 16^4 weak-field links eps=0.3, m=0.05, "
                        "1 Gaussian source, FP32 12-real inner, FP64 reliable updates delta=0.1, "
                        "tol 1e-10",
            "lattice": list(dims),
            "nrhs": 1,
        },
        "cg_time_to_solution_ms": {"mixed_f32_12": round(t_mixed * 1e3, 3),
                                   "fp64": round(t_fp64 * 1e3, 3),
                                   "speedup_mixed_vs_fp64": round(t_fp64 / t_mixed, 3),
                                   "mixed_f16_links_12": round(t_f16 * 1e3, 3),
                                   "mixed_f16_links_iters": s16[0].iters},
        "cg_engines_mixed_ms": engines,
        "cg_solver_launch_shapes": solver_shapes,
        "cg_iterations": {"mixed": s_mx.iters, "mixed_reliable_updates": s_mx.reliable_updates,
                          "fp64": s_64.iters},
        "true_rel_residual": {"mixed": s_mx.true_rel_residual, "fp64": s_64.true_rel_residual},
        "roofline": {
            "kernel": f"k_dslash<float, 12, {shape32[0]}, {shape32[1]}> (FP32 12-real half-Dslash, 16^4, "
                      f"one source)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "avg_launch_us": round(t_k * 1e6, 3),
            "launch_floor_us": round(t_floor * 1e6, 3),
            "launch_shape": list(shape32),
            "kernel_src_sha": sha,
            "bytes_per_site": BYTES_SITE_F32_12,
            "sites_per_launch": hv,
        },
        "dslash_sweep": d32,
        "multi_rhs_32^4": multi,
        "f16_links_32^4_weak": f16w,
        "naik_cg_16^4": naik,
        "hmc_md_16^4": md,
        "mesons_16^3x32": mes,
        "uneven_batch": uneven,
        "force_16^4": frc,
        "copy_probe_gbs": round(copy_gbs, 1),
        "read_probe_gbs": round(read_gbs, 1),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
