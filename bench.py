"""Benchmark: staggered Dslash + even-odd CG on one MI355X.

Workload (one step): the multi-source solve of the CG benchmark extended to
many right-hand sides -- a 32^4 lattice with Haar-random SU(3) links (seed 0),
twelve complex-Gaussian sources (seed 1), m = 0.02 for every source, solved
together to a true FP64 relative residual of 1e-10 per source: FP32 inner
iterations on 12-real links, FP64 reliable updates when |r| drops below
0.1 max|r|, one batch (one launch per CG pass for all twelve sources,
replayed from HIP graphs).  Inputs are resident in HBM before the timed
region; a step includes packing the sources, every inner iteration and
reliable update, and unpacking the solutions.  K steps are timed one by one
(host synchronisation around each); ms_per_step is their median and value
the sustained GFLOP/s of the median step.

Reported beside it (same run):
  * the same twelve systems in plain FP64: as one FP64 batch and as twelve
    FP64 single-source solves one after another (medians of five), i.e. the
    time-to-solution comparison mixed vs FP64 at equal and at single batching;
  * the roofline of the dominant kernel of the step, the D_eo pass of the
    iteration (half-Dslash with the A epilogue and the <p, A p> partials,
    under the launch shape the solver tuner gave it), from HIP events around
    each of its launches in an event-timed run of the same batch (two chunks
    of its solve, eager launches), and the other passes of the iteration
    from the same run;
  * the 16^4 weak-field single-source solve (mixed vs FP64, every engine, FP16
    inner links);
  * the half-Dslash on 32^4 and 48^4 in FP32-12, FP64-18 and FP16-12, one and
    twelve sources, with and without the Naik term; the copy and read probes;
  * the 32^4 twelve-source batch with FP16 inner links and its first source
    alone; the improved operator's CG, an HMC trajectory, meson correlators,
    the uneven batch and the 16^4 fermion force;
  * the CPU oracle on the host cores: FP64 CG iterations of the step's first
    system, and the half-Dslash at 16^4 and 32^4 on all threads and on one.

Flop convention: 570 flops per output site per half-Dslash; one CG iteration
costs 606 V per source (two half-Dslash + BLAS-1), one reliable update 582 V.

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
MALL_BYTES = 256 << 20  # Infinity Cache of the MI355X
FLOPS_SITE = 570
FLOPS_SITE_NAIK = 1146  # 16 SU(3) x colour-vector products + 15 vector sums


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the 32^4 FP16-link and one-source comparisons")
    ap.add_argument("--solver-shape", default=None,
                    help="nbt,lps,order[,deo_nbt,deo_lps] of the step's batch instead of its "
                         "tuner (profiler runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed step, its FP64 comparisons and its pass timing")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the dominant-kernel timing and the copy probe (for counter runs)")
    ap.add_argument("--dslash-point", default=None, metavar="NBT,LPS,ORDER,NRHS",
                    help="only the standalone 32^4 FP32-12 half-Dslash of NRHS sources under "
                         "the given shape: three plain launches and a graph-timed figure "
                         "(for counter runs)")
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


# Algorithmic bytes per output site of the passes of one mixed iteration
# (FP32 12-real links, FP32 colour vectors): links are read once per launch
# that has work, a colour vector of every served source once per site.
LINK_B_F32_12 = 384   # 8 links x 12 reals x 4 B
VEC_B_F32 = 24        # one FP32 colour vector (3 complex)
PASS_BYTES = {
    # pass: (bytes per output site per launch, per served source)
    "doe": (LINK_B_F32_12, 2 * VEC_B_F32),   # p read, t written
    "deo": (LINK_B_F32_12, 3 * VEC_B_F32),   # t and p read, A p written
    "xr": (0, 3 * VEC_B_F32),                # r, A p read; r written (x += alpha p deferred)
    "p": (0, 5 * VEC_B_F32),                 # r, p, x read; p, x written
}

# HBM-side bytes per launch of the dominant kernel (the D_eo pass of the
# twelve-source step, all sources served) from two rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the same
# counters read for the library's copy and read probes on 1 GiB (FETCH x 2,
# WRITE x 1), from profiles/cg_mixed_32x32x32x32_12src_counters.md.  Reported
# only while the engine sources and the launch shape are the ones the counters
# were taken with; keyed by the D_eo pass's "nbt,lps,order".
TRAFFIC = {"sha": "790b325ec7814658", "bytes": {"4,1,0": 1176544528, "1,1,0": 867501792}}
KERNEL_SOURCES = ("qx_engine_kernels.h", "qx_device.h", "qx_internal.h", "qx_launch.h",
                  "qx_dispatch.h")


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1612_02750_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _sync_time(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def _flops(stats, V):
    return sum(s.iters * 606 + s.reliable_updates * 582 for s in stats) * V


def config3_system(torch, qx, synth):
    """The step's system: 32^4 Haar links (seed 0), 12 Gaussian sources (seed 1)."""
    dims, nsrc = (32, 32, 32, 32), 12
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.haar_gauge(dims, 0)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", 18)
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    del Ud
    bd = torch.from_numpy(synth.gauss_source(nsrc, lat.hv, 1)).cuda()
    return lat, g64, g32, bd


def pass_roofline(passes, hv):
    """Per pass of the event-timed run: average duration of the launches that
    had work, the sources they served on average, algorithmic bytes per launch
    and the fraction of the HBM peak."""
    out = {}
    for name, (per_site, per_src) in PASS_BYTES.items():
        q = passes[name]
        if not q["active_launches"]:
            continue
        us = q["active_ms"] / q["active_launches"] * 1e3
        nrun = q["source_launches"] / q["active_launches"]
        by = (per_site + per_src * nrun) * hv
        out[name] = {"avg_us": round(us, 2), "launches": q["active_launches"],
                     "sources_served": round(nrun, 3), "algorithmic_bytes": int(by),
                     "gbs": round(by / (us * 1e-6) / 1e9, 1),
                     "frac": round(by / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    for name in ("finalize", "update"):
        q = passes[name]
        if q["launches"]:
            out[name] = {"avg_us": round(q["ms"] / q["launches"] * 1e3, 2),
                         "launches": q["launches"]}
    return out


def headline(torch, qx, synth, args):
    """The timed step (module docstring) with its FP64 comparisons and the
    event timing of its passes."""
    m, tol = 0.02, 1e-10
    lat, g64, g32, bd = config3_system(torch, qx, synth)
    nsrc, V, hv = bd.shape[0], lat.V, lat.hv
    g32.tune(nsrc)
    g64.tune(nsrc)
    g64.tune(1)
    x_mx = torch.empty_like(bd)
    mixed = qx.Batch([(g64, g32, bd, [m] * nsrc, x_mx)], tol=tol, mode=qx.CG_MIXED_F32)
    if args.solver_shape:  # a fixed shape (profiler runs), else the solver's own tuner
        set_solver_shape(mixed, args.solver_shape)
    else:
        mixed.tune(2)
    main_shape, deo_shape = mixed.launch()
    shape = list(main_shape) + list(deo_shape)
    log(f"step: solver launch shape {shape} (nbt, lps, order; D_eo nbt, lps)")
    for _ in range(args.warmup):
        mixed.solve()
    times, st = [], None
    for _ in range(args.steps):
        t, st = _sync_time(torch, mixed.solve)
        times.append(t)
    t_step = float(np.median(times))
    flops = _flops(st, V)
    log(f"step: {[round(t * 1e3, 1) for t in times]} ms, median {t_step * 1e3:.1f} ms, "
        f"iters {max(s.iters for s in st)}, updates {max(s.reliable_updates for s in st)}, "
        f"max residual {max(s.true_rel_residual for s in st):.2e}")
    # the passes of the same batch, event-timed (two chunks from the start)
    passes, st_p = mixed.profile(2)
    roof = pass_roofline(passes, hv)
    log(f"passes: {roof}")
    out = {"times_ms": [round(t * 1e3, 2) for t in times], "t_step": t_step, "flops": flops,
           "stats": st, "shape": shape, "passes": roof,
           "profile_iters": [s.iters for s in st_p]}
    # FP64: one batch of the twelve sources, and twelve single-source solves
    x_b = torch.empty_like(bd)
    b64 = qx.Batch([(g64, None, bd, [m] * nsrc, x_b)], tol=tol, mode=qx.CG_FP64)
    out["fp64_batch_shape"] = list(b64.tune(2))
    b64.solve()
    tb = []
    for _ in range(5):
        t, stb = _sync_time(torch, b64.solve)
        tb.append(t)
    del b64, x_b
    x_s = torch.empty_like(bd)
    singles = [qx.Batch([(g64, None, bd[k:k + 1], [m], x_s[k:k + 1])], tol=tol, mode=qx.CG_FP64)
               for k in range(nsrc)]
    shape1 = list(singles[0].tune(2))
    for b in singles[1:]:
        b.set_launch(*shape1)
    singles[0].solve()
    ts = []
    for _ in range(5):
        t, st1 = _sync_time(torch, lambda: [b.solve()[0] for b in singles])
        ts.append(t)
    del singles, x_s
    out.update({
        "fp64_batch_ms": [round(t * 1e3, 2) for t in tb], "t_fp64_batch": float(np.median(tb)),
        "fp64_seq_ms": [round(t * 1e3, 2) for t in ts], "t_fp64_seq": float(np.median(ts)),
        "fp64_single_shape": shape1,
        "fp64_iters_max": max(s.iters for s in stb),
        "max_true_rel_residual": max(max(s.true_rel_residual for s in st),
                                     max(s.true_rel_residual for s in stb),
                                     max(s.true_rel_residual for s in st1)),
    })
    log(f"fp64 batch {out['fp64_batch_ms']} ms, fp64 one by one {out['fp64_seq_ms']} ms")
    out["_keep"] = (lat, g64, g32, bd, x_mx)
    return out


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
    # every operand of the launch (all links, the input and output vectors)
    # fits the 256 MB Infinity Cache: the fraction is then a cache-served
    # figure, not an HBM one
    resident = by <= MALL_BYTES
    out[key] = {
        "us": round(t * 1e6, 2),
        "gflops": round(flops_site * nrhs * lat.hv / t / 1e9, 1),
        "gbs_algorithmic": round(by / t / 1e9, 1),
        "frac_hbm_peak": round(by / t / 1e9 / HBM_PEAK_GBS, 3),
        "operands_mb": round(by / 1e6, 1),
        "cache_resident": resident,
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


def multi_rhs_extras(torch, qx, synth, h):
    """The step's system with FP16 12-real inner links (one batch of the twelve
    sources), and its first source alone with FP32 and with FP16 inner links."""
    m = 0.02
    lat, g64, g32, bd, _ = h["_keep"]
    nsrc = bd.shape[0]
    # the step's links again (the FP16 handle is packed from the canonical field)
    g16 = qx.Gauge(lat, torch.from_numpy(synth.haar_gauge(lat.dims, 0)).cuda(), "f16", 12)
    g16.tune(nsrc)
    g16.set_launch(1, *g32.tune(1))
    out = {"workload": "32^4 Haar links, 12 Gaussian sources, m=0.02, tol 1e-10"}
    x16 = torch.empty_like(bd)
    b16 = qx.Batch([(g64, g16, bd, [m] * nsrc, x16)], tol=1e-10, mode=qx.CG_MIXED_F32)
    out["f16_links_batch_shape"] = list(b16.tune(2))
    b16.solve()
    t, st16 = _sync_time(torch, b16.solve)
    out["mixed_f16_links_batch_12_ms"] = round(t * 1e3, 2)
    out["mixed_f16_links_iters_max"] = max(s.iters for s in st16)
    del b16, x16
    # the same batch in one cooperative launch per chunk of iterations (grid
    # barriers between the passes), beside the launch-per-pass headline.  The
    # persistent engine takes its shape from the inner-link handle and has no
    # tuner of its own: it runs under (4, 2, 1), the fastest of the shapes
    # measured for it here (2.9 s; one source per thread and one wavefront per
    # site, which the Dslash tuner may pick for the kernel alone, 4.9 s)
    g32.set_launch(nsrc, 4, 2, 1)
    xp = torch.empty_like(bd)
    bp = qx.Batch([(g64, g32, bd, [m] * nsrc, xp)], tol=1e-10, mode=qx.CG_MIXED_F32,
                  engine=qx.ENGINE_PERSISTENT)
    bp.solve()
    runs, stp = [], None
    for _ in range(3):
        t, stp = _sync_time(torch, bp.solve)
        runs.append(round(t * 1e3, 2))
    out["persistent_engine_batch_12"] = {
        "ms": sorted(runs)[1], "runs_ms": runs, "iters_max": max(q.iters for q in stp),
        "true_rel_residual_max": max(q.true_rel_residual for q in stp)}
    del bp, xp
    one = {}
    for name, glo in (("f32_links", g32), ("f16_links", g16)):
        x1 = torch.empty_like(bd[:1])
        b1 = qx.Batch([(g64, glo, bd[:1], [m], x1)], tol=1e-10, mode=qx.CG_MIXED_F32)
        shape = list(b1.tune(2))
        b1.solve()
        t, s1 = _sync_time(torch, lambda: [b1.solve(), b1.solve()][-1])
        one[name] = {"ms": round(t / 2 * 1e3, 2), "iters": s1[0].iters,
                     "true_rel_residual": s1[0].true_rel_residual, "solver_launch_shape": shape}
        del b1, x1
    out["one_source_mixed"] = one
    out["max_true_rel_residual"] = max([s.true_rel_residual for s in st16] +
                                       [out["persistent_engine_batch_12"]["true_rel_residual_max"]] +
                                       [v["true_rel_residual"] for v in one.values()])
    log(f"32^4 x 12 sources, FP16 inner links and one source: {out}")
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


def dslash_point(torch, qx, synth, spec):
    """The half-Dslash of the sweep's 32^4 FP32-12 point (Haar links, seed 0;
    Gaussian sources, seed 1) for nrhs sources under a fixed launch shape:
    three plain launches (what a counter run reads), then the graph-timed
    average of 20."""
    nbt, lps, order, nrhs = (int(v) for v in spec.split(","))
    dims = (32, 32, 32, 32)
    lat = qx.Lattice(dims)
    g = qx.Gauge(lat, torch.from_numpy(synth.haar_gauge(dims, 0)).cuda(), "f32", 12)
    xin = qx.pack(lat, torch.from_numpy(synth.gauss_source(nrhs, lat.hv, 1)).cuda(), "f32")
    g.set_launch(nrhs, nbt, lps, order)
    out = None
    for _ in range(3):
        out = qx.dslash(g, xin, 0, nrhs, out=out)
    torch.cuda.synchronize()
    t = qx.time_dslash(g, xin, 0, nrhs, out=out, reps=20)
    return {"dslash_point": [nbt, lps, order, nrhs], "us": round(t * 1e6, 2)}


def deo_kernel_name(nbt, lps, nsrc=12):
    """The D_eo kernel of the launch-per-pass engine for nsrc FP32-12 sources
    under (nbt, lps): with one wavefront per site and two or more source
    groups the block's groups share the link loads through LDS."""
    if lps == 1 and -(-nsrc // nbt) >= 2:
        return f"k_iter_deo_ll<float, 12, {nbt}, float>"
    return f"k_iter_deo<float, 12, {nbt}, {lps}, float>"


def set_solver_shape(B, spec):
    """spec "nbt,lps,order" or "nbt,lps,order,deo_nbt,deo_lps" (the D_eo pass
    of the launch-per-pass engine under a shape of its own)."""
    v = [int(x) for x in spec.split(",")]
    B.set_launch(*v[:3])
    if len(v) == 5 and tuple(v[3:]) != tuple(v[:2]):
        B.set_deo_launch(*v[3:])


def kernels_only(torch, qx, synth, spec):
    """Counter runs: the step's batch under the given solver launch shape,
    its first two chunks (32 iterations, every source served), eagerly."""
    m = 0.02
    lat, g64, g32, bd = config3_system(torch, qx, synth)
    x = torch.empty_like(bd)
    B = qx.Batch([(g64, g32, bd, [m] * bd.shape[0], x)], tol=1e-10, mode=qx.CG_MIXED_F32)
    set_solver_shape(B, spec)
    passes, st = B.profile(2)
    torch.cuda.synchronize()
    return pass_roofline(passes, lat.hv), [s.iters for s in st]


def config2_16(torch, qx, synth):
    """16^4 weak-field links eps 0.3, m 0.05, one source, tol 1e-10: the mixed
    solve (AUTO engine, solver-tuned shape) against plain FP64, under each
    engine, and with FP16 inner links."""
    dims, m, eps, tol, delta = (16, 16, 16, 16), 0.05, 0.3, 1e-10, 0.1
    lat = qx.Lattice(dims)
    Ud = torch.from_numpy(synth.weak_gauge(dims, eps, 0)).cuda()
    bd = torch.from_numpy(synth.gauss_source(1, lat.hv, 1)).cuda()
    g64 = qx.Gauge(lat, Ud, "f64", 18)
    g32 = qx.Gauge(lat, Ud, "f32", 12)
    shape32, shape64 = g32.tune(1), g64.tune(1)
    out = {"workload": "16^4 weak-field links eps=0.3, m=0.05, 1 Gaussian source, tol 1e-10"}
    x_mx, x_64 = torch.empty_like(bd), torch.empty_like(bd)
    mixed = qx.Batch([(g64, g32, bd, [m], x_mx)], tol=tol, mode=qx.CG_MIXED_F32, delta=delta)
    plain = qx.Batch([(g64, None, bd, [m], x_64)], tol=tol, mode=qx.CG_FP64)
    out["solver_launch_shapes"] = {"mixed": list(mixed.tune(2)), "fp64": list(plain.tune(2))}
    for b in (mixed, plain):
        b.solve()
    tm = [_sync_time(torch, mixed.solve)[0] for _ in range(10)]
    tp = [_sync_time(torch, plain.solve)[0] for _ in range(10)]
    st, s64 = mixed.solve(), plain.solve()
    out.update({"mixed_ms": round(float(np.median(tm)) * 1e3, 3),
                "fp64_ms": round(float(np.median(tp)) * 1e3, 3),
                "mixed_iters": st[0].iters, "mixed_reliable_updates": st[0].reliable_updates,
                "fp64_iters": s64[0].iters,
                "true_rel_residual": {"mixed": st[0].true_rel_residual,
                                      "fp64": s64[0].true_rel_residual}})
    out["speedup_mixed_vs_fp64"] = round(out["fp64_ms"] / out["mixed_ms"], 3)
    out["gflops_mixed"] = round(_flops(st, lat.V) / (out["mixed_ms"] * 1e-3) / 1e9, 1)
    engines = {}
    for name, eng in (("launch", qx.ENGINE_LAUNCH), ("fused", qx.ENGINE_FUSED),
                      ("persistent", qx.ENGINE_PERSISTENT)):
        xe = torch.empty_like(bd)
        be = qx.Batch([(g64, g32, bd, [m], xe)], tol=tol, mode=qx.CG_MIXED_F32, delta=delta,
                      engine=eng)
        be.solve()
        te = [_sync_time(torch, be.solve)[0] for _ in range(3)]
        engines[name] = round(float(np.median(te)) * 1e3, 3)
        del be
    out["engines_mixed_ms"] = engines
    g16 = qx.Gauge(lat, Ud, "f16", 12)
    g16.set_launch(1, *shape32)
    x16 = torch.empty_like(bd)
    b16 = qx.Batch([(g64, g16, bd, [m], x16)], tol=tol, mode=qx.CG_MIXED_F32, delta=delta)
    b16.solve()
    t16 = [_sync_time(torch, b16.solve)[0] for _ in range(3)]
    s16 = b16.solve()
    out["mixed_f16_links_ms"] = round(float(np.median(t16)) * 1e3, 3)
    out["mixed_f16_links_iters"] = s16[0].iters
    log(f"16^4 config 2: {out}")
    return out


def cpu_baseline(torch, qx, synth):
    """The oracle on the host cores: FP64 CG iterations of the step's first
    system (calls of 20 iterations from a zero guess until 12 s have passed),
    and the half-Dslash at 16^4 and 32^4 on every thread and on one."""
    import oracle

    threads = oracle.threads()
    dims, m = (32, 32, 32, 32), 0.02
    V = int(np.prod(dims))
    U = synth.haar_gauge(dims, 0)
    b = synth.gauss_source(1, V // 2, 1)[0]
    t0 = time.perf_counter()
    iters, calls = 0, 0
    while True:
        _, _, it, _ = oracle.cg(dims, U, m, b, tol=1e-10, max_iter=20)
        iters += it
        calls += 1
        t = time.perf_counter() - t0
        if t >= 12.0:
            break
    gflops = iters * 606 * V / t / 1e9
    dsl = {}
    for d in ((16, 16, 16, 16), (32, 32, 32, 32)):
        Ud = synth.haar_gauge(d, 0) if d != dims else U
        chi = synth.gauss_source(1, int(np.prod(d)) // 2, 2)[0]
        for nthr in (threads, 1):
            oracle.set_threads(nthr)
            reps = 20 if d[0] == 16 else (5 if nthr > 1 else 3)
            ts = []
            for _ in range(reps):
                t1 = time.perf_counter()
                oracle.dslash_eo(d, Ud, chi, 0)
                ts.append(time.perf_counter() - t1)
            tm = float(np.median(ts))
            dsl[f"{d[0]}^4_{nthr}thr"] = {"ms": round(tm * 1e3, 2),
                                          "gflops": round(570 * int(np.prod(d)) / 2 / tm / 1e9, 2)}
        oracle.set_threads(threads)
    out = {
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"FP64 CG iterations of the step's first system (32^4 Haar, m=0.02, source 0): "
                  f"{calls} calls of 20 iterations from a zero guess, {iters} iterations in "
                  f"{t:.1f} s on {threads} OpenMP threads; same flop convention",
        "dslash_medians": dsl,
    }
    log(f"cpu oracle: {out}")
    return out


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
        print(json.dumps({"error": "this benchmark runs on one GPU only (one process, one MI355X); "
                                   "run it with --gpus 1"}))
        sys.exit(2)
    import torch

    import paper_1612_02750_amd as qx
    from paper_1612_02750_amd import synth

    qx.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    if args.dslash_point:
        print(json.dumps(dslash_point(torch, qx, synth, args.dslash_point)))
        return

    if args.kernels_only:
        shape = args.solver_shape or "4,2,0"
        roof, iters = kernels_only(torch, qx, synth, shape)
        copy_probe(torch, qx, timed=False)
        print(json.dumps({"kernels_only": True, "solver_shape": shape, "passes": roof,
                          "iters_after": iters}))
        return

    h = headline(torch, qx, synth, args)
    keep = h.pop("_keep")
    lat = keep[0]
    V, hv = lat.V, lat.hv
    st = h["stats"]
    value = h["flops"] / h["t_step"] / 1e9
    deo = h["passes"]["deo"]
    sha = kernel_sha()
    traffic = None
    if TRAFFIC["sha"] == sha:
        # keyed by the D_eo pass's (nbt, lps) and the block order
        sh = h["shape"]
        traffic = TRAFFIC["bytes"].get(f"{sh[3]},{sh[4]},{sh[2]}")
    torch.cuda.empty_cache()

    extras = {}
    if not args.headline_only:
        extras["config2_16^4"] = config2_16(torch, qx, synth)
        extras["dslash_sweep"] = dslash_sweep(torch, qx)
        copy_gbs, read_gbs = copy_probe(torch, qx)
        extras["copy_probe_gbs"] = round(copy_gbs, 1)
        extras["read_probe_gbs"] = round(read_gbs, 1)
        if not args.no_multi:
            extras["multi_rhs_32^4_extras"] = multi_rhs_extras(torch, qx, synth, {"_keep": keep})
            extras["f16_links_32^4_weak"] = f16_links_weak32(torch, qx, synth)
        extras["naik_cg_16^4"] = naik_cg(torch, qx, synth)
        extras["hmc_md_16^4"] = hmc_md(torch, qx, synth)
        extras["mesons_16^3x32"] = mesons(torch, qx, synth)
        extras["uneven_batch"] = uneven_batch(torch, qx, synth)
        extras["force_16^4"] = force_16(torch, qx, synth)
    del keep
    torch.cuda.empty_cache()
    cpu = None if args.no_cpu else cpu_baseline(torch, qx, synth)

    t_mx, t_b, t_s = h["t_step"], h["t_fp64_batch"], h["t_fp64_seq"]
    out = {
        "metric": "Dslash GFLOP/s + % HBM roofline; CG time-to-solution @1e-10, mixed vs FP64",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mx * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 reliable updates",
        "data": "synthetic",
        "config": {
            "workload": "multi-source mixed-precision even-odd CG: 32^4 Haar-random SU(3) links "
                        "(seed 0), 12 complex-Gaussian sources (seed 1) solved together, m=0.02, "
                        "FP32 12-real inner, FP64 reliable updates delta=0.1, tol 1e-10 (true FP64 "
                        "residual per source)",
            "lattice": [32, 32, 32, 32],
            "nrhs": 12,
            "solver_launch_shape": h["shape"],  # nbt, lps, order; D_eo pass nbt, lps
        },
        "step_times_ms": h["times_ms"],
        "cg_time_to_solution_ms": {
            "mixed_batch_12": round(t_mx * 1e3, 2),
            "fp64_batch_12": round(t_b * 1e3, 2),
            "fp64_one_by_one_12": round(t_s * 1e3, 2),
            "speedup_vs_fp64_batch": round(t_b / t_mx, 3),
            "speedup_vs_fp64_one_by_one": round(t_s / t_mx, 3),
            "fp64_batch_runs_ms": h["fp64_batch_ms"],
            "fp64_one_by_one_runs_ms": h["fp64_seq_ms"],
            "fp64_solver_launch_shapes": {"batch": h["fp64_batch_shape"],
                                          "single": h["fp64_single_shape"]},
        },
        "cg_iterations": {"mixed_max": max(s.iters for s in st),
                          "mixed_reliable_updates_max": max(s.reliable_updates for s in st),
                          "fp64_max": h["fp64_iters_max"]},
        "max_true_rel_residual": h["max_true_rel_residual"],
        "roofline": {
            "kernel": f"{deo_kernel_name(h['shape'][3], h['shape'][4])} "
                      f"(D_eo half-Dslash of the step with the A epilogue and <p, Ap> partials; "
                      f"block order {h['shape'][2]})",
            "bound": "hbm",
            "achieved": deo["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": deo["frac"],
            "traffic": traffic,
            "avg_launch_us": deo["avg_us"],
            "launches_timed": deo["launches"],
            "sources_served": deo["sources_served"],
            "bytes_per_launch": deo["algorithmic_bytes"],
            "bytes_per_site": f"{PASS_BYTES['deo'][0]} + {PASS_BYTES['deo'][1]} per source",
            "sites_per_launch": hv,
            "kernel_src_sha": sha,
            "passes": h["passes"],
        },
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
