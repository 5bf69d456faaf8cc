// Host-callable launchers of the gfx950 kernels (internal to libqx.so).
#pragma once

#include <vector>

#include "qx_internal.h"

namespace qx {

// Launch shape of the stencil kernels: every block covers 64 sites with
// lps * groups wavefronts; lps wavefronts share the eight hops of a site,
// each group takes nbt sources (groups = ceil(nsrc / nbt)).
struct LaunchShape {
  int nbt = 1;  // sources per thread: 1, 2 or 4 (FP32 arithmetic also 6 and 12)
  int lps = 2;  // wavefronts per site: 1, 2, 4 or 8
  int xcd = 1;  // block order: 0 as dispatched, 1 XCD-contiguous, 2 and 3 XCD-contiguous
                // with (z, t)-tiled traversal, 4 and 5 one z or t slab per XCD walked
                // plane by plane with non-temporal output stores (tile_block)
};
constexpr int kMaxOrder = 5;

inline int shape_groups(const LaunchShape& s, int nsrc) { return (nsrc + s.nbt - 1) / s.nbt; }
// LDS bytes of the hop reduction (0 without hop splitting).
inline size_t shape_lds(const LaunchShape& s, int nsrc, size_t cplx_sz) {
  return s.lps > 1 ? (size_t)shape_groups(s, nsrc) * s.lps * 3 * 64 * cplx_sz : 0;
}
// Most wavefronts per stencil block: 16, or 8 when a thread holds more than
// 8 bytes of real accumulators per colour (FP64 with 2+ sources, FP32 with 4),
// which then get up to 256 VGPRs.
inline int max_waves(int nbt, size_t cplx_sz) { return (cplx_sz / 2) * nbt > 8 ? 8 : 16; }
// Is the shape launchable for nsrc sources with complex numbers of cplx_sz bytes?
// Shape with at most four sources per thread (and at most two wavefronts per
// site when it had more), for a kernel without the wide pairs.
inline LaunchShape narrow_shape(LaunchShape s) {
  if (s.nbt > 4) {
    s.nbt = 4;
    if (s.lps > 2) s.lps = 2;
  }
  return s;
}
inline bool shape_ok(const LaunchShape& s, int nsrc, size_t cplx_sz) {
  const bool nbt_ok = s.nbt == 1 || s.nbt == 2 || s.nbt == 4 ||
                      (cplx_sz == 8 && (s.nbt == 6 || s.nbt == 12));
  const bool lps_ok = s.lps == 1 || s.lps == 2 || s.lps == 4 || s.lps == 8;
  if (!nbt_ok || !lps_ok || s.xcd < 0 || s.xcd > kMaxOrder || nsrc < 1) return false;
  const int waves = s.lps * shape_groups(s, nsrc);
  return waves <= max_waves(s.nbt, cplx_sz) && shape_lds(s, nsrc, cplx_sz) <= 64 * 1024;
}

// Bytes of one complex number of the arithmetic of the given precision
// (QX_PREC_F64 = 0 -> 16; F32 and F16, which computes in FP32 -> 8).
inline size_t cplx_bytes(int prec) { return prec == 0 ? 16 : 8; }
// Bytes of one stored complex link element (F16 = 2 -> 4).
inline size_t link_cplx_bytes(int prec) { return prec == 0 ? 16 : prec == 1 ? 8 : 4; }
// Bytes of one packed source of a half-lattice field: [3][hv] complex, or for
// F16 [hv] records of 16 bytes (three binary16 pairs and an FP32 scale).
inline size_t source_bytes(const Geo& g, int prec) {
  return prec == 2 ? (size_t)16 * g.hv : (size_t)3 * g.hv * cplx_bytes(prec);
}

hipError_t launch_pack_gauge(const Geo& g, const void* U, int prec, int recon, void* packed,
                             unsigned long long* err_bits, hipStream_t s);
hipError_t launch_pack_field(const Geo& g, int nrhs, int prec, const void* canon, void* packed,
                             hipStream_t s);
hipError_t launch_unpack_field(const Geo& g, int nrhs, int prec, const void* packed, void* canon,
                               hipStream_t s);
hipError_t launch_index_maps(const Geo& g, int32_t* lex_of_eo, int32_t* nbr_eo, hipStream_t s);
// st: n SrcState (device); gs: the persistent engine's GridSync or nullptr;
// out: n qx_cg_stats_t (device).
hipError_t launch_batch_stats(const void* st, int n, const void* gs, void* out, hipStream_t s);

// out = scale * (2D) in, from parity 1 - pout to pout, nsrc sources (any count;
// passes of at most 16 * nbt sources).
hipError_t launch_dslash(const Geo& g, int prec, int recon, const void* links, int pout,
                         const void* in, void* out, int nsrc, double scale, LaunchShape sh,
                         hipStream_t s);
// out_k = m2[k] in_k - D_eo D_oe in_k (tmp: odd scratch); square: m2 holds the
// masses, squared on the host per pass.
hipError_t launch_apply_A(const Geo& g, int prec, int recon, const void* links, int nrhs,
                          const double* m2, const void* in, void* out, void* tmp, LaunchShape sh,
                          hipStream_t s, bool square = false);

// A without a caller workspace: the odd intermediate of nrhs sources
// (nrhs * source_bytes) in the library's device array of kNoAllocScratchBytes
// (hipErrorInvalidValue when it does not fit).  Allocates nothing; calls that
// overlap on one GPU share the array and race.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
hipError_t launch_apply_A_noalloc(const Geo& g, int prec, int recon, const void* links, int nrhs,
                                  const double* masses, const void* in, void* out, LaunchShape sh,
                                  hipStream_t s);

// ------------------------------------------------------------------ engine

// Pass kinds of the solver launches (the QX_PASS_* values of qx.h).
enum PassKind : int { PASS_P = 0, PASS_DOE = 1, PASS_DEO = 2, PASS_XR = 3, PASS_FINALIZE = 4,
                      PASS_UPDATE = 5, NPASS = 6 };

// Event timing of the solver's launches (measurement only): while an engine
// configuration carries one, every launch of its iteration and update
// sequences is bracketed by two HIP events on the launch's stream, tagged with
// its pass kind and with the number of sources the host expects it to serve
// (nrun, set before the launches are enqueued).  Events come from a pool that
// lives as long as the object.
struct PassProf {
  struct Rec {
    int kind, nrun;
    hipEvent_t e0, e1;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  int nrun = 0;
  hipError_t err = hipSuccess;

  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) {
        err = r;
        return nullptr;
      }
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int kind, hipStream_t s) {
    Rec r{kind, nrun, next(), next()};
    if (!r.e0 || !r.e1) return;
    const hipError_t e = hipEventRecord(r.e0, s);
    if (e != hipSuccess) err = e;
    recs.push_back(r);
  }
  void end(hipStream_t s) {
    if (recs.empty()) return;
    const hipError_t e = hipEventRecord(recs.back().e1, s);
    if (e != hipSuccess) err = e;
  }
  ~PassProf() {
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

// One solver launch configuration: the systems (device table), their source
// states, the inner precision and link storage, the FP64 link storage, the
// number of sources each thread handles (nb), and the launch shape.
struct EngineCfg {
  int prec_lo = 0, recon_lo = 18, recon_hi = 18;
  bool links16 = false;  // inner links stored as binary16 (prec_lo FP32: the vectors stay FP32)
  int nsrc_max = 1;  // most sources of any system (sets the groups of a block)
  LaunchShape shape;
  // (sources per thread, wavefronts per site) of the launch-per-pass D_eo
  // pass, which the solver tuner picks apart from the other stencils (its A
  // epilogue and FP64 dot products change the register balance); the block
  // order is shape's.  The other engines use `shape` throughout.
  LaunchShape deo_shape;
  int nsys = 0, nblk_total = 0, nvblk_total = 0, nsrc_total = 0;
  const SysDesc* d_sys = nullptr;
  SrcState* d_st = nullptr;   // the source states (slot 0)
  SrcState* d_st1 = nullptr;  // second slot of the fused launch sequence
  bool fused = false;         // three launches per iteration (redundant reductions), see the engine
  bool two = false;           // with fused: two launches per iteration (x/r step folded into D_oe)
  PassProf* prof = nullptr;   // event timing of every launch (measurement only), or null
};

// Launch statement `launch` bracketed by the pass timer of c (when set).
#define QX_TIMED(c, kind, s, launch)       \
  do {                                     \
    if ((c).prof) (c).prof->begin(kind, s); \
    launch;                                \
    if ((c).prof) (c).prof->end(s);        \
  } while (0)

bool engine_supported(const EngineCfg& c);
hipError_t engine_init(const EngineCfg& c, int zero_xhi, hipStream_t s);
// parity: of the iteration's index in its chunk (the fused sequence alternates
// two p slots; its chunks hold an even number of iterations).
hipError_t engine_iteration(const EngineCfg& c, int parity, hipStream_t s);
// last: the update ends a chunk (every step done before the host reads the
// states); otherwise the two-launch sequence leaves its last step to the next
// D_oe pass.
hipError_t engine_reliable_update(const EngineCfg& c, bool last, hipStream_t s);
// Co-resident blocks of the persistent solver kernel on this device (0 if it
// cannot be launched), and one cooperative launch of up to `iters` iterations.
int engine_persistent_capacity(const EngineCfg& c);
hipError_t engine_persistent(const EngineCfg& c, int iters, GridSync* gs, int grid, hipStream_t s);

// ------------------------------------------------------------------ force

hipError_t launch_force(const Geo& g, int nsrc, const void* x, const void* lam, const void* y,
                        const void* nu, void* G, hipStream_t s);
hipError_t launch_su3_force(const Geo& g, const void* U, const void* G, double* F, hipStream_t s);
// out = sc * in over n complex128 values.
hipError_t launch_scale_c128(const void* in, double sc, size_t n, void* out, hipStream_t s);
// out = sum_i Re(conj(a_i) b_i) over n complex128 values (two deterministic passes).
hipError_t launch_redot(const void* a, const void* b, size_t n, double* partials, int nblk,
                        double* out, hipStream_t s);

// ----------------------------------------------------- molecular dynamics
// (canonical FP64 layouts: U [4][V][3][3] complex, p [4][V][8] real)

// out = sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3), nblk partial sums.
hipError_t launch_plaquette_sum(const Geo& g, const void* U, double* partials, int nblk,
                                double* out, hipStream_t s);
// G (+)= -(beta/3) A^dag (A: the six staples of every link).
hipError_t launch_gauge_grad(const Geo& g, const void* U, double beta, void* G, int accumulate,
                             hipStream_t s);
// p^a -= eps Re[i tr(T_a U G^dag)].
hipError_t launch_mom_update(const Geo& g, const void* U, const void* G, double eps, double* p,
                             hipStream_t s);
// U <- exp(i eps sum_a p^a T_a) U.
hipError_t launch_link_update(const Geo& g, const double* p, double eps, void* U, hipStream_t s);
// out = sum v^2 over n doubles.
hipError_t launch_sumsq(const double* v, int64_t n, double* partials, int nblk, double* out,
                        hipStream_t s);

// ------------------------------------------------------------------ mesons

// Three canonical point sources (one per colour) at even checkerboard site cb_src.
hipError_t launch_point_source(const Geo& g, int cb_src, void* b, hipStream_t s);
// C[k][t] (device) from packed x (even) and y = D_oe x (odd) of three sources.
hipError_t launch_meson_contract(const Geo& g, const void* xp, const void* yp, double mass,
                                 int t_src, int nmask, const int* masks, double* C, hipStream_t s);

// Read bytes (a multiple of 16) once; out: 8192 unsigned words of scratch.
hipError_t launch_read(const void* src, size_t bytes, unsigned* out, hipStream_t s);
// dst = src, bytes a multiple of 16.
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace qx
