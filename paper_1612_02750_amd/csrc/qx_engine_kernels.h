// Conjugate-gradient engine on gfx950: the kernels of one CG iteration, of a
// reliable update and of the initialisation, for a batch of systems.
//
// Every engine launch covers all systems of a batch.  Stencil launches give a
// system blocks of 64 sites; vector launches give each of its sources blocks
// of 256 complex elements.  A source takes part in a launch only in the phase
// the kernel serves (PH_RUN for the iteration, PH_RU / PH_RU2 for the update),
// so converged sources cost nothing but the link loads they share with the
// others.
//
// Reductions need no memory fence inside a kernel: every block stores its
// partial sums (fixed-order wave and block sums) with plain stores, and after
// the kernel boundary a finalize kernel with one block per source adds the
// partials in index order and applies the state update (alpha, beta, the
// reliable-update and convergence decisions).  On MI355X an agent-scope fence
// writes back the issuing XCD's L2, so a fence per block (last-block
// reductions, grid barriers) costs far more than the extra launch.
//
// One iteration is six launches: the p update (p = r + beta p), D_oe, D_eo
// fused with the A epilogue and the <p, Ap> partials, the alpha finalize, the
// x/r update with the |r|^2 partials, and the beta finalize.  (Applying the p
// update on the fly inside D_oe saves a pass but doubles the neighbour loads
// the compiler hoists, which spills registers; the separate pass is cheaper.)
//
// Vector slots: inner precision vlo = {x_lo, r, p, Ap, t(odd), p'}, FP64
// vhi = {x_hi, r_hi, b, t_hi(odd)}; each slot is [nsrc][3][hv]; p' is the
// second p slot of the fused sequence.
//
// Template parameters of the iteration kernels: R is the inner arithmetic and
// vector storage (float or double), LS the storage of the inner links (R, or
// __half under FP32 vectors: the links are converted to R as they are loaded).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "qx_device.h"
#include "qx_dispatch.h"
#include "qx_engine_impl.h"
#include "qx_launch.h"

namespace qx {

namespace {

constexpr int kStatusOk = 0;
constexpr int kStatusNotConverged = 5;
constexpr int kStatusBreakdown = 6;

__device__ __forceinline__ const SysDesc& sys_of_block(const SysDesc* __restrict__ sys, int nsys,
                                                       int b) {
  int i = 0;
  while (i + 1 < nsys && b >= sys[i + 1].blk0) ++i;
  return sys[i];
}

__device__ __forceinline__ const SysDesc& sys_of_vblock(const SysDesc* __restrict__ sys, int nsys,
                                                        int b) {
  int i = 0;
  while (i + 1 < nsys && b >= sys[i + 1].vblk0) ++i;
  return sys[i];
}

__device__ __forceinline__ const SysDesc& sys_of_source(const SysDesc* __restrict__ sys, int nsys,
                                                        int k) {
  int i = 0;
  while (i + 1 < nsys && k >= sys[i + 1].src0) ++i;
  return sys[i];
}

template <typename R>
__device__ __forceinline__ cplx<R>* slot(void* base, int i, size_t vs) {
  return (cplx<R>*)base + i * vs;
}

// State reads: FRESH bypasses the scalar cache, needed when another block of
// the same (persistent) launch wrote the state.
template <bool FRESH, typename T>
__device__ __forceinline__ T rd(const T& x) {
  if constexpr (FRESH) return *(const volatile T*)&x;
  return x;
}

template <bool FRESH>
using StateRef = typename std::conditional<FRESH, volatile SrcState&, SrcState&>::type;

// Sources of a system in the given phase, as a bit mask (at most 64 sources).
template <bool FRESH>
__device__ __forceinline__ unsigned long long phase_bits(const SrcState* st, int nsrc, int phase) {
  unsigned long long m = 0;
  for (int k = 0; k < nsrc; ++k)
    if (rd<FRESH>(st[k].phase) == phase) m |= 1ull << k;
  return m;
}

template <int NBT>
__device__ __forceinline__ unsigned group_bits(unsigned long long m, int k0) {
  return (unsigned)(m >> k0) & ((1u << NBT) - 1u);
}

// Input of the FP64 residual stencil: x_hi + x_lo, the solution after the
// pending accumulation.
template <typename Rlo>
struct SumIn {
  const cplx<double>* __restrict__ hi;
  const cplx<Rlo>* __restrict__ lo;
  size_t ss, hv;
  int jmax;  // last readable slot (FieldIn)
  __device__ __forceinline__ cplx<double> operator()(int j, int c, int site) const {
    const int jj = j < jmax ? j : jmax;
    const cplx<double> a = ld_cplx<false>(hi + jj * ss + c * hv, (unsigned)site);
    const cplx<Rlo> b = ld_cplx<false>(lo + jj * ss + c * hv, (unsigned)site);
    return {a.re + (double)b.re, a.im + (double)b.im};
  }
};

// Sum over a 256-element vector tile of a per-element value: four chunks of
// 64 elements, chunk c taken by wavefront c % (waves of the block) and summed
// by one butterfly, the chunk sums added in chunk order.  The result (valid in
// thread 0) does not depend on the block size.  f(e) computes element e's
// value (and may update vectors); it is called once per element of the tile.
template <typename F>
__device__ __forceinline__ double tile_sum(int tile, size_t n, double* sh, F&& f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  for (int c = w; c < kVTile / 64; c += nw) {
    const size_t e = (size_t)tile * kVTile + c * 64 + lane;
    double v = e < n ? f(e) : 0.0;
    v = wave_sum(v);
    if (lane == 0) sh[c] = v;
  }
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int c = 0; c < kVTile / 64; ++c) t += sh[c];
  __syncthreads();
  return t;
}

// Sum of a[0..n) in an order that does not depend on the block size: 256
// virtual lanes, lane j adding a[j], a[j + 256], ... in turn, each virtual
// wavefront of 64 lanes reduced by one butterfly, the four wavefront sums
// added in order.  Every thread of the block calls it (the block is a whole
// number of wavefronts) and every thread gets the result.  sh: 4 doubles.
// A virtual lane's values are loaded 32 (then 8) at a time before they are
// added (in the same order), so that a lane has that many loads in flight.
__device__ __forceinline__ double lane_sum(const double* __restrict__ a, int i, int n) {
  double v = 0.0;
  for (; i + 31 * 256 < n; i += 32 * 256) {
    double t[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) t[u] = a[i + u * 256];
#pragma unroll
    for (int u = 0; u < 32; ++u) v += t[u];
  }
  for (; i + 7 * 256 < n; i += 8 * 256) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = a[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; i < n; i += 256) v += a[i];
  return v;
}

__device__ __forceinline__ double canon_sum(const double* __restrict__ a, int n, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  for (int vw = w; vw < 4; vw += nw) {
    double v = lane_sum(a, vw * 64 + lane, n);
    v = wave_sum(v);
    if (lane == 0) sh[vw] = v;
  }
  __syncthreads();
  const double t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return t;
}

// canon_sum of N arrays of n values at once (one pass over the arrays, one
// set of butterflies); out[k] is what canon_sum(a[k], n, .) would return.
// sh: 4 * N doubles.
template <int N>
__device__ __forceinline__ void canon_sum_n(const double* const (&a)[N], int n, double* sh,
                                            double (&out)[N]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  for (int vw = w; vw < 4; vw += nw) {
    double v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = 0.0;
    for (int i = vw * 64 + lane; i < n; i += 256)
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] += a[k][i];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double t = wave_sum(v[k]);
      if (lane == 0) sh[k * 4 + vw] = t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = ((sh[k * 4] + sh[k * 4 + 1]) + sh[k * 4 + 2]) + sh[k * 4 + 3];
  __syncthreads();
}

}  // namespace

// =================================================================== init

// x_lo = 0, p = 0 (and x_hi = 0 without an initial guess); partials of |b|^2.
template <typename R>
__global__ void __launch_bounds__(256) k_init(const SysDesc* __restrict__ sys, int nsys,
                                              int zero_xhi, int xcd) {
  __shared__ double sh[16];
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const size_t n = (size_t)3 * d.g.hv, vs = n * d.nsrc;
  cplx<R>* xlo = slot<R>(d.vlo, 0, vs) + k * n;
  cplx<R>* p = slot<R>(d.vlo, 2, vs) + k * n;
  cplx<double>* xhi = slot<double>(d.vhi, 0, vs) + k * n;
  const cplx<double>* bb = slot<double>(d.vhi, 2, vs) + k * n;
  const double t = tile_sum(tile, n, sh, [&](size_t e) {
    xlo[e] = {(R)0, (R)0};
    p[e] = {(R)0, (R)0};
    if (zero_xhi) xhi[e] = {0.0, 0.0};
    const cplx<double> bv = bb[e];
    return bv.re * bv.re + bv.im * bv.im;
  });
  if (threadIdx.x == 0) d.partials_v[(size_t)k * d.vtiles + tile] = t;
}

namespace {

// x_hi = 0 for zero sources (the solution of A x = 0).
__global__ void __launch_bounds__(256) k_zero_done(const SysDesc* __restrict__ sys, int nsys,
                                                   const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const size_t n = (size_t)3 * d.g.hv, e = (size_t)tile * kVTile + threadIdx.x;
  const SrcState& q = st[d.src0 + k];
  if (!(q.phase == PH_DONE && q.bnorm2 == 0.0) || e >= n) return;
  slot<double>(d.vhi, 0, n * d.nsrc)[k * n + e] = {0.0, 0.0};
}

}  // namespace

// ============================================================== finalize

enum FinKind : int { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_RU = 3, FIN_COMMIT = 4 };

// Total of the partials a reduction of the given kind left for source k: the
// stencil passes' (<p, Ap>, FP64 |r|^2) or the vector passes' (|b|^2, |r|^2).
__device__ __forceinline__ double partial_total(const SysDesc& d, int k, int kind, double* sh) {
  if (kind == FIN_ALPHA || kind == FIN_RU)
    return canon_sum(d.partials + (size_t)k * d.nblk, d.nblk, sh);
  return canon_sum(d.partials_v + (size_t)k * d.vtiles, d.vtiles, sh);
}

// Decisions taken from a reduction.  The finalize kernels apply them to the
// source state; the fused passes also act on them in every block, so both go
// through these functions.
struct AlphaStep {
  bool ok;       // <p, Ap> > 0 and finite; otherwise a breakdown
  double alpha;  // rho / <p, Ap>
};
__device__ __forceinline__ AlphaStep alpha_step(double rho, double pAp) {
  const bool ok = pAp > 0.0 && isfinite(pAp);
  return {ok, ok ? rho / pAp : 0.0};
}

enum BetaOutcome : int { BETA_GO = 0, BETA_UPDATE = 1, BETA_MAXED = 2, BETA_NONFINITE = 3 };
struct BetaStep {
  int outcome;
  double rmax;  // max |r| since the last update, including this one
  double beta;  // |r|^2 / rho when the recurrence goes on
};
// iters: the iteration count including this step.
__device__ __forceinline__ BetaStep beta_step(double t, int iters, int max_iter, double rmax,
                                              double stop2, double delta, double rho) {
  if (!isfinite(t)) return {BETA_NONFINITE, rmax, 0.0};
  const double rn = sqrt(t);
  const double rm = rn > rmax ? rn : rmax;
  if (iters >= max_iter) return {BETA_MAXED, rm, 0.0};
  if (t <= stop2 || rn < delta * rm) return {BETA_UPDATE, rm, 0.0};
  return {BETA_GO, rm, t / rho};
}

enum RuOutcome : int { RU_GO = 0, RU_CONVERGED = 1, RU_NONFINITE = 2, RU_STOP = 3 };
struct RuStep {
  int outcome;
  double beta;  // 0 after the initial residual, else |r_hi|^2 / rho
};
__device__ __forceinline__ RuStep ru_step(double t, double stop2, int reason, double rho) {
  if (t <= stop2) return {RU_CONVERGED, 0.0};
  if (!isfinite(t)) return {RU_NONFINITE, 0.0};
  if (reason == RU_FINAL) return {RU_STOP, 0.0};
  return {RU_GO, reason == RU_INIT ? 0.0 : t / rho};
}

// The state update of one source after a reduction (one thread).
template <bool FRESH>
__device__ __forceinline__ void finalize_source(int kind, StateRef<FRESH> q, double t) {
  switch (kind) {
    case FIN_INIT:  // |b|^2: a zero source is done (x = 0), a non-finite one broke down
      q.bnorm2 = t;
      q.stop2 = q.stop2 * t;
      if (t == 0.0) {
        q.phase = PH_DONE;
        q.status = kStatusOk;
        q.relres = 0.0;
      } else if (!isfinite(t)) {
        q.phase = PH_DONE;
        q.status = kStatusBreakdown;
        q.relres = t;
      }
      break;
    case FIN_ALPHA: {  // <p, Ap>: alpha, or a breakdown
      const AlphaStep a = alpha_step(q.rho, t);
      q.pAp = t;
      q.pend = 0;
      if (a.ok) {
        q.alpha = a.alpha;
      } else {
        q.phase = PH_RU;
        q.reason = RU_FINAL;
        q.status = kStatusBreakdown;
      }
      break;
    }
    case FIN_BETA: {  // |r|^2 of the recurrence: continue, update, or stop
      const int it = q.iters + 1;
      const BetaStep b = beta_step(t, it, q.max_iter, q.rmax, q.stop2, q.delta, q.rho);
      q.iters = it;
      q.rmax = b.rmax;
      if (b.outcome == BETA_GO) {
        q.beta = b.beta;
        q.rho = t;
        q.pend = 1;
      } else {
        q.phase = PH_RU;
        q.reason = b.outcome == BETA_UPDATE ? RU_DROP : RU_FINAL;
        if (b.outcome == BETA_MAXED) q.status = kStatusNotConverged;
        if (b.outcome == BETA_NONFINITE) q.status = kStatusBreakdown;
      }
      break;
    }
    case FIN_RU: {  // FP64 |b - A x|^2: converged, or restart the recurrence from it
      const RuStep r = ru_step(t, q.stop2, q.reason, q.rho);
      q.updates = q.updates + 1;
      q.relres = sqrt(t / q.bnorm2);
      if (r.outcome == RU_GO) {
        q.beta = r.beta;
        q.rho = t;
        q.rmax = sqrt(t);
        q.phase = PH_RU2;
      } else {
        q.phase = PH_DONE;
        if (r.outcome == RU_CONVERGED) q.status = kStatusOk;
        if (r.outcome == RU_NONFINITE) q.status = kStatusBreakdown;
      }
      break;
    }
    case FIN_COMMIT:  // a finished update lets the source iterate again
      q.phase = PH_RUN;
      q.pend = 0;
      break;
  }
}

__device__ __forceinline__ int fin_phase(int kind) {
  return kind == FIN_ALPHA || kind == FIN_BETA ? PH_RUN
         : kind == FIN_RU                      ? PH_RU
         : kind == FIN_COMMIT                  ? PH_RU2
                                               : -1;
}

// Finalize source g (global index) of the batch.
template <bool FRESH>
__device__ __forceinline__ void finalize_one(const SysDesc* __restrict__ sys, int nsys,
                                             SrcState* st, int g, int kind, double* sh) {
  const SysDesc& d = sys_of_source(sys, nsys, g);
  const int k = g - d.src0;
  const int ph = fin_phase(kind);
  if (ph >= 0 && rd<FRESH>(st[g].phase) != ph) return;
  const double t = kind != FIN_COMMIT ? partial_total(d, k, kind, sh) : 0.0;
  if (threadIdx.x == 0) {
    finalize_source<FRESH>(kind, st[g], t);
    // The x/r pass of these engines leaves x_lo += alpha p to the next p pass
    // (which reads p anyway) or to the next reliable update: pending after a
    // beta step, applied by the time of the next alpha step or update.
    StateRef<FRESH> q = st[g];
    if (kind == FIN_BETA) q.xpend = 1;
    if (kind == FIN_ALPHA || kind == FIN_RU) q.xpend = 0;
  }
}

namespace {

// One block per source of the batch.
__global__ void __launch_bounds__(256) k_finalize(const SysDesc* __restrict__ sys, int nsys,
                                                  SrcState* st, int kind) {
  __shared__ double sh[16];
  finalize_one<false>(sys, nsys, st, blockIdx.x, kind, sh);
}

hipError_t finalize(const EngineCfg& c, int kind, hipStream_t s) {
  QX_TIMED(c, kind == FIN_RU || kind == FIN_COMMIT ? PASS_UPDATE : PASS_FINALIZE, s,
           hipLaunchKernelGGL(k_finalize, dim3(c.nsrc_total), dim3(256), 0, s, c.d_sys, c.nsys,
                              c.d_st, kind));
  return hipGetLastError();
}

}  // namespace

// ============================================================== iteration
//
// The passes of an iteration are written per tile (a 64-site stencil tile or
// a 256-element vector tile) so that the same code serves the launch-per-pass
// kernels and the persistent kernel.

// E1: t = 2 D_oe p for running sources.
// LL: as in deo_tile, the source groups share the tile's links through LDS.
template <typename R, int RECON, int NBT, int LPS, bool FRESH, typename LS, bool LL = false>
__device__ __forceinline__ void doe_tile(const SysDesc* __restrict__ sys, int nsys,
                                         const SrcState* st, int b, int order) {
  static_assert(!LL || LPS == 1, "shared links need one wavefront per site");
  cplx<R>* red = reinterpret_cast<cplx<R>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id(), dp = w % LPS, grp = w / LPS;
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const SrcState* q0 = st + d.src0;
  const unsigned long long run = phase_bits<FRESH>(q0, d.nsrc, PH_RUN);
  if (!run) return;
  const int cb = tile_block(b - d.blk0, d.g, order) * kTile + lane;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  const int k0 = grp * NBT;
  const unsigned act = cb < d.g.hv ? group_bits<NBT>(run, k0) : 0u;
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  const cplx<R>* in = slot<R>(d.vlo, 2, vs) + k0 * ss;
  // x and y neighbours shuffled from the lanes that hold them while the
  // own-index values fit beside the hop's (six FP32 or two FP64 sources per thread)
  constexpr bool kXY = sizeof(cplx<R>) * NBT <= 48;
  if constexpr (LL) {
    const qx_u32x4* ll = reinterpret_cast<const qx_u32x4*>(qx_lds);
    Site s;
    site_geometry(d.g, 1, cb < d.g.hv ? cb : d.g.hv - 1, s);
    stage_links<RECON>(d.g, (const cplx<LS>*)d.links_lo, 1, cb < d.g.hv ? cb : d.g.hv - 1, s, w,
                       (int)(blockDim.x >> 6), reinterpret_cast<qx_u32x4*>(qx_lds), lane);
    __syncthreads();
    if (act) {
      if constexpr (kXY)
        stencil_part_ll<R, RECON, NBT>(
            d.g, (const cplx<LS>*)d.links_lo, cb, s,
            FieldInXY<R>{in, ss, hv, d.nsrc - 1 - k0, cb & ~(kTile - 1)}, ll, acc);
      else
        stencil_part_ll<R, RECON, NBT>(d.g, (const cplx<LS>*)d.links_lo, cb, s,
                                       FieldIn<R>{in, ss, hv, d.nsrc - 1 - k0}, ll, acc);
    }
  } else if (act) {
    Site s;
    site_geometry(d.g, 1, cb, s);
    if constexpr (kXY)
      stencil_part<R, RECON, NBT, LPS>(
          d.g, (const cplx<LS>*)d.links_lo, 1, cb, s, dp,
          FieldInXY<R>{in, ss, hv, d.nsrc - 1 - k0, cb & ~(kTile - 1)}, acc);
    else
      stencil_part<R, RECON, NBT, LPS>(d.g, (const cplx<LS>*)d.links_lo, 1, cb, s, dp,
                                       FieldIn<R>{in, ss, hv, d.nsrc - 1 - k0}, acc);
  }
  cplx<R>* t = slot<R>(d.vlo, 4, vs);
  const bool nt = order_nt(order);
  for_each_item<R, NBT, LPS>(acc, red, dp, grp, lane, [&](int j, int c, cplx<R> v) {
    if (act >> j & 1u) st_cplx(t + (k0 + j) * ss + c * hv + cb, v, nt);
  });
  if constexpr (LPS > 1) __syncthreads();  // the LDS buffer is reused by the next tile
}

// E2: Ap = m^2 p - 1/4 (2D_eo) t and the partials of Re<p, Ap>.
// LL (one wavefront per site, LPS 1): the block's source groups share the
// tile's link loads through LDS (stage_links), which then holds no reduction
// buffer.
template <typename R, int RECON, int NBT, int LPS, bool FRESH, typename LS, bool LL = false>
__device__ __forceinline__ void deo_tile(const SysDesc* __restrict__ sys, int nsys,
                                         const SrcState* st, int b, int order, int pslot,
                                         double* sh, double* tot) {
  static_assert(!LL || LPS == 1, "shared links need one wavefront per site");
  cplx<R>* red = reinterpret_cast<cplx<R>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id(), dp = w % LPS, grp = w / LPS;
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const SrcState* q0 = st + d.src0;
  const unsigned long long run = phase_bits<FRESH>(q0, d.nsrc, PH_RUN);
  if (!run) return;
  const int bl = tile_block(b - d.blk0, d.g, order), cb = bl * kTile + lane;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  const int k0 = grp * NBT;
  const unsigned act = cb < d.g.hv ? group_bits<NBT>(run, k0) : 0u;
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  const FieldIn<R> tin{slot<R>(d.vlo, 4, vs) + k0 * ss, ss, hv, d.nsrc - 1 - k0};
  if constexpr (LL) {
    const qx_u32x4* ll = reinterpret_cast<const qx_u32x4*>(qx_lds);
    Site s;
    site_geometry(d.g, 0, cb < d.g.hv ? cb : d.g.hv - 1, s);
    stage_links<RECON>(d.g, (const cplx<LS>*)d.links_lo, 0, cb < d.g.hv ? cb : d.g.hv - 1, s, w,
                       (int)(blockDim.x >> 6), reinterpret_cast<qx_u32x4*>(qx_lds), lane);
    __syncthreads();
    if (act) stencil_part_ll<R, RECON, NBT>(d.g, (const cplx<LS>*)d.links_lo, cb, s, tin, ll, acc);
  } else if (act) {
    Site s;
    site_geometry(d.g, 0, cb, s);
    stencil_part<R, RECON, NBT, LPS>(d.g, (const cplx<LS>*)d.links_lo, 0, cb, s, dp, tin, acc);
  }
  double dot[NBT];
#pragma unroll
  for (int j = 0; j < NBT; ++j) dot[j] = 0.0;
  const cplx<R>* p = slot<R>(d.vlo, pslot, vs);
  cplx<R>* Ap = slot<R>(d.vlo, 3, vs);
  const bool nt = order_nt(order);
  // p of every item the thread finishes, loaded before the slots' barriers
  const auto ld_p = [&](int j, int c) {
    return (act >> j & 1u) ? p[(k0 + j) * ss + c * hv + cb] : cplx<R>{(R)0, (R)0};
  };
  for_each_item_ld<R, NBT, LPS>(acc, red, dp, grp, lane, ld_p,
                                [&](int j, int c, cplx<R> v, cplx<R> pv) {
    if (!(act >> j & 1u)) return;
    const R m2 = (R)rd<FRESH>(q0[k0 + j].m2);
    const size_t i = (k0 + j) * ss + c * hv + cb;
    // one rounding (a quarter of v is exact), whatever the kernel contracts
    const cplx<R> r = {fmadd(m2, pv.re, (R)-0.25 * v.re), fmadd(m2, pv.im, (R)-0.25 * v.im)};
    st_cplx(Ap + i, r, nt);
    dot[j] += (double)pv.re * (double)r.re + (double)pv.im * (double)r.im;
  });
  const int G = (int)(blockDim.x >> 6) / LPS;
  group_sum<NBT>(dot, LPS, grp, dp, G, sh, tot);
  if (threadIdx.x == 0)
    for (int k = 0; k < d.nsrc; ++k) d.partials[(size_t)k * d.nblk + bl] = tot[k];
  __syncthreads();  // the shared scratch is reused by the next tile
}

// |v|^2 in FP64 (one expression for every x/r pass, so that they round alike).
template <typename R>
__device__ __forceinline__ double norm2_d(const cplx<R>& v) {
  return (double)v.re * (double)v.re + (double)v.im * (double)v.im;
}

// x_lo += alpha p, r -= alpha Ap over vector tile `tile` of source k of a
// system, and the partial of |r|^2.  Works for any block size.
// (UPDATE_X false: r only; x_lo += alpha p is left pending, SrcState::xpend.)
template <typename R, bool UPDATE_X>
__device__ __forceinline__ void xr_body(const SysDesc& d, int k, int tile, R al, int pslot,
                                        double* sh) {
  const size_t n = (size_t)3 * d.g.hv, vs = n * d.nsrc;
  cplx<R>* x = slot<R>(d.vlo, 0, vs) + k * n;
  cplx<R>* r = slot<R>(d.vlo, 1, vs) + k * n;
  const cplx<R>* p = slot<R>(d.vlo, pslot, vs) + k * n;
  const cplx<R>* Ap = slot<R>(d.vlo, 3, vs) + k * n;
  const double t = tile_sum(tile, n, sh, [&](size_t e) {
    const unsigned u = (unsigned)e;
    const cplx<R> av = ld_cplx<false>(Ap, u);
    cplx<R> rv = ld_cplx<false>(r, u);
    if constexpr (UPDATE_X) {
      const cplx<R> pv = ld_cplx<false>(p, u);
      cplx<R> xv = ld_cplx<false>(x, u);
      xv.re = fma(al, pv.re, xv.re);
      xv.im = fma(al, pv.im, xv.im);
      st_cplx(x + e, xv, false);
    }
    rv.re = fma(-al, av.re, rv.re);
    rv.im = fma(-al, av.im, rv.im);
    st_cplx(r + e, rv, false);
    return norm2_d(rv);
  });
  if (threadIdx.x == 0) d.partials_v[(size_t)k * d.vtiles + tile] = t;
}

// p = r + beta p over vector tile `tile` of source k, after x_lo += alpha p
// with the old p when the last x/r step left it pending (xp).  Works for any
// block size.
template <typename R>
__device__ __forceinline__ void p_body(const SysDesc& d, int k, int tile, R be, bool xp, R al) {
  const size_t n = (size_t)3 * d.g.hv, vs = n * d.nsrc;
  const cplx<R>* r = slot<R>(d.vlo, 1, vs) + k * n;
  cplx<R>* p = slot<R>(d.vlo, 2, vs) + k * n;
  cplx<R>* x = slot<R>(d.vlo, 0, vs) + k * n;
  for (int t = threadIdx.x; t < kVTile; t += blockDim.x) {
    const size_t e = (size_t)tile * kVTile + t;
    if (e >= n) break;
    const unsigned u = (unsigned)e;
    const cplx<R> rv = ld_cplx<false>(r, u), pv = ld_cplx<false>(p, u);
    if (xp) {
      cplx<R> xv = ld_cplx<false>(x, u);
      xv.re = fma(al, pv.re, xv.re);
      xv.im = fma(al, pv.im, xv.im);
      st_cplx(x + e, xv, false);
    }
    st_cplx(p + e, cplx<R>{fma(be, pv.re, rv.re), fma(be, pv.im, rv.im)}, false);
  }
}

// E3: x_lo += alpha p, r -= alpha Ap and the partials of |r|^2, for running sources.
template <typename R, bool FRESH>
__device__ __forceinline__ void xr_tile(const SysDesc* __restrict__ sys, int nsys,
                                        const SrcState* st, int b, double* sh) {
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  if (rd<FRESH>(st[d.src0 + k].phase) != PH_RUN) return;
  xr_body<R, false>(d, k, tile, (R)rd<FRESH>(st[d.src0 + k].alpha), 2, sh);
}

// E0: p = r + beta p for running sources whose search direction the previous
// iteration left pending.
template <typename R, bool FRESH>
__device__ __forceinline__ void p_tile(const SysDesc* __restrict__ sys, int nsys,
                                       const SrcState* st, int b) {
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const SrcState& q = st[d.src0 + k];
  if (rd<FRESH>(q.phase) != PH_RUN || !rd<FRESH>(q.pend)) return;
  p_body<R>(d, k, tile, (R)rd<FRESH>(q.beta), rd<FRESH>(q.xpend) != 0, (R)rd<FRESH>(q.alpha));
}

// The p pass of the launch-per-pass engine: one wavefront per vector tile,
// four elements per lane with all their loads issued before the stores (the
// arithmetic of p_body).
template <typename R>
__global__ void __launch_bounds__(64) k_iter_p(const SysDesc* __restrict__ sys, int nsys,
                                               const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const SrcState& q = st[d.src0 + k];
  if (q.phase != PH_RUN || !q.pend) return;
  const bool xp = q.xpend != 0;
  const R be = (R)q.beta, al = (R)q.alpha;
  const size_t n = (size_t)3 * d.g.hv, vs = n * d.nsrc;
  const cplx<R>* r = slot<R>(d.vlo, 1, vs) + k * n;
  cplx<R>* p = slot<R>(d.vlo, 2, vs) + k * n;
  cplx<R>* x = slot<R>(d.vlo, 0, vs) + k * n;
  constexpr int U = kVTile / 64;
  const unsigned e0 = (unsigned)tile * kVTile + threadIdx.x;
  // elements past n (the last tile of a source) read and write nothing
  const unsigned last = (unsigned)n - 1;
  cplx<R> rv[U], pv[U], xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const unsigned e = e0 + 64 * u, ec = e < last ? e : last;
    rv[u] = ld_cplx<false>(r, ec);
    pv[u] = ld_cplx<false>(p, ec);
    xv[u] = xp ? ld_cplx<false>(x, ec) : cplx<R>{(R)0, (R)0};
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const unsigned e = e0 + 64 * u;
    if (e > last) break;
    if (xp) {
      cplx<R> xn = xv[u];
      xn.re = fma(al, pv[u].re, xn.re);
      xn.im = fma(al, pv[u].im, xn.im);
      st_cplx(x + e, xn, false);
    }
    st_cplx(p + e, cplx<R>{fma(be, pv[u].re, rv[u].re), fma(be, pv[u].im, rv[u].im)}, false);
  }
}

template <typename R, int RECON, int NBT, int LPS, typename LS, bool LL = false>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>)) k_iter_doe(const SysDesc* __restrict__ sys,
                                                                    int nsys, const SrcState* st,
                                                                    int xcd) {
  doe_tile<R, RECON, NBT, LPS, false, LS, LL>(sys, nsys, st, logical_block(xcd), xcd);
}

template <typename R, int RECON, int NBT, int LPS, typename LS>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>)) k_iter_deo(const SysDesc* __restrict__ sys,
                                                                    int nsys, const SrcState* st,
                                                                    int pslot, int xcd) {
  __shared__ double sh[16 * 64];
  __shared__ double tot[64];
  deo_tile<R, RECON, NBT, LPS, false, LS>(sys, nsys, st, logical_block(xcd), xcd, pslot, sh, tot);
}

// Dynamic LDS of k_iter_deo_ll for G source groups of NBT: the staged links,
// then the group sums' 16 and 1 doubles per source of the block.
template <int RECON, typename LS>
inline size_t deo_ll_lds(int G, int NBT) {
  return kLinkLdsBytes<RECON, LS> + (size_t)G * NBT * 17 * sizeof(double);
}

// k_iter_deo with one wavefront per site and several source groups, which
// share the tile's link loads through LDS.
template <typename R, int RECON, int NBT, typename LS>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>)) k_iter_deo_ll(
    const SysDesc* __restrict__ sys, int nsys, const SrcState* st, int pslot, int xcd) {
  double* sh = reinterpret_cast<double*>(reinterpret_cast<char*>(qx_lds) +
                                         kLinkLdsBytes<RECON, LS>);
  const int ns = (int)(blockDim.x >> 6) * NBT;
  deo_tile<R, RECON, NBT, 1, false, LS, true>(sys, nsys, st, logical_block(xcd), xcd, pslot, sh,
                                              sh + 16 * ns);
}

// The x/r pass of the launch-per-pass engine (x_lo += alpha p deferred): one
// wavefront per vector tile, four elements per lane with their loads issued
// together; the tile's |r|^2 partial is tile_sum's (a butterfly per 64
// elements, the four added in order), so it matches xr_body bit for bit.
template <typename R>
__global__ void __launch_bounds__(64) k_iter_xr(const SysDesc* __restrict__ sys, int nsys,
                                                const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const SrcState& q = st[d.src0 + k];
  if (q.phase != PH_RUN) return;
  const R al = (R)q.alpha;
  const size_t n = (size_t)3 * d.g.hv, vs = n * d.nsrc;
  cplx<R>* r = slot<R>(d.vlo, 1, vs) + k * n;
  const cplx<R>* Ap = slot<R>(d.vlo, 3, vs) + k * n;
  constexpr int U = kVTile / 64;
  const unsigned e0 = (unsigned)tile * kVTile + threadIdx.x, last = (unsigned)n - 1;
  cplx<R> av[U], rv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const unsigned e = e0 + 64 * u, ec = e < last ? e : last;
    av[u] = ld_cplx<false>(Ap, ec);
    rv[u] = ld_cplx<false>(r, ec);
  }
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const unsigned e = e0 + 64 * u;
    cplx<R> rn = rv[u];
    rn.re = fma(-al, av[u].re, rn.re);
    rn.im = fma(-al, av[u].im, rn.im);
    v[u] = 0.0;
    if (e <= last) {
      st_cplx(r + e, rn, false);
      v[u] = norm2_d(rn);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = wave_sum(v[u]);
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[u];
    d.partials_v[(size_t)k * d.vtiles + tile] = t;
  }
}

// ------------------------------------------------- fused launch sequence
//
// With few partials per source (small lattices) the two finalize launches of
// an iteration and three of a reliable update are folded into the vector
// pass that follows them: every block of a source adds the source's partials
// itself (canon_sum: the same sum, in the same order, in every block and in
// k_finalize), applies the state update to a private copy and acts on it.
// The source's first vector tile writes the updated state to the other of two
// state slots (st_out); every kernel of the launch reads only the slot the
// previous launches wrote (st_in), so no block reads a state another block of
// the same launch is writing.  An iteration is k_fiter_doe (slot 0 -> 1, with
// the p update of the previous step folded in: p alternates between two
// vector slots so that the neighbours read the old p while a block writes the
// new one), k_iter_deo (reading slot 1), k_fiter_xr (slot 1 -> 0); a reliable
// update is k_ru_doe (slot 0), k_ru_residual (copying slot 0 -> 1),
// k_fru_finish (slot 1 -> 0).  Sources start and end each iteration and each
// update in slot 0, as the other engines keep them; p is in vector slot 2
// after every even number of iterations, where updates happen.

// The state written by the designated thread of a fused pass: a copy of the
// source's state with the reduction applied (the same update k_finalize
// makes), plus the fused-sequence flags.
template <int KIND>
__device__ __forceinline__ void write_state(const SrcState& in, SrcState* out, bool apply,
                                            double t, int have_rr) {
  *out = in;
  if (apply) finalize_source<false>(KIND, *out, t);
  if (KIND == FIN_RU && out->phase == PH_RU2) finalize_source<false>(FIN_COMMIT, *out, 0.0);
  out->pend = 0;
  out->have_rr = have_rr;
}

// Stencil input of the fused D_oe pass: r + beta_j p at the neighbours for
// sources whose p update is due (bit j of upd), else p, in the same
// arithmetic as p_body.
template <typename R, int NBT>
struct PendIn {
  const cplx<R>* __restrict__ r;  // first source of the thread
  const cplx<R>* __restrict__ p;
  size_t ss, hv;
  int jmax;  // last readable slot (FieldIn)
  unsigned upd;
  R beta[NBT];
  // both vectors are loaded for every slot (no branch between the loads)
  __device__ __forceinline__ cplx<R> operator()(int j, int c, int site) const {
    const int jj = j < jmax ? j : jmax;
    const cplx<R> pv = ld_cplx<false>(p + jj * ss + c * hv, (unsigned)site);
    const cplx<R> rv = ld_cplx<false>(r + jj * ss + c * hv, (unsigned)site);
    const cplx<R> n = {fma(beta[j], pv.re, rv.re), fma(beta[j], pv.im, rv.im)};
    return (upd >> j & 1u) ? n : pv;
  }
};

// F1: the beta step of the last x/r update folded into the D_oe pass.  Every
// block adds each stepping source's |r|^2 partials and takes the decision of
// k_finalize; it then writes p_new = r + beta p (or a copy of p, for sources
// that keep p: fresh after an update, or waiting for one) at its own even
// sites into slot pout, and computes t = 2 D_oe p_new for running sources
// with p_new formed on the fly at the neighbours from slot pin.  The system's
// first block writes the updated states (slot st_out).
template <typename R, int RECON, int NBT, int LPS, typename LS>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>))
    k_fiter_doe(const SysDesc* __restrict__ sys, int nsys, const SrcState* __restrict__ st_in,
                SrcState* __restrict__ st_out, int pin, int pout, int xcd) {
  __shared__ double sh[4];
  __shared__ double beta_sh[64], t_sh[64];
  cplx<R>* red = reinterpret_cast<cplx<R>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id(), dp = w % LPS, grp = w / LPS;
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const SrcState* q0 = st_in + d.src0;
  // decisions, the same in every block: run (stencil), upd (p = r + beta p),
  // keep (p copied), step (the beta step was taken)
  unsigned long long run = 0, upd = 0, keep = 0, step = 0;
  for (int k = 0; k < d.nsrc; ++k) {
    const SrcState& q = q0[k];
    double t = 0.0, be = 0.0;
    if (q.phase == PH_RUN && q.have_rr) {
      t = canon_sum(d.partials_v + (size_t)k * d.vtiles, d.vtiles, sh);
      const BetaStep bs = beta_step(t, q.iters + 1, q.max_iter, q.rmax, q.stop2, q.delta, q.rho);
      step |= 1ull << k;
      if (bs.outcome == BETA_GO) {
        run |= 1ull << k;
        upd |= 1ull << k;
        be = bs.beta;
      } else {
        keep |= 1ull << k;
      }
    } else if (q.phase == PH_RUN) {
      run |= 1ull << k;
      keep |= 1ull << k;
    } else if (q.phase == PH_RU) {
      keep |= 1ull << k;
    }
    if (threadIdx.x == 0) {
      beta_sh[k] = be;
      t_sh[k] = t;
    }
  }
  __syncthreads();
  if (b == d.blk0)
    for (int k = threadIdx.x; k < d.nsrc; k += blockDim.x) {
      const bool sk = step >> k & 1ull;
      write_state<FIN_BETA>(q0[k], st_out + d.src0 + k, sk, t_sh[k], sk ? 0 : q0[k].have_rr);
    }
  if (!(run | keep)) return;
  const int cb = tile_block(b - d.blk0, d.g, xcd) * kTile + lane;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  const int k0 = grp * NBT;
  const bool in_range = cb < d.g.hv;
  const cplx<R>* p_in = slot<R>(d.vlo, pin, vs);
  const cplx<R>* r_in = slot<R>(d.vlo, 1, vs);
  PendIn<R, NBT> src{r_in + k0 * ss, p_in + k0 * ss, ss, hv, d.nsrc - 1 - k0,
                     group_bits<NBT>(upd, k0), {}};
#pragma unroll
  for (int j = 0; j < NBT; ++j) src.beta[j] = k0 + j < d.nsrc ? (R)beta_sh[k0 + j] : (R)0;
  // p_new at the block's own even sites
  if (dp == 0 && in_range) {
    cplx<R>* p_out = slot<R>(d.vlo, pout, vs);
    const unsigned mine = group_bits<NBT>(upd | keep, k0);
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (!(mine >> j & 1u)) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) p_out[(k0 + j) * ss + c * hv + cb] = src(j, c, cb);
    }
  }
  if (!run) return;
  const unsigned act = in_range ? group_bits<NBT>(run, k0) : 0u;
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  if (act) {
    Site s;
    site_geometry(d.g, 1, cb, s);
    stencil_part<R, RECON, NBT, LPS>(d.g, (const cplx<LS>*)d.links_lo, 1, cb, s, dp, src, acc);
  }
  cplx<R>* t = slot<R>(d.vlo, 4, vs);
  const bool nt = order_nt(xcd);
  for_each_item<R, NBT, LPS>(acc, red, dp, grp, lane, [&](int j, int c, cplx<R> v) {
    if (act >> j & 1u) st_cplx(t + (k0 + j) * ss + c * hv + cb, v, nt);
  });
}

// F3: the alpha step from the <p, Ap> partials (or a breakdown), then
// x_lo += alpha p, r -= alpha Ap and the |r|^2 partials.
template <typename R>
__global__ void __launch_bounds__(256) k_fiter_xr(const SysDesc* __restrict__ sys, int nsys,
                                                  const SrcState* __restrict__ st_in,
                                                  SrcState* __restrict__ st_out, int pslot,
                                                  int xcd) {
  __shared__ double sh[16];
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const int g = d.src0 + k;
  const SrcState& q = st_in[g];
  const bool run = q.phase == PH_RUN;
  double t = 0.0;
  AlphaStep as{false, 0.0};
  if (run) {
    t = canon_sum(d.partials + (size_t)k * d.nblk, d.nblk, sh);
    as = alpha_step(q.rho, t);
  }
  const bool go = run && as.ok;
  if (tile == 0 && threadIdx.x == 0) write_state<FIN_ALPHA>(q, st_out + g, run, t, go ? 1 : q.have_rr);
  if (go) xr_body<R, true>(d, k, tile, (R)as.alpha, pslot, sh);
}

// R3 fused: the FP64 residual step (converged, broken down, or restart the
// recurrence), then r = lo(r_hi), p = r + beta p for sources that go on.
template <typename R>
__global__ void __launch_bounds__(256) k_fru_finish(const SysDesc* __restrict__ sys, int nsys,
                                                    const SrcState* __restrict__ st_in,
                                                    SrcState* __restrict__ st_out, int xcd) {
  __shared__ double sh[4];
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_vblock(sys, nsys, b);
  const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
  const int g = d.src0 + k;
  const SrcState& q = st_in[g];
  const bool ru = q.phase == PH_RU;
  double t = 0.0;
  RuStep rs{RU_STOP, 0.0};
  if (ru) {
    t = canon_sum(d.partials + (size_t)k * d.nblk, d.nblk, sh);
    rs = ru_step(t, q.stop2, q.reason, q.rho);
  }
  if (tile == 0 && threadIdx.x == 0) write_state<FIN_RU>(q, st_out + g, ru, t, ru ? 0 : q.have_rr);
  if (!(ru && rs.outcome == RU_GO)) return;
  const size_t n = (size_t)3 * d.g.hv, vs = n * d.nsrc;
  const R be = (R)rs.beta;
  const cplx<double>* rhi = slot<double>(d.vhi, 1, vs) + k * n;
  cplx<R>* r = slot<R>(d.vlo, 1, vs) + k * n;
  cplx<R>* p = slot<R>(d.vlo, 2, vs) + k * n;
  for (int e0 = threadIdx.x; e0 < kVTile; e0 += blockDim.x) {
    const size_t e = (size_t)tile * kVTile + e0;
    if (e >= n) break;
    const cplx<double> h = rhi[e];
    const cplx<R> rv = {(R)h.re, (R)h.im}, pv = p[e];
    r[e] = rv;
    p[e] = {fma(be, pv.re, rv.re), fma(be, pv.im, rv.im)};
  }
}

// ------------------------------------------ two-launch fused sequence
//
// k_f2_doe (states slot 0 -> 1) and k_f2_deo (slot 1 -> 0).  The D_eo pass
// leaves four partial sums per source: <p, Ap>, Re<r, Ap>, |Ap|^2 and |r|^2
// of the stored r.  The next D_oe pass adds them in every block, takes the
// alpha step with that |r|^2, forms
// |r - alpha Ap|^2 = |r|^2 - 2 alpha Re<r, Ap> + alpha^2 |Ap|^2 and takes the
// beta step from it (the expansion is taken one step at a time from the
// stored r's norm, so its cancellation error does not accumulate); each block then updates x, r and p at its own even sites
// (r and p alternate between two vector slots each, so that the neighbours
// read the old values while a block writes the new ones) and computes
// t = 2 D_oe p_new with p_new formed on the fly at the neighbours.  The x/r
// pass and its reduction of the three-launch sequence disappear; |r|^2 comes
// from the expansion instead of a sum over the stored r, so the rounding (not
// the mathematics) differs from the other engines.  Reliable updates are the
// fused sequence's.

// Stencil input of k_f2_doe: p_new = (r - alpha Ap) + beta p at the
// neighbours for sources whose step is due (bits j of sub and upd), r + beta p
// for sources restarting after a reliable update (upd only), else p; the same
// arithmetic as the own-site updates.
template <typename R, int NBT>
struct StepIn {
  const cplx<R>* __restrict__ r;  // first source of the thread
  const cplx<R>* __restrict__ ap;
  const cplx<R>* __restrict__ p;
  size_t ss, hv;
  int jmax;  // last readable slot (FieldIn)
  unsigned upd, sub;
  R alpha[NBT], beta[NBT];
  // the three vectors are loaded for every slot (no branch between the loads)
  __device__ __forceinline__ cplx<R> operator()(int j, int c, int site) const {
    const int jj = j < jmax ? j : jmax;
    const cplx<R> pv = ld_cplx<false>(p + jj * ss + c * hv, (unsigned)site);
    const cplx<R> rv = ld_cplx<false>(r + jj * ss + c * hv, (unsigned)site);
    const cplx<R> av = ld_cplx<false>(ap + jj * ss + c * hv, (unsigned)site);
    const cplx<R> rs = {fma(-alpha[j], av.re, rv.re), fma(-alpha[j], av.im, rv.im)};
    const cplx<R> rn = (sub >> j & 1u) ? rs : rv;
    const cplx<R> n = {fma(beta[j], pv.re, rn.re), fma(beta[j], pv.im, rn.im)};
    return (upd >> j & 1u) ? n : pv;
  }
};

// |r - alpha Ap|^2 from |r|^2 = rho and the partial sums of Re<r, Ap> and
// |Ap|^2; a value rounded below zero (a residual that vanished) is zero.
__device__ __forceinline__ double next_rho(double rho, double alpha, double rap, double apap) {
  const double t = rho - 2.0 * alpha * rap + alpha * alpha * apap;
  return t < 0.0 ? 0.0 : t;
}

template <typename R, int RECON, int NBT, int LPS, typename LS>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>))
    k_f2_doe(const SysDesc* __restrict__ sys, int nsys, const SrcState* __restrict__ st_in,
             SrcState* __restrict__ st_out, int pin, int pout, int rin, int rout, int xcd) {
  __shared__ double sh[16];
  __shared__ double al_sh[64], be_sh[64], pap_sh[64], t_sh[64], rho_sh[64];
  __shared__ int code_sh[64];
  cplx<R>* red = reinterpret_cast<cplx<R>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id(), dp = w % LPS, grp = w / LPS;
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const SrcState* q0 = st_in + d.src0;
  // decisions, the same in every block: run (stencil), step (x and r
  // updated), upd (p = r_new + beta p), keep (p and r copied); a source whose
  // reliable update left its FP64 |r|^2 partials (PH_RU with have_rr) takes
  // the update's last step here (converged, stopped, or restart with
  // p = lo(r_hi) + beta p, lo(r_hi) already in the r slot)
  unsigned long long run = 0, step = 0, upd = 0, keep = 0;
  for (int k = 0; k < d.nsrc; ++k) {
    const SrcState& q = q0[k];
    const unsigned long long bit = 1ull << k;
    double al = 0.0, be = 0.0, pap = 0.0, t = 0.0, rho = q.rho;
    int code = 0;  // 1: the alpha step failed (breakdown), 2: alpha and beta steps taken,
                   // 3: a reliable update finished here
    if (q.phase == PH_RU && q.have_rr) {
      t = canon_sum(d.partials + (size_t)k * d.nblk, d.nblk, sh);
      const RuStep rs = ru_step(t, q.stop2, q.reason, q.rho);
      code = 3;
      if (rs.outcome == RU_GO) {
        run |= bit;
        upd |= bit;
        be = rs.beta;
      }
    } else if (q.phase == PH_RUN && q.have_rr) {
      const double* const parts[4] = {d.partials + (size_t)k * d.nblk,
                                      d.partials_x + (size_t)k * d.nblk,
                                      d.partials_x + (size_t)(d.nsrc + k) * d.nblk,
                                      d.partials_x + (size_t)(2 * d.nsrc + k) * d.nblk};
      double sums[4];
      canon_sum_n<4>(parts, d.nblk, sh, sums);
      pap = sums[0];
      const double rap = sums[1], apap = sums[2];
      rho = sums[3];
      const AlphaStep as = alpha_step(rho, pap);
      if (as.ok) {
        al = as.alpha;
        t = next_rho(rho, al, rap, apap);
        const BetaStep bs = beta_step(t, q.iters + 1, q.max_iter, q.rmax, q.stop2, q.delta, rho);
        code = 2;
        step |= bit;
        if (bs.outcome == BETA_GO) {
          run |= bit;
          upd |= bit;
          be = bs.beta;
        } else {
          keep |= bit;
        }
      } else {
        code = 1;
        keep |= bit;
      }
    } else if (q.phase == PH_RUN) {
      run |= bit;
      keep |= bit;
    } else if (q.phase == PH_RU) {
      keep |= bit;
    }
    if (threadIdx.x == 0) {
      al_sh[k] = al;
      be_sh[k] = be;
      pap_sh[k] = pap;
      t_sh[k] = t;
      rho_sh[k] = rho;
      code_sh[k] = code;
    }
  }
  __syncthreads();
  if (b == d.blk0)
    for (int k = threadIdx.x; k < d.nsrc; k += blockDim.x) {
      SrcState q = q0[k];
      if (code_sh[k] == 3) {
        finalize_source<false>(FIN_RU, q, t_sh[k]);
        if (q.phase == PH_RU2) finalize_source<false>(FIN_COMMIT, q, 0.0);
      }
      if (code_sh[k] == 1 || code_sh[k] == 2) q.rho = rho_sh[k];  // |r|^2 of the stored r
      if (code_sh[k] == 1 || code_sh[k] == 2) finalize_source<false>(FIN_ALPHA, q, pap_sh[k]);
      if (code_sh[k] == 2) finalize_source<false>(FIN_BETA, q, t_sh[k]);
      q.pend = 0;
      q.have_rr = (run >> k & 1ull) ? 1 : 0;  // the D_eo pass leaves its partial sums
      st_out[d.src0 + k] = q;
    }
  if (!(run | step | keep)) return;
  const int cb = tile_block(b - d.blk0, d.g, xcd) * kTile + lane;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  const int k0 = grp * NBT;
  const bool in_range = cb < d.g.hv;
  const cplx<R>* r_in = slot<R>(d.vlo, rin, vs);
  const cplx<R>* ap = slot<R>(d.vlo, 3, vs);
  const cplx<R>* p_in = slot<R>(d.vlo, pin, vs);
  StepIn<R, NBT> src{r_in + k0 * ss, ap + k0 * ss, p_in + k0 * ss, ss, hv, d.nsrc - 1 - k0,
                     group_bits<NBT>(upd, k0), group_bits<NBT>(step, k0), {}, {}};
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    src.alpha[j] = k0 + j < d.nsrc ? (R)al_sh[k0 + j] : (R)0;
    src.beta[j] = k0 + j < d.nsrc ? (R)be_sh[k0 + j] : (R)0;
  }
  // x, r and p at the block's own even sites
  if (dp == 0 && in_range) {
    cplx<R>* x = slot<R>(d.vlo, 0, vs);
    cplx<R>* r_out = slot<R>(d.vlo, rout, vs);
    cplx<R>* p_out = slot<R>(d.vlo, pout, vs);
    const unsigned gs = group_bits<NBT>(step, k0), gu = group_bits<NBT>(upd, k0);
    const unsigned gk = group_bits<NBT>(keep, k0);
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (!((gs | gk | gu) >> j & 1u)) continue;
      const R al = src.alpha[j], be = src.beta[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const size_t i = (k0 + j) * ss + c * hv + cb;
        const cplx<R> pv = p_in[i];
        cplx<R> rv = r_in[i];
        if (gs >> j & 1u) {
          const cplx<R> av = ap[i];
          cplx<R> xv = x[i];
          xv.re = fma(al, pv.re, xv.re);
          xv.im = fma(al, pv.im, xv.im);
          x[i] = xv;
          rv = {fma(-al, av.re, rv.re), fma(-al, av.im, rv.im)};
        }
        r_out[i] = rv;
        p_out[i] = (gu >> j & 1u) ? cplx<R>{fma(be, pv.re, rv.re), fma(be, pv.im, rv.im)} : pv;
      }
    }
  }
  if (!run) return;
  const unsigned act = in_range ? group_bits<NBT>(run, k0) : 0u;
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  if (act) {
    Site s;
    site_geometry(d.g, 1, cb, s);
    stencil_part<R, RECON, NBT, LPS>(d.g, (const cplx<LS>*)d.links_lo, 1, cb, s, dp, src, acc);
  }
  cplx<R>* t = slot<R>(d.vlo, 4, vs);
  const bool nt = order_nt(xcd);
  for_each_item<R, NBT, LPS>(acc, red, dp, grp, lane, [&](int j, int c, cplx<R> v) {
    if (act >> j & 1u) st_cplx(t + (k0 + j) * ss + c * hv + cb, v, nt);
  });
}

// Ap = m^2 p - 1/4 (2D_eo) t and the partials of <p, Ap>, Re<r, Ap>, |Ap|^2
// and |r|^2 for running sources; the system's first block copies the states
// from slot 1 (st_in) to slot 0.
template <typename R, int RECON, int NBT, int LPS, typename LS>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>))
    k_f2_deo(const SysDesc* __restrict__ sys, int nsys, const SrcState* __restrict__ st_in,
             SrcState* __restrict__ st_out, int pslot, int rslot, int xcd) {
  __shared__ double sh[16 * 64];
  __shared__ double tot[4][64];
  cplx<R>* red = reinterpret_cast<cplx<R>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id(), dp = w % LPS, grp = w / LPS;
  const int b = logical_block(xcd);
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const SrcState* q0 = st_in + d.src0;
  if (b == d.blk0)
    for (int k = threadIdx.x; k < d.nsrc; k += blockDim.x) st_out[d.src0 + k] = q0[k];
  const unsigned long long run = phase_bits<false>(q0, d.nsrc, PH_RUN);
  if (!run) return;
  const int bl = tile_block(b - d.blk0, d.g, xcd), cb = bl * kTile + lane;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  const int k0 = grp * NBT;
  const unsigned act = cb < d.g.hv ? group_bits<NBT>(run, k0) : 0u;
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  if (act) {
    Site s;
    site_geometry(d.g, 0, cb, s);
    stencil_part<R, RECON, NBT, LPS>(
        d.g, (const cplx<LS>*)d.links_lo, 0, cb, s, dp,
        FieldIn<R>{slot<R>(d.vlo, 4, vs) + k0 * ss, ss, hv, d.nsrc - 1 - k0}, acc);
  }
  double dpa[NBT], dra[NBT], daa[NBT], drr[NBT];
#pragma unroll
  for (int j = 0; j < NBT; ++j) dpa[j] = dra[j] = daa[j] = drr[j] = 0.0;
  const cplx<R>* p = slot<R>(d.vlo, pslot, vs);
  const cplx<R>* r = slot<R>(d.vlo, rslot, vs);
  cplx<R>* Ap = slot<R>(d.vlo, 3, vs);
  const bool nt = order_nt(xcd);
  // p and r of every item the thread finishes, loaded before the slots' barriers
  struct PR {
    cplx<R> p, r;
  };
  const auto ld_pr = [&](int j, int c) {
    const size_t i = (k0 + j) * ss + c * hv + cb;
    return (act >> j & 1u) ? PR{p[i], r[i]} : PR{{(R)0, (R)0}, {(R)0, (R)0}};
  };
  for_each_item_ld<R, NBT, LPS>(acc, red, dp, grp, lane, ld_pr,
                                [&](int j, int c, cplx<R> v, PR pr) {
    if (!(act >> j & 1u)) return;
    const R m2 = (R)q0[k0 + j].m2;
    const size_t i = (k0 + j) * ss + c * hv + cb;
    const cplx<R> pv = pr.p, rv = pr.r;
    const cplx<R> a = {fmadd(m2, pv.re, (R)-0.25 * v.re), fmadd(m2, pv.im, (R)-0.25 * v.im)};
    st_cplx(Ap + i, a, nt);
    dpa[j] += (double)pv.re * (double)a.re + (double)pv.im * (double)a.im;
    dra[j] += (double)rv.re * (double)a.re + (double)rv.im * (double)a.im;
    daa[j] += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
    drr[j] += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
  });
  const int G = (int)(blockDim.x >> 6) / LPS;
  group_sum<NBT>(dpa, LPS, grp, dp, G, sh, tot[0]);
  group_sum<NBT>(dra, LPS, grp, dp, G, sh, tot[1]);
  group_sum<NBT>(daa, LPS, grp, dp, G, sh, tot[2]);
  group_sum<NBT>(drr, LPS, grp, dp, G, sh, tot[3]);
  if (threadIdx.x == 0)
    for (int k = 0; k < d.nsrc; ++k) {
      d.partials[(size_t)k * d.nblk + bl] = tot[0][k];
      d.partials_x[(size_t)k * d.nblk + bl] = tot[1][k];
      d.partials_x[(size_t)(d.nsrc + k) * d.nblk + bl] = tot[2][k];
      d.partials_x[(size_t)(2 * d.nsrc + k) * d.nblk + bl] = tot[3][k];
    }
}

// ------------------------------------------------------- persistent kernel
//
// One cooperative launch runs up to `iters` iterations of every system: each
// pass is a grid-stride loop over tiles (or sources, for the finalize passes)
// followed by a grid barrier.  The barrier is a generation counter at agent
// scope; a wait gives up after `timeout` ticks of the constant-rate device
// clock and raises the error word, so that every block leaves the kernel.
// The loop ends when no source is running or one waits for a reliable update
// (the host then runs the update), a decision every block takes from the same
// state after a barrier.  Each barrier costs every block an agent-scope
// release and acquire; the launch-per-pass engine is the default.

__device__ __forceinline__ bool grid_sync(GridSync* gs, unsigned nblocks, long long timeout,
                                          int* ok_sh) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();  // release this block's writes
    const unsigned arrived =
        __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1u) {
      __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&gs->gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // poll with relaxed loads (no cache maintenance per poll), acquire once below
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&gs->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > timeout) {
          __hip_atomic_store(&gs->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();  // acquire the other blocks' writes
    *ok_sh = ok;
  }
  __syncthreads();
  return *ok_sh != 0;
}

template <typename R, int RECON, int NBT, int LPS, typename LS>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>))
    k_cg_persistent(const SysDesc* __restrict__ sys, int nsys, SrcState* st, int nsrc_total,
                    int nblk_total, int nvblk_total, int iters, GridSync* gs,
                    long long timeout) {
  __shared__ double sh[16 * 64];
  __shared__ double tot[64];
  __shared__ int ok;
  for (int it = 0; it < iters; ++it) {
    // leave when nothing runs or some source waits for a reliable update
    bool run = false, ru = false;
    for (int k = 0; k < nsrc_total; ++k) {
      const int ph = rd<true>(st[k].phase);
      run |= ph == PH_RUN;
      ru |= ph == PH_RU;
    }
    if (!run || ru) break;
    for (int b = blockIdx.x; b < nvblk_total; b += gridDim.x) p_tile<R, true>(sys, nsys, st, b);
    if (!grid_sync(gs, gridDim.x, timeout, &ok)) return;
    for (int b = blockIdx.x; b < nblk_total; b += gridDim.x)
      doe_tile<R, RECON, NBT, LPS, true, LS>(sys, nsys, st, b, 0);
    if (!grid_sync(gs, gridDim.x, timeout, &ok)) return;
    for (int b = blockIdx.x; b < nblk_total; b += gridDim.x)
      deo_tile<R, RECON, NBT, LPS, true, LS>(sys, nsys, st, b, 0, 2, sh, tot);
    if (!grid_sync(gs, gridDim.x, timeout, &ok)) return;
    for (int g = blockIdx.x; g < nsrc_total; g += gridDim.x)
      finalize_one<true>(sys, nsys, st, g, FIN_ALPHA, sh);
    if (!grid_sync(gs, gridDim.x, timeout, &ok)) return;
    for (int b = blockIdx.x; b < nvblk_total; b += gridDim.x)
      xr_tile<R, true>(sys, nsys, st, b, sh);
    if (!grid_sync(gs, gridDim.x, timeout, &ok)) return;
    for (int g = blockIdx.x; g < nsrc_total; g += gridDim.x)
      finalize_one<true>(sys, nsys, st, g, FIN_BETA, sh);
    if (!grid_sync(gs, gridDim.x, timeout, &ok)) return;
  }
}

// ========================================================= reliable update

// The update kernels run in every update slot, usually with nothing to do:
// they take a grid of at most kUpdGrid blocks that strides over the stencil
// blocks or vector tiles, so that an idle launch costs little (the GPU
// dispatches about one workgroup per clock: an idle grid of one block per
// vector tile of a 32^4 twelve-source batch, 73 728 blocks, takes 30 us).
constexpr int kUpdGrid = 2048;

// Does any source of the batch (all nsrc states) stand in `phase` (with
// xpend set, when xp)?  The whole block answers at once, one state per
// thread, so that an update kernel with nothing to do returns after one load
// instead of visiting its blocks' states one after another.
__device__ __forceinline__ bool any_source_in(const SrcState* st, int nsrc, int phase, bool xp) {
  int hit = 0;
  for (int k = threadIdx.x; k < nsrc; k += blockDim.x)
    hit |= st[k].phase == phase && (!xp || st[k].xpend);
  return __syncthreads_or(hit) != 0;
}

// R0: x_lo += alpha p for sources waiting for an update whose last x/r step
// left that term pending (launch-per-pass and persistent engines), in the
// arithmetic of xr_body.
template <typename R>
__global__ void __launch_bounds__(256) k_ru_xfix(const SysDesc* __restrict__ sys, int nsys,
                                                 const SrcState* st, int nsrc, int nvblk) {
  if (!any_source_in(st, nsrc, PH_RU, true)) return;
  for (int b = blockIdx.x; b < nvblk; b += gridDim.x) {
    const SysDesc& d = sys_of_vblock(sys, nsys, b);
    const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
    const SrcState& q = st[d.src0 + k];
    const size_t n = (size_t)3 * d.g.hv, e = (size_t)tile * kVTile + threadIdx.x;
    if (q.phase != PH_RU || !q.xpend || e >= n) continue;
    const size_t vs = n * d.nsrc, i = k * n + e;
    const R al = (R)q.alpha;
    const cplx<R> pv = slot<R>(d.vlo, 2, vs)[i];
    cplx<R>* x = slot<R>(d.vlo, 0, vs);
    cplx<R> xv = x[i];
    xv.re = fma(al, pv.re, xv.re);
    xv.im = fma(al, pv.im, xv.im);
    x[i] = xv;
  }
}

// R1: t_hi = 2 D_oe (x_hi + x_lo) in FP64 for sources waiting for an update.
template <typename Rlo, int RECON, int NBT>
__device__ __forceinline__ void ru_doe_block(const SysDesc* __restrict__ sys, int nsys,
                                             const SrcState* st, int b, int xcd) {
  const int lane = threadIdx.x & 63, grp = wave_id();
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const unsigned long long ru = phase_bits<false>(st + d.src0, d.nsrc, PH_RU);
  const int cb = tile_block(b - d.blk0, d.g, xcd) * kTile + lane;
  const int k0 = grp * NBT;
  const unsigned act = cb < d.g.hv ? group_bits<NBT>(ru, k0) : 0u;
  if (!act) return;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  cplx<double> acc[NBT][3];
  zero_acc<double, NBT>(acc);
  Site s;
  site_geometry(d.g, 1, cb, s);
  stencil_part<double, RECON, NBT, 1>(
      d.g, (const cplx<double>*)d.links_hi, 1, cb, s, 0,
      SumIn<Rlo>{slot<double>(d.vhi, 0, vs) + k0 * ss, slot<Rlo>(d.vlo, 0, vs) + k0 * ss, ss, hv,
                 d.nsrc - 1 - k0},
      acc);
  cplx<double>* t = slot<double>(d.vhi, 3, vs);
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    if (!(act >> j & 1u)) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) t[(k0 + j) * ss + c * hv + cb] = acc[j][c];
  }
}

template <typename Rlo, int RECON, int NBT>
__global__ void __launch_bounds__((kMaxThreads<double, NBT>))
    k_ru_doe(const SysDesc* __restrict__ sys, int nsys, const SrcState* st, int nsrc, int nblk,
             int xcd) {
  if (!any_source_in(st, nsrc, PH_RU, false)) return;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) ru_doe_block<Rlo, RECON, NBT>(sys, nsys, st, b, xcd);
}

// R2: x_hi += x_lo, x_lo = 0, r_hi = b - (m^2 x_hi - 1/4 (2D_eo) t_hi) and the
// partials of |r_hi|^2, all in FP64.
// st_copy (fused sequence, else null): the system's first block copies its
// source states there.
// mark (the two-launch sequence between chunk ends): also store lo(r_hi) in
// the r slot and flag the updating sources (have_rr) for k_f2_doe, which takes
// the update's last step.
template <typename Rlo, int RECON, int NBT>
__device__ __forceinline__ void ru_residual_block(const SysDesc* __restrict__ sys, int nsys,
                                                  SrcState* st, int b, int xcd,
                                                  SrcState* st_copy, int mark, double* sh,
                                                  double* tot) {
  const int lane = threadIdx.x & 63, grp = wave_id();
  const SysDesc& d = sys_of_block(sys, nsys, b);
  const SrcState* q0 = st + d.src0;
  if (st_copy && b == d.blk0)
    for (int k = threadIdx.x; k < d.nsrc; k += blockDim.x) st_copy[d.src0 + k] = q0[k];
  const unsigned long long ru = phase_bits<false>(q0, d.nsrc, PH_RU);
  if (!ru) return;
  if (mark && b == d.blk0)
    for (int k = threadIdx.x; k < d.nsrc; k += blockDim.x)
      if (ru >> k & 1ull) st[d.src0 + k].have_rr = 1;
  const int bl = tile_block(b - d.blk0, d.g, xcd), cb = bl * kTile + lane;
  const size_t hv = d.g.hv, ss = 3 * hv, vs = ss * d.nsrc;
  const int k0 = grp * NBT;
  const unsigned act = cb < d.g.hv ? group_bits<NBT>(ru, k0) : 0u;
  double rr[NBT];
#pragma unroll
  for (int j = 0; j < NBT; ++j) rr[j] = 0.0;
  if (act) {
    cplx<double> acc[NBT][3];
    zero_acc<double, NBT>(acc);
    Site s;
    site_geometry(d.g, 0, cb, s);
    stencil_part<double, RECON, NBT, 1>(
        d.g, (const cplx<double>*)d.links_hi, 0, cb, s, 0,
        FieldIn<double>{slot<double>(d.vhi, 3, vs) + k0 * ss, ss, hv, d.nsrc - 1 - k0}, acc);
    cplx<double>* xhi = slot<double>(d.vhi, 0, vs);
    cplx<double>* rhi = slot<double>(d.vhi, 1, vs);
    const cplx<double>* bb = slot<double>(d.vhi, 2, vs);
    cplx<Rlo>* xlo = slot<Rlo>(d.vlo, 0, vs);
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (!(act >> j & 1u)) continue;
      const double m2 = q0[k0 + j].m2;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const size_t i = (k0 + j) * ss + c * hv + cb;
        const cplx<Rlo> xl = xlo[i];
        cplx<double> xv = xhi[i];
        xv.re += (double)xl.re;
        xv.im += (double)xl.im;
        xhi[i] = xv;
        xlo[i] = {(Rlo)0, (Rlo)0};
        const cplx<double> bv = bb[i];
        const cplx<double> r = {bv.re - fmadd(m2, xv.re, -0.25 * acc[j][c].re),
                                bv.im - fmadd(m2, xv.im, -0.25 * acc[j][c].im)};
        rhi[i] = r;
        if (mark) slot<Rlo>(d.vlo, 1, vs)[i] = {(Rlo)r.re, (Rlo)r.im};
        rr[j] += r.re * r.re + r.im * r.im;
      }
    }
  }
  const int G = (int)(blockDim.x >> 6);
  group_sum<NBT>(rr, 1, grp, 0, G, sh, tot);
  // only the updating sources' entries: the two-launch sequence keeps the
  // <p, Ap> partials of the running ones across the update
  if (threadIdx.x == 0)
    for (int k = 0; k < d.nsrc; ++k)
      if (ru >> k & 1ull) d.partials[(size_t)k * d.nblk + bl] = tot[k];
}

template <typename Rlo, int RECON, int NBT>
__global__ void __launch_bounds__((kMaxThreads<double, NBT>))
    k_ru_residual(const SysDesc* __restrict__ sys, int nsys, SrcState* st, int nsrc, int nblk,
                  int xcd, SrcState* st_copy, int mark) {
  __shared__ double sh[16 * 64];
  __shared__ double tot[64];
  // the state copy of the fused sequence is wanted even when nothing updates
  if (!st_copy && !any_source_in(st, nsrc, PH_RU, false)) return;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    ru_residual_block<Rlo, RECON, NBT>(sys, nsys, st, b, xcd, st_copy, mark, sh, tot);
    __syncthreads();  // sh and tot serve the next block
  }
}

// R3: r = lo(r_hi), p = r + beta p for sources whose update did not converge.
template <typename R>
__global__ void __launch_bounds__(256) k_ru_finish(const SysDesc* __restrict__ sys, int nsys,
                                                   const SrcState* st, int nsrc, int nvblk) {
  if (!any_source_in(st, nsrc, PH_RU2, false)) return;
  for (int b = blockIdx.x; b < nvblk; b += gridDim.x) {
    const SysDesc& d = sys_of_vblock(sys, nsys, b);
    const int rel = b - d.vblk0, k = rel / d.vtiles, tile = rel - k * d.vtiles;
    const SrcState& q = st[d.src0 + k];
    const size_t n = (size_t)3 * d.g.hv, e = (size_t)tile * kVTile + threadIdx.x;
    if (q.phase != PH_RU2 || e >= n) continue;
    const size_t vs = n * d.nsrc, i = k * n + e;
    const R be = (R)q.beta;
    const cplx<double> h = slot<double>(d.vhi, 1, vs)[i];
    const cplx<R> rv = {(R)h.re, (R)h.im};
    cplx<R>* p = slot<R>(d.vlo, 2, vs);
    const cplx<R> pv = p[i];
    slot<R>(d.vlo, 1, vs)[i] = rv;
    p[i] = {fma(be, pv.re, rv.re), fma(be, pv.im, rv.im)};
  }
}

// =============================================== host side, one type pair
//
// The launch sequences of one (inner precision, link storage) pair; each pair
// is instantiated in its own translation unit (qx_engine_inst.hip), and
// qx_engine.hip dispatches to them.

template <typename R>
hipError_t init_impl(const EngineCfg& c, int zero_xhi, hipStream_t s) {
  const dim3 grid(c.nvblk_total), block(kVTile);
  hipLaunchKernelGGL(k_init<R>, grid, block, 0, s, c.d_sys, c.nsys, zero_xhi, c.shape.xcd);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = finalize(c, FIN_INIT, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_zero_done, grid, block, 0, s, c.d_sys, c.nsys, c.d_st, c.shape.xcd);
    e = hipGetLastError();
  }
  return e;
}

template <typename R, int RECON, typename LS>
hipError_t iteration_impl(const EngineCfg& c, int parity, hipStream_t s) {
  const int G = shape_groups(c.shape, c.nsrc_max);
  const dim3 sgrid(c.nblk_total), sblock(64 * c.shape.lps * G);
  const size_t lds = shape_lds(c.shape, c.nsrc_max, cplx_bytes(c.prec_lo));
  const dim3 vgrid(c.nvblk_total), vblock(kVTile);
  if (c.fused && c.two) {
    // p alternates between slots 2 and 5, r between 1 and 6
    const int pin = parity ? 5 : 2, pout = parity ? 2 : 5;
    const int rin = parity ? 6 : 1, rout = parity ? 1 : 6;
    return with_nbt_lps<false>(c.shape.nbt, c.shape.lps, [&]<int NBT, int LPS>() {
      QX_TIMED(c, PASS_DOE, s,
               hipLaunchKernelGGL((k_f2_doe<R, RECON, NBT, LPS, LS>), sgrid, sblock, lds, s,
                                  c.d_sys, c.nsys, c.d_st, c.d_st1, pin, pout, rin, rout,
                                  c.shape.xcd));
      QX_TIMED(c, PASS_DEO, s,
               hipLaunchKernelGGL((k_f2_deo<R, RECON, NBT, LPS, LS>), sgrid, sblock, lds, s,
                                  c.d_sys, c.nsys, c.d_st1, c.d_st, pout, rout, c.shape.xcd));
      return hipGetLastError();
    });
  }
  if (c.fused) {
    // p alternates between slots 2 and 5; the states between the two slots
    const int pin = parity ? 5 : 2, pout = parity ? 2 : 5;
    return with_nbt_lps<false>(c.shape.nbt, c.shape.lps, [&]<int NBT, int LPS>() {
      QX_TIMED(c, PASS_DOE, s,
               hipLaunchKernelGGL((k_fiter_doe<R, RECON, NBT, LPS, LS>), sgrid, sblock, lds, s,
                                  c.d_sys, c.nsys, c.d_st, c.d_st1, pin, pout, c.shape.xcd));
      QX_TIMED(c, PASS_DEO, s,
               hipLaunchKernelGGL((k_iter_deo<R, RECON, NBT, LPS, LS>), sgrid, sblock, lds, s,
                                  c.d_sys, c.nsys, c.d_st1, pout, c.shape.xcd));
      QX_TIMED(c, PASS_XR, s,
               hipLaunchKernelGGL(k_fiter_xr<R>, vgrid, vblock, 0, s, c.d_sys, c.nsys, c.d_st1,
                                  c.d_st, pout, c.shape.xcd));
      return hipGetLastError();
    });
  }
  // the launch-per-pass stencils have the wide shapes for FP32 one-hop links
  constexpr bool kWide = sizeof(R) == 4 && RECON != 36 && std::is_same_v<LS, R>;
  hipError_t e = with_nbt_lps<kWide>(c.shape.nbt, c.shape.lps, [&]<int NBT, int LPS>() {
    QX_TIMED(c, PASS_P, s,
             hipLaunchKernelGGL(k_iter_p<R>, vgrid, dim3(64), 0, s, c.d_sys, c.nsys, c.d_st,
                                c.shape.xcd));
    // several source groups of one wavefront per site share the link loads
    constexpr size_t kLL = kLinkLdsBytes<RECON, LS>;
    if constexpr (LPS == 1 && kLL != 0) {
      if (G >= 2) {
        QX_TIMED(c, PASS_DOE, s,
                 hipLaunchKernelGGL((k_iter_doe<R, RECON, NBT, 1, LS, true>), sgrid, sblock, kLL,
                                    s, c.d_sys, c.nsys, c.d_st, c.shape.xcd));
        return hipGetLastError();
      }
    }
    QX_TIMED(c, PASS_DOE, s,
             hipLaunchKernelGGL((k_iter_doe<R, RECON, NBT, LPS, LS>), sgrid, sblock, lds, s,
                                c.d_sys, c.nsys, c.d_st, c.shape.xcd));
    return hipGetLastError();
  });
  // the D_eo pass under its own (sources per thread, wavefronts per site)
  if (e == hipSuccess)
    e = with_nbt_lps<kWide>(c.deo_shape.nbt, c.deo_shape.lps, [&]<int NBT, int LPS>() {
      const LaunchShape& dsh = c.deo_shape;
      const int dg = shape_groups(dsh, c.nsrc_max);
      const dim3 dblock(64 * dsh.lps * dg);
      // several source groups of one wavefront per site share the link loads
      constexpr size_t kLL = kLinkLdsBytes<RECON, LS>;
      if constexpr (LPS == 1 && kLL != 0) {
        if (dg >= 2) {
          const size_t llds = deo_ll_lds<RECON, LS>(dg, NBT);
          QX_TIMED(c, PASS_DEO, s,
                   hipLaunchKernelGGL((k_iter_deo_ll<R, RECON, NBT, LS>), sgrid, dblock, llds, s,
                                      c.d_sys, c.nsys, c.d_st, 2, c.shape.xcd));
          return hipGetLastError();
        }
      }
      const size_t dlds = shape_lds(dsh, c.nsrc_max, sizeof(cplx<R>));
      QX_TIMED(c, PASS_DEO, s,
               hipLaunchKernelGGL((k_iter_deo<R, RECON, NBT, LPS, LS>), sgrid, dblock, dlds, s,
                                  c.d_sys, c.nsys, c.d_st, 2, c.shape.xcd));
      return hipGetLastError();
    });
  if (e == hipSuccess) e = finalize(c, FIN_ALPHA, s);
  if (e == hipSuccess) {
    QX_TIMED(c, PASS_XR, s,
             hipLaunchKernelGGL(k_iter_xr<R>, vgrid, dim3(64), 0, s, c.d_sys, c.nsys, c.d_st,
                                c.shape.xcd));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = finalize(c, FIN_BETA, s);
  return e;
}

// RECON: the storage of the FP64 links (the update works on them).
template <typename Rlo, int RECON>
hipError_t reliable_update_impl(const EngineCfg& c, bool last, hipStream_t s) {
  // FP64 stencils: at most two sources per thread where the batch's sources
  // fit one block that way (with four, the update kernels spill: 450-500
  // bytes per lane), else at most four
  LaunchShape rsh{narrow_nbt(c.shape.nbt), 1, c.shape.xcd};
  if (rsh.nbt > 2) {
    LaunchShape r2 = rsh;
    r2.nbt = 2;
    if (shape_ok(r2, c.nsrc_max, cplx_bytes(0))) rsh = r2;
  }
  const int G = shape_groups(rsh, c.nsrc_max);
  const dim3 sgrid(c.nblk_total), sblock(64 * G);
  const dim3 vgrid(c.nvblk_total), vblock(kVTile);
  // the two-launch sequence leaves an update's last step to its next D_oe
  // pass, except at the end of a chunk (the host reads the states there)
  const bool handoff = c.fused && c.two && !last;
  SrcState* copy = c.fused && !handoff ? c.d_st1 : nullptr;
  // capped grids (kUpdGrid): most update slots find nothing to do
  const dim3 ugrid(std::min(c.nblk_total, kUpdGrid)), uvgrid(std::min(c.nvblk_total, kUpdGrid));
  hipError_t e = hipSuccess;
  if (!c.fused) {
    QX_TIMED(c, PASS_UPDATE, s,
             hipLaunchKernelGGL(k_ru_xfix<Rlo>, uvgrid, vblock, 0, s, c.d_sys, c.nsys, c.d_st,
                                c.nsrc_total, c.nvblk_total));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = with_nbt(rsh.nbt, [&]<int NBT>() {
    QX_TIMED(c, PASS_UPDATE, s,
             hipLaunchKernelGGL((k_ru_doe<Rlo, RECON, NBT>), ugrid, sblock, 0, s, c.d_sys, c.nsys,
                                c.d_st, c.nsrc_total, c.nblk_total, c.shape.xcd));
    QX_TIMED(c, PASS_UPDATE, s,
             hipLaunchKernelGGL((k_ru_residual<Rlo, RECON, NBT>), ugrid, sblock, 0, s, c.d_sys,
                                c.nsys, c.d_st, c.nsrc_total, c.nblk_total, c.shape.xcd, copy,
                                handoff ? 1 : 0));
    return hipGetLastError();
  });
  if (handoff) return e;
  if (c.fused) {
    if (e == hipSuccess) {
      QX_TIMED(c, PASS_UPDATE, s,
               hipLaunchKernelGGL(k_fru_finish<Rlo>, vgrid, vblock, 0, s, c.d_sys, c.nsys,
                                  c.d_st1, c.d_st, c.shape.xcd));
      e = hipGetLastError();
    }
    return e;
  }
  if (e == hipSuccess) e = finalize(c, FIN_RU, s);
  if (e == hipSuccess) {
    QX_TIMED(c, PASS_UPDATE, s,
             hipLaunchKernelGGL(k_ru_finish<Rlo>, uvgrid, vblock, 0, s, c.d_sys, c.nsys, c.d_st,
                                c.nsrc_total, c.nvblk_total));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = finalize(c, FIN_COMMIT, s);
  return e;
}

template <typename R, int RECON, typename LS>
int persistent_per_cu_impl(const EngineCfg& c) {
  const int G = shape_groups(c.shape, c.nsrc_max);
  const int threads = 64 * c.shape.lps * G;
  const size_t lds = shape_lds(c.shape, c.nsrc_max, cplx_bytes(c.prec_lo));
  int per_cu = 0;
  hipError_t e = with_nbt_lps<false>(c.shape.nbt, c.shape.lps, [&]<int NBT, int LPS>() {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_cg_persistent<R, RECON, NBT, LPS, LS>), threads, lds);
  });
  return e == hipSuccess ? per_cu : 0;
}

template <typename R, int RECON, typename LS>
hipError_t persistent_impl(const EngineCfg& c, int iters, GridSync* gs, int grid,
                           long long timeout, hipStream_t s) {
  const int G = shape_groups(c.shape, c.nsrc_max);
  const int threads = 64 * c.shape.lps * G;
  const size_t lds = shape_lds(c.shape, c.nsrc_max, cplx_bytes(c.prec_lo));
  const SysDesc* sys = c.d_sys;
  int nsys = c.nsys, nsrc = c.nsrc_total, nblk = c.nblk_total, nvblk = c.nvblk_total;
  SrcState* st = c.d_st;
  void* args[] = {&sys, &nsys, &st, &nsrc, &nblk, &nvblk, &iters, &gs, &timeout};
  return with_nbt_lps<false>(c.shape.nbt, c.shape.lps, [&]<int NBT, int LPS>() {
    return hipLaunchCooperativeKernel(
        reinterpret_cast<const void*>(&k_cg_persistent<R, RECON, NBT, LPS, LS>), dim3(grid),
        dim3(threads), args, (unsigned)lds, s);
  });
}

}  // namespace qx
