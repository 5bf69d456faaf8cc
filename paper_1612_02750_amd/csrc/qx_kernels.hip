// gfx950 kernels of libqx.so: packing, index maps, the staggered Dslash, the
// even-site operator A = m^2 - D_eo D_oe, the conjugate-gradient engine with
// reliable updates, and the fermion force.
//
// Operator (textbook Kogut-Susskind form of the staggered operator the paper
// names in Sec. 4):
//   (D chi)(x) = 1/2 sum_mu eta_mu(x) [bc U_mu(x) chi(x+mu) - bc U_mu(x-mu)^dag chi(x-mu)]
// Inside the kernels the links carry eta * bc (folded at pack time) and the
// stencil computes 2D; the factor 1/2 (or 1/4 for D_eo D_oe) is applied in the
// epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qx_device.h"
#include "qx_launch.h"

namespace qx {

namespace {

constexpr int kStatusOk = 0;
constexpr int kStatusNotConverged = 5;
constexpr int kStatusBreakdown = 6;

inline unsigned grid_for(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Calls f.template operator()<NB>() with the smallest supported NB >= n.
template <typename F>
hipError_t with_nb(int n, F&& f) {
  if (n <= 1) return f.template operator()<1>();
  if (n <= 2) return f.template operator()<2>();
  if (n <= 4) return f.template operator()<4>();
  if (n <= 8) return f.template operator()<8>();
  if (n <= 12) return f.template operator()<12>();
  return hipErrorInvalidValue;
}

template <typename F>
hipError_t with_prec_recon(int prec, int recon, F&& f) {
  if (prec == 0 && recon == 18) return f.template operator()<double, 18>();
  if (prec == 0 && recon == 12) return f.template operator()<double, 12>();
  if (prec == 1 && recon == 18) return f.template operator()<float, 18>();
  if (prec == 1 && recon == 12) return f.template operator()<float, 12>();
  return hipErrorInvalidValue;
}

}  // namespace

// =================================================================== packing

// Canonical complex128 [4][V][3][3] -> packed [parity][mu][e][cb] with the
// staggered phase and boundary sign folded in.  With 12-real storage the FP64
// reconstruction error of the canonical link is max-reduced into err_bits.
template <typename R, int RECON>
__global__ void __launch_bounds__(256) k_pack_gauge(Geo g, const cplx<double>* __restrict__ U,
                                                    cplx<R>* __restrict__ out,
                                                    unsigned long long* err_bits) {
  constexpr int E = RECON == 12 ? 6 : 9;
  const int64_t V = 2 * (int64_t)g.hv;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double err = 0.0;
  if (i < 4 * V) {
    const int mu = (int)(i / V);
    const int lex = (int)(i - mu * V);
    int t = lex;
    const int x0 = t % g.L0;
    t /= g.L0;
    const int x1 = t % g.L1;
    t /= g.L1;
    const int x2 = t % g.L2;
    const int x3 = t / g.L2;
    const int p = (x0 + x1 + x2 + x3) & 1;
    const int cb = lex >> 1;
    const double sg = (double)link_sign(g, mu, x0, x1, x2, x3);
    const cplx<double>* u = U + i * 9;
    cplx<double> v[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) v[e] = u[e];
    cplx<R>* o = out + (size_t)(p * 4 + mu) * E * g.hv + cb;
#pragma unroll
    for (int e = 0; e < E; ++e) o[(size_t)e * g.hv] = {(R)(sg * v[e].re), (R)(sg * v[e].im)};
    if constexpr (RECON == 12) {
      // row 2 against conj(row0 x row1)
      const cplx<double> a0 = cmul(v[1], v[5]), b0 = cmul(v[2], v[4]);
      const cplx<double> a1 = cmul(v[2], v[3]), b1 = cmul(v[0], v[5]);
      const cplx<double> a2 = cmul(v[0], v[4]), b2 = cmul(v[1], v[3]);
      const double d0 = fabs(v[6].re - (a0.re - b0.re)) + fabs(v[6].im + (a0.im - b0.im));
      const double d1 = fabs(v[7].re - (a1.re - b1.re)) + fabs(v[7].im + (a1.im - b1.im));
      const double d2 = fabs(v[8].re - (a2.re - b2.re)) + fabs(v[8].im + (a2.im - b2.im));
      err = fmax(fmax(d0, d1), d2);
      if (err != err) err = __builtin_inf();
    }
  }
  if constexpr (RECON == 12) {
    if (err_bits) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) err = fmax(err, __shfl_xor(err, off, 64));
      if ((threadIdx.x & 63) == 0 && err > 0.0)
        atomicMax(err_bits, (unsigned long long)__double_as_longlong(err));
    }
  }
}

// canonical complex128 [nsrc][hv][3] -> packed [nsrc][3][hv]
template <typename R>
__global__ void __launch_bounds__(256) k_pack_field(int hv, int nsrc,
                                                    const cplx<double>* __restrict__ in,
                                                    cplx<R>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nsrc * hv) return;
  const int64_t s = i / hv, cb = i - s * hv;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<double> v = in[i * 3 + c];
    out[(s * 3 + c) * hv + cb] = {(R)v.re, (R)v.im};
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_unpack_field(int hv, int nsrc,
                                                      const cplx<R>* __restrict__ in,
                                                      cplx<double>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nsrc * hv) return;
  const int64_t s = i / hv, cb = i - s * hv;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<R> v = in[(s * 3 + c) * hv + cb];
    out[i * 3 + c] = {(double)v.re, (double)v.im};
  }
}

__global__ void __launch_bounds__(256) k_index_maps(Geo g, int32_t* __restrict__ lex_of_eo,
                                                    int32_t* __restrict__ nbr) {
  const int64_t eo = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (eo >= 2 * (int64_t)g.hv) return;
  const int p = eo >= g.hv;
  const int cb = (int)(eo - (int64_t)p * g.hv);
  Site s;
  site_geometry(g, p, cb, s);
  lex_of_eo[eo] = 2 * cb + (s.x0 & 1);
  const int other = (1 - p) * g.hv;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    nbr[eo * 8 + mu] = other + s.fwd[mu];
    nbr[eo * 8 + 4 + mu] = other + s.bwd[mu];
  }
}

hipError_t launch_pack_gauge(const Geo& g, const void* U, int prec, int recon, void* packed,
                             unsigned long long* err_bits, hipStream_t s) {
  const size_t n = 8 * (size_t)g.hv;
  return with_prec_recon(prec, recon, [&]<typename R, int RECON>() {
    hipLaunchKernelGGL((k_pack_gauge<R, RECON>), dim3(grid_for(n, 256)), dim3(256), 0, s, g,
                       (const cplx<double>*)U, (cplx<R>*)packed, err_bits);
    return hipGetLastError();
  });
}

hipError_t launch_pack_field(const Geo& g, int nrhs, int prec, const void* canon, void* packed,
                             hipStream_t s) {
  const size_t n = (size_t)nrhs * g.hv;
  if (prec == 0)
    hipLaunchKernelGGL(k_pack_field<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv, nrhs,
                       (const cplx<double>*)canon, (cplx<double>*)packed);
  else
    hipLaunchKernelGGL(k_pack_field<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv, nrhs,
                       (const cplx<double>*)canon, (cplx<float>*)packed);
  return hipGetLastError();
}

hipError_t launch_unpack_field(const Geo& g, int nrhs, int prec, const void* packed, void* canon,
                               hipStream_t s) {
  const size_t n = (size_t)nrhs * g.hv;
  if (prec == 0)
    hipLaunchKernelGGL(k_unpack_field<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv,
                       nrhs, (const cplx<double>*)packed, (cplx<double>*)canon);
  else
    hipLaunchKernelGGL(k_unpack_field<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv,
                       nrhs, (const cplx<float>*)packed, (cplx<double>*)canon);
  return hipGetLastError();
}

hipError_t launch_index_maps(const Geo& g, int32_t* lex_of_eo, int32_t* nbr_eo, hipStream_t s) {
  hipLaunchKernelGGL(k_index_maps, dim3(grid_for(2 * (size_t)g.hv, 256)), dim3(256), 0, s, g,
                     lex_of_eo, nbr_eo);
  return hipGetLastError();
}

// ============================================================ plain operators

// out_k = scale * (2D in_k) at the sites of parity pout, k < nsrc <= NB.
template <typename R, int RECON, int NB>
__global__ void __launch_bounds__(512) k_dslash(Geo g, const cplx<R>* __restrict__ links, int pout,
                                                const cplx<R>* __restrict__ in,
                                                cplx<R>* __restrict__ out, int nsrc, R scale,
                                                int xcd) {
  const int cb = logical_block(xcd) * blockDim.x + threadIdx.x;
  if (cb >= g.hv) return;
  const size_t hv = (size_t)g.hv;
  const unsigned act = (1u << nsrc) - 1u;
  cplx<R> acc[NB][3];
  stencil<R, RECON, NB>(g, links, pout, cb, in, 3 * hv, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k >= nsrc) break;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      out[(k * 3 + a) * hv + cb] = {scale * acc[k][a].re, scale * acc[k][a].im};
  }
}

struct Masses12 {
  double m2[12];
};

// out_k = m2_k p_k - 1/4 (2D_eo) t_k at even sites (t = 2 D_oe p on odd sites).
template <typename R, int RECON, int NB>
__global__ void __launch_bounds__(512) k_deo_axpy(Geo g, const cplx<R>* __restrict__ links,
                                                  const cplx<R>* __restrict__ t,
                                                  const cplx<R>* __restrict__ p,
                                                  cplx<R>* __restrict__ out, int nsrc, Masses12 m,
                                                  int xcd) {
  const int cb = logical_block(xcd) * blockDim.x + threadIdx.x;
  if (cb >= g.hv) return;
  const size_t hv = (size_t)g.hv;
  const unsigned act = (1u << nsrc) - 1u;
  cplx<R> acc[NB][3];
  stencil<R, RECON, NB>(g, links, 0, cb, t, 3 * hv, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k >= nsrc) break;
    const R m2 = (R)m.m2[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t j = (k * 3 + a) * hv + cb;
      const cplx<R> pv = p[j];
      out[j] = {m2 * pv.re - (R)0.25 * acc[k][a].re, m2 * pv.im - (R)0.25 * acc[k][a].im};
    }
  }
}

hipError_t launch_dslash(const Geo& g, int prec, int recon, const void* links, int pout,
                         const void* in, void* out, int nsrc, double scale, LaunchShape sh,
                         hipStream_t s) {
  const size_t csz = cplx_bytes(prec);
  const size_t field = (size_t)3 * g.hv * csz;
  for (int k0 = 0; k0 < nsrc; k0 += 12) {
    const int n = nsrc - k0 < 12 ? nsrc - k0 : 12;
    const char* pin = (const char*)in + k0 * field;
    char* pout_ = (char*)out + k0 * field;
    hipError_t e = with_prec_recon(prec, recon, [&]<typename R, int RECON>() {
      return with_nb(n, [&]<int NB>() {
        hipLaunchKernelGGL((k_dslash<R, RECON, NB>), dim3(grid_for(g.hv, sh.block)),
                           dim3(sh.block), 0, s, g, (const cplx<R>*)links, pout,
                           (const cplx<R>*)pin, (cplx<R>*)pout_, n, (R)scale, sh.xcd);
        return hipGetLastError();
      });
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_apply_A(const Geo& g, int prec, int recon, const void* links, int nrhs,
                          const double* m2, const void* in, void* out, void* tmp, LaunchShape sh,
                          hipStream_t s) {
  hipError_t e = launch_dslash(g, prec, recon, links, 1, in, tmp, nrhs, 1.0, sh, s);
  if (e != hipSuccess) return e;
  const size_t field = (size_t)3 * g.hv * cplx_bytes(prec);
  for (int k0 = 0; k0 < nrhs; k0 += 12) {
    const int n = nrhs - k0 < 12 ? nrhs - k0 : 12;
    Masses12 m{};
    for (int k = 0; k < n; ++k) m.m2[k] = m2[k0 + k];
    e = with_prec_recon(prec, recon, [&]<typename R, int RECON>() {
      return with_nb(n, [&]<int NB>() {
        hipLaunchKernelGGL((k_deo_axpy<R, RECON, NB>), dim3(grid_for(g.hv, sh.block)),
                           dim3(sh.block), 0, s, g, (const cplx<R>*)links,
                           (const cplx<R>*)((const char*)tmp + k0 * field),
                           (const cplx<R>*)((const char*)in + k0 * field),
                           (cplx<R>*)((char*)out + k0 * field), n, m, sh.xcd);
        return hipGetLastError();
      });
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ==================================================================== engine
//
// Every engine launch covers all systems of a batch: block b belongs to the
// system whose [blk0, blk0 + nblk) range holds it, and each thread handles one
// checkerboard site for all NB sources of its system.  Sources whose phase
// does not match the kernel's are skipped, so converged sources cost nothing
// but the link loads they share with the others.
//
// Vector slots: inner precision vlo = {x_lo, r, p, Ap, t(odd)}, FP64
// vhi = {x_hi, r_hi, b, t_hi(odd)}; each slot is [nsrc][3][hv].

namespace {

__device__ __forceinline__ const SysDesc& find_sys(const SysDesc* __restrict__ sys, int nsys,
                                                   int b) {
  int i = 0;
  while (i + 1 < nsys && b >= sys[i + 1].blk0) ++i;
  return sys[i];
}

template <int NB>
__device__ __forceinline__ unsigned phase_mask(const SrcState* st, int nsrc, int phase) {
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < NB; ++k)
    if (k < nsrc && st[k].phase == phase) m |= 1u << k;
  return m;
}

template <typename R>
__device__ __forceinline__ cplx<R>* slot(void* base, int i, size_t vs) {
  return (cplx<R>*)base + i * vs;
}

}  // namespace

// Init: x_lo = 0, p = 0, optionally x_hi = 0; |b|^2 -> bnorm2, stop2 *= bnorm2;
// a zero source is done at once (x = 0), a non-finite one is a breakdown.
template <typename R, int NB>
__global__ void __launch_bounds__(512) k_init(const SysDesc* __restrict__ sys, int nsys,
                                              SrcState* st, int zero_xhi, int xcd) {
  __shared__ double sh[NB * 16];
  __shared__ int flag;
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const int bl = b - d.blk0, cb = bl * blockDim.x + threadIdx.x;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  double nb2[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) nb2[k] = 0.0;
  if (cb < d.g.hv) {
    cplx<R>* xlo = slot<R>(d.vlo, 0, vs);
    cplx<R>* p = slot<R>(d.vlo, 2, vs);
    cplx<double>* xhi = slot<double>(d.vhi, 0, vs);
    const cplx<double>* bb = slot<double>(d.vhi, 2, vs);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (k >= d.nsrc) break;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = (k * 3 + a) * hv + cb;
        xlo[j] = {(R)0, (R)0};
        p[j] = {(R)0, (R)0};
        if (zero_xhi) xhi[j] = {0.0, 0.0};
        const cplx<double> v = bb[j];
        nb2[k] += v.re * v.re + v.im * v.im;
      }
    }
  }
  block_sum<NB>(nb2, sh);
  if (publish_partials<NB>(nb2, d.nsrc, d.partials, d.nblk, bl, d.counter, &flag)) {
    double tot[NB];
    total_partials<NB>(tot, d.nsrc, d.partials, d.nblk, d.counter, sh);
    if (threadIdx.x == 0) {
      for (int k = 0; k < NB && k < d.nsrc; ++k) {
        SrcState& q = st[d.src0 + k];
        q.bnorm2 = tot[k];
        q.stop2 *= tot[k];
        if (tot[k] == 0.0) {
          q.phase = PH_DONE;
          q.status = kStatusOk;
          q.relres = 0.0;
        } else if (!isfinite(tot[k])) {
          q.phase = PH_DONE;
          q.status = kStatusBreakdown;
          q.relres = tot[k];
        }
      }
    }
  }
}

// x_hi = 0 for zero sources (the solution of A x = 0).
template <int NB>
__global__ void __launch_bounds__(512) k_zero_done(const SysDesc* __restrict__ sys, int nsys,
                                                   const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const int cb = (b - d.blk0) * blockDim.x + threadIdx.x;
  if (cb >= d.g.hv) return;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  cplx<double>* xhi = slot<double>(d.vhi, 0, vs);
  for (int k = 0; k < NB && k < d.nsrc; ++k) {
    const SrcState& q = st[d.src0 + k];
    if (q.phase == PH_DONE && q.bnorm2 == 0.0)
      for (int a = 0; a < 3; ++a) xhi[(k * 3 + a) * hv + cb] = {0.0, 0.0};
  }
}

// E1: t = 2 D_oe p for running sources.
template <typename R, int RECON, int NB>
__global__ void __launch_bounds__(512) k_iter_doe(const SysDesc* __restrict__ sys, int nsys,
                                                  const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const unsigned act = phase_mask<NB>(st + d.src0, d.nsrc, PH_RUN);
  const int cb = (b - d.blk0) * blockDim.x + threadIdx.x;
  if (!act || cb >= d.g.hv) return;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  const cplx<R>* p = slot<R>(d.vlo, 2, vs);
  cplx<R>* t = slot<R>(d.vlo, 4, vs);
  cplx<R> acc[NB][3];
  stencil<R, RECON, NB>(d.g, (const cplx<R>*)d.links_lo, 1, cb, p, 3 * hv, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (!(act >> k & 1u)) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) t[(k * 3 + a) * hv + cb] = acc[k][a];
  }
}

// E2: Ap = m^2 p - 1/4 (2D_eo) t, Re<p, Ap>; the last block forms alpha.
template <typename R, int RECON, int NB>
__global__ void __launch_bounds__(512) k_iter_deo(const SysDesc* __restrict__ sys, int nsys,
                                                  SrcState* st, int xcd) {
  __shared__ double sh[NB * 16];
  __shared__ int flag;
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  SrcState* q0 = st + d.src0;
  const unsigned act = phase_mask<NB>(q0, d.nsrc, PH_RUN);
  if (!act) return;
  const int bl = b - d.blk0, cb = bl * blockDim.x + threadIdx.x;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  double dot[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) dot[k] = 0.0;
  if (cb < d.g.hv) {
    const cplx<R>* p = slot<R>(d.vlo, 2, vs);
    cplx<R>* Ap = slot<R>(d.vlo, 3, vs);
    const cplx<R>* t = slot<R>(d.vlo, 4, vs);
    cplx<R> acc[NB][3];
    stencil<R, RECON, NB>(d.g, (const cplx<R>*)d.links_lo, 0, cb, t, 3 * hv, act, acc);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!(act >> k & 1u)) continue;
      const R m2 = (R)q0[k].m2;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = (k * 3 + a) * hv + cb;
        const cplx<R> pv = p[j];
        const cplx<R> r = {m2 * pv.re - (R)0.25 * acc[k][a].re,
                           m2 * pv.im - (R)0.25 * acc[k][a].im};
        Ap[j] = r;
        dot[k] += (double)pv.re * (double)r.re + (double)pv.im * (double)r.im;
      }
    }
  }
  block_sum<NB>(dot, sh);
  if (publish_partials<NB>(dot, d.nsrc, d.partials, d.nblk, bl, d.counter, &flag)) {
    double tot[NB];
    total_partials<NB>(tot, d.nsrc, d.partials, d.nblk, d.counter, sh);
    if (threadIdx.x == 0) {
      for (int k = 0; k < NB && k < d.nsrc; ++k) {
        if (!(act >> k & 1u)) continue;
        SrcState& q = q0[k];
        q.pAp = tot[k];
        if (!(tot[k] > 0.0) || !isfinite(tot[k])) {
          q.phase = PH_RU;
          q.reason = RU_FINAL;
          q.status = kStatusBreakdown;
        } else {
          q.alpha = q.rho / tot[k];
        }
      }
    }
  }
}

// E3: x_lo += alpha p, r -= alpha Ap, |r|^2; the last block decides between
// continuing (beta), a reliable update, or the end of the iteration budget.
template <typename R, int NB>
__global__ void __launch_bounds__(512) k_iter_xr(const SysDesc* __restrict__ sys, int nsys,
                                                 SrcState* st, int xcd) {
  __shared__ double sh[NB * 16];
  __shared__ int flag;
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  SrcState* q0 = st + d.src0;
  const unsigned act = phase_mask<NB>(q0, d.nsrc, PH_RUN);
  if (!act) return;
  const int bl = b - d.blk0, cb = bl * blockDim.x + threadIdx.x;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  double rr[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) rr[k] = 0.0;
  if (cb < d.g.hv) {
    cplx<R>* x = slot<R>(d.vlo, 0, vs);
    cplx<R>* r = slot<R>(d.vlo, 1, vs);
    const cplx<R>* p = slot<R>(d.vlo, 2, vs);
    const cplx<R>* Ap = slot<R>(d.vlo, 3, vs);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!(act >> k & 1u)) continue;
      const R al = (R)q0[k].alpha;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = (k * 3 + a) * hv + cb;
        const cplx<R> pv = p[j], av = Ap[j];
        cplx<R> xv = x[j], rv = r[j];
        xv.re = fma(al, pv.re, xv.re);
        xv.im = fma(al, pv.im, xv.im);
        rv.re = fma(-al, av.re, rv.re);
        rv.im = fma(-al, av.im, rv.im);
        x[j] = xv;
        r[j] = rv;
        rr[k] += (double)rv.re * (double)rv.re + (double)rv.im * (double)rv.im;
      }
    }
  }
  block_sum<NB>(rr, sh);
  if (publish_partials<NB>(rr, d.nsrc, d.partials, d.nblk, bl, d.counter, &flag)) {
    double tot[NB];
    total_partials<NB>(tot, d.nsrc, d.partials, d.nblk, d.counter, sh);
    if (threadIdx.x == 0) {
      for (int k = 0; k < NB && k < d.nsrc; ++k) {
        if (!(act >> k & 1u)) continue;
        SrcState& q = q0[k];
        const double rn2 = tot[k];
        q.iters += 1;
        if (!isfinite(rn2)) {
          q.phase = PH_RU;
          q.reason = RU_FINAL;
          q.status = kStatusBreakdown;
          continue;
        }
        const double rn = sqrt(rn2);
        if (rn > q.rmax) q.rmax = rn;
        if (q.iters >= q.max_iter) {
          q.phase = PH_RU;
          q.reason = RU_FINAL;
          q.status = kStatusNotConverged;
        } else if (rn2 <= q.stop2 || rn < q.delta * q.rmax) {
          q.phase = PH_RU;
          q.reason = RU_DROP;
        } else {
          q.beta = rn2 / q.rho;
          q.rho = rn2;
        }
      }
    }
  }
}

// E4: p = r + beta p for running sources.
template <typename R, int NB>
__global__ void __launch_bounds__(512) k_iter_p(const SysDesc* __restrict__ sys, int nsys,
                                                const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const SrcState* q0 = st + d.src0;
  const unsigned act = phase_mask<NB>(q0, d.nsrc, PH_RUN);
  const int cb = (b - d.blk0) * blockDim.x + threadIdx.x;
  if (!act || cb >= d.g.hv) return;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  const cplx<R>* r = slot<R>(d.vlo, 1, vs);
  cplx<R>* p = slot<R>(d.vlo, 2, vs);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (!(act >> k & 1u)) continue;
    const R be = (R)q0[k].beta;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t j = (k * 3 + a) * hv + cb;
      const cplx<R> rv = r[j], pv = p[j];
      p[j] = {fma(be, pv.re, rv.re), fma(be, pv.im, rv.im)};
    }
  }
}

// R1: x_hi += x_lo, x_lo = 0 for sources waiting for a reliable update.
template <typename R, int NB>
__global__ void __launch_bounds__(512) k_ru_accum(const SysDesc* __restrict__ sys, int nsys,
                                                  const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const unsigned act = phase_mask<NB>(st + d.src0, d.nsrc, PH_RU);
  const int cb = (b - d.blk0) * blockDim.x + threadIdx.x;
  if (!act || cb >= d.g.hv) return;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  cplx<R>* xlo = slot<R>(d.vlo, 0, vs);
  cplx<double>* xhi = slot<double>(d.vhi, 0, vs);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (!(act >> k & 1u)) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t j = (k * 3 + a) * hv + cb;
      const cplx<R> v = xlo[j];
      cplx<double> h = xhi[j];
      h.re += (double)v.re;
      h.im += (double)v.im;
      xhi[j] = h;
      xlo[j] = {(R)0, (R)0};
    }
  }
}

// R2: t_hi = 2 D_oe x_hi in FP64.
template <int RECON, int NB>
__global__ void __launch_bounds__(512) k_ru_doe(const SysDesc* __restrict__ sys, int nsys,
                                                const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const unsigned act = phase_mask<NB>(st + d.src0, d.nsrc, PH_RU);
  const int cb = (b - d.blk0) * blockDim.x + threadIdx.x;
  if (!act || cb >= d.g.hv) return;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  const cplx<double>* xhi = slot<double>(d.vhi, 0, vs);
  cplx<double>* t = slot<double>(d.vhi, 3, vs);
  cplx<double> acc[NB][3];
  stencil<double, RECON, NB>(d.g, (const cplx<double>*)d.links_hi, 1, cb, xhi, 3 * hv, act, acc);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (!(act >> k & 1u)) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) t[(k * 3 + a) * hv + cb] = acc[k][a];
  }
}

// R3: r_hi = b - (m^2 x_hi - 1/4 (2D_eo) t_hi) and |r_hi|^2 in FP64; the last
// block declares convergence on this true residual or prepares the restart
// of the recurrence (beta, rho, rmax).
template <int RECON, int NB>
__global__ void __launch_bounds__(512) k_ru_residual(const SysDesc* __restrict__ sys, int nsys,
                                                     SrcState* st, int xcd) {
  __shared__ double sh[NB * 16];
  __shared__ int flag;
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  SrcState* q0 = st + d.src0;
  const unsigned act = phase_mask<NB>(q0, d.nsrc, PH_RU);
  if (!act) return;
  const int bl = b - d.blk0, cb = bl * blockDim.x + threadIdx.x;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  double rr[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) rr[k] = 0.0;
  if (cb < d.g.hv) {
    const cplx<double>* xhi = slot<double>(d.vhi, 0, vs);
    cplx<double>* rhi = slot<double>(d.vhi, 1, vs);
    const cplx<double>* bb = slot<double>(d.vhi, 2, vs);
    const cplx<double>* t = slot<double>(d.vhi, 3, vs);
    cplx<double> acc[NB][3];
    stencil<double, RECON, NB>(d.g, (const cplx<double>*)d.links_hi, 0, cb, t, 3 * hv, act, acc);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!(act >> k & 1u)) continue;
      const double m2 = q0[k].m2;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t j = (k * 3 + a) * hv + cb;
        const cplx<double> xv = xhi[j], bv = bb[j];
        const cplx<double> r = {bv.re - (m2 * xv.re - 0.25 * acc[k][a].re),
                                bv.im - (m2 * xv.im - 0.25 * acc[k][a].im)};
        rhi[j] = r;
        rr[k] += r.re * r.re + r.im * r.im;
      }
    }
  }
  block_sum<NB>(rr, sh);
  if (publish_partials<NB>(rr, d.nsrc, d.partials, d.nblk, bl, d.counter, &flag)) {
    double tot[NB];
    total_partials<NB>(tot, d.nsrc, d.partials, d.nblk, d.counter, sh);
    if (threadIdx.x == 0) {
      for (int k = 0; k < NB && k < d.nsrc; ++k) {
        if (!(act >> k & 1u)) continue;
        SrcState& q = q0[k];
        const double r2 = tot[k];
        q.updates += 1;
        q.relres = sqrt(r2 / q.bnorm2);
        if (r2 <= q.stop2) {
          q.phase = PH_DONE;
          q.status = kStatusOk;
        } else if (!isfinite(r2)) {
          q.phase = PH_DONE;
          q.status = kStatusBreakdown;
        } else if (q.reason == RU_FINAL) {
          q.phase = PH_DONE;
        } else {
          q.beta = q.reason == RU_INIT ? 0.0 : r2 / q.rho;
          q.rho = r2;
          q.rmax = sqrt(r2);
          q.phase = PH_RU2;
        }
      }
    }
  }
}

// R4: r = lo(r_hi), p = r + beta p.
template <typename R, int NB>
__global__ void __launch_bounds__(512) k_ru_finish(const SysDesc* __restrict__ sys, int nsys,
                                                   const SrcState* st, int xcd) {
  const int b = logical_block(xcd);
  const SysDesc& d = find_sys(sys, nsys, b);
  const SrcState* q0 = st + d.src0;
  const unsigned act = phase_mask<NB>(q0, d.nsrc, PH_RU2);
  const int cb = (b - d.blk0) * blockDim.x + threadIdx.x;
  if (!act || cb >= d.g.hv) return;
  const size_t hv = d.g.hv, vs = 3 * hv * d.nsrc;
  cplx<R>* r = slot<R>(d.vlo, 1, vs);
  cplx<R>* p = slot<R>(d.vlo, 2, vs);
  const cplx<double>* rhi = slot<double>(d.vhi, 1, vs);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (!(act >> k & 1u)) continue;
    const R be = (R)q0[k].beta;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t j = (k * 3 + a) * hv + cb;
      const cplx<double> h = rhi[j];
      const cplx<R> rv = {(R)h.re, (R)h.im};
      const cplx<R> pv = p[j];
      r[j] = rv;
      p[j] = {fma(be, pv.re, rv.re), fma(be, pv.im, rv.im)};
    }
  }
}

// R5: sources whose update is complete resume iterating.
__global__ void __launch_bounds__(256) k_ru_commit(SrcState* st, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (st[i].phase == PH_RU2) st[i].phase = PH_RUN;
}

bool engine_supported(const EngineCfg& c) {
  const bool ok_lo = (c.prec_lo == 0 || c.prec_lo == 1) && (c.recon_lo == 18 || c.recon_lo == 12);
  const bool ok_hi = c.recon_hi == 18 || c.recon_hi == 12;
  const bool ok_nb = c.nb >= 1 && c.nb <= 12;
  const bool ok_bs = c.shape.block == 64 || c.shape.block == 128 || c.shape.block == 256 ||
                     c.shape.block == 512;
  return ok_lo && ok_hi && ok_nb && ok_bs && c.nsys >= 1 && c.nblk_total >= 1;
}

namespace {
template <typename F>
hipError_t with_lo(const EngineCfg& c, F&& f) {
  return with_prec_recon(c.prec_lo, c.recon_lo, [&]<typename R, int RECON>() {
    return with_nb(c.nb, [&]<int NB>() { return f.template operator()<R, RECON, NB>(); });
  });
}
}  // namespace

hipError_t engine_init(const EngineCfg& c, int zero_xhi, hipStream_t s) {
  const dim3 grid(c.nblk_total), block(c.shape.block);
  return with_lo(c, [&]<typename R, int RECON, int NB>() {
    hipLaunchKernelGGL((k_init<R, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st, zero_xhi,
                       c.shape.xcd);
    hipLaunchKernelGGL((k_zero_done<NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    return hipGetLastError();
  });
}

hipError_t engine_iteration(const EngineCfg& c, hipStream_t s) {
  const dim3 grid(c.nblk_total), block(c.shape.block);
  return with_lo(c, [&]<typename R, int RECON, int NB>() {
    hipLaunchKernelGGL((k_iter_doe<R, RECON, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    hipLaunchKernelGGL((k_iter_deo<R, RECON, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    hipLaunchKernelGGL((k_iter_xr<R, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    hipLaunchKernelGGL((k_iter_p<R, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    return hipGetLastError();
  });
}

hipError_t engine_reliable_update(const EngineCfg& c, hipStream_t s) {
  const dim3 grid(c.nblk_total), block(c.shape.block);
  return with_lo(c, [&]<typename R, int RECON, int NB>() {
    hipLaunchKernelGGL((k_ru_accum<R, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    if (c.recon_hi == 12) {
      hipLaunchKernelGGL((k_ru_doe<12, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                         c.shape.xcd);
      hipLaunchKernelGGL((k_ru_residual<12, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                         c.shape.xcd);
    } else {
      hipLaunchKernelGGL((k_ru_doe<18, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                         c.shape.xcd);
      hipLaunchKernelGGL((k_ru_residual<18, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                         c.shape.xcd);
    }
    hipLaunchKernelGGL((k_ru_finish<R, NB>), grid, block, 0, s, c.d_sys, c.nsys, c.d_st,
                       c.shape.xcd);
    hipLaunchKernelGGL(k_ru_commit, dim3(1), dim3(256), 0, s, c.d_st, c.nsrc_total);
    return hipGetLastError();
  });
}

// ===================================================================== force

// G_mu(z) = 1/2 eps(z) eta_mu(z) bc_mu(z) sum_s [W1 W1(z+mu)^dag + W2 W2(z+mu)^dag](z)
// with W1 = (lam even, y odd), W2 = (x even, nu odd); one thread per site z
// writing its four links of the canonical [4][V][3][3] gradient.
__global__ void __launch_bounds__(256) k_force(Geo g, int nsrc, const cplx<double>* __restrict__ x,
                                               const cplx<double>* __restrict__ lam,
                                               const cplx<double>* __restrict__ y,
                                               const cplx<double>* __restrict__ nu,
                                               cplx<double>* __restrict__ G) {
  const int64_t V = 2 * (int64_t)g.hv;
  const int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  const size_t hv = g.hv;
  int t = (int)lex;
  int xc[4];
  xc[0] = t % g.L0;
  t /= g.L0;
  xc[1] = t % g.L1;
  t /= g.L1;
  xc[2] = t % g.L2;
  xc[3] = t / g.L2;
  const int p = (xc[0] + xc[1] + xc[2] + xc[3]) & 1;
  const size_t cb = (size_t)(lex >> 1);
  const cplx<double>* W1z = p == 0 ? lam : y;
  const cplx<double>* W1n = p == 0 ? y : lam;
  const cplx<double>* W2z = p == 0 ? x : nu;
  const cplx<double>* W2n = p == 0 ? nu : x;
  const int L[4] = {g.L0, g.L1, g.L2, g.L3};
  const int64_t stride[4] = {1, g.L0, (int64_t)g.L0 * g.L1, (int64_t)g.L0 * g.L1 * g.L2};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int64_t ln = xc[mu] + 1 == L[mu] ? lex - (int64_t)(L[mu] - 1) * stride[mu]
                                            : lex + stride[mu];
    const size_t cbn = (size_t)(ln >> 1);
    const double sg = 0.5 * (p ? -1.0 : 1.0) * link_sign(g, mu, xc[0], xc[1], xc[2], xc[3]);
    cplx<double> m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = {0.0, 0.0};
    for (int s = 0; s < nsrc; ++s) {
      cplx<double> a1[3], c1[3], a2[3], c2[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        a1[a] = W1z[(s * 3 + a) * hv + cb];
        c1[a] = W1n[(s * 3 + a) * hv + cbn];
        a2[a] = W2z[(s * 3 + a) * hv + cb];
        c2[a] = W2n[(s * 3 + a) * hv + cbn];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // a * conj(c)
          m[3 * a + c].re += a1[a].re * c1[c].re + a1[a].im * c1[c].im +
                             a2[a].re * c2[c].re + a2[a].im * c2[c].im;
          m[3 * a + c].im += a1[a].im * c1[c].re - a1[a].re * c1[c].im +
                             a2[a].im * c2[c].re - a2[a].re * c2[c].im;
        }
    }
    cplx<double>* o = G + ((int64_t)mu * V + lex) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) o[e] = {sg * m[e].re, sg * m[e].im};
  }
}

// F^a = Re[i tr(T_a Q)] = -1/2 Im[sum_ij (lambda_a)_ij Q_ji], Q = U G^dag,
// written out for the eight Gell-Mann matrices.
__global__ void __launch_bounds__(256) k_su3_force(int64_t nlinks,
                                                   const cplx<double>* __restrict__ U,
                                                   const cplx<double>* __restrict__ G,
                                                   double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlinks) return;
  cplx<double> u[9], gg[9], Q[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    u[e] = U[i * 9 + e];
    gg[e] = G[i * 9 + e];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cplx<double> s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // u[a][k] * conj(g[b][k])
        s.re += u[3 * a + k].re * gg[3 * b + k].re + u[3 * a + k].im * gg[3 * b + k].im;
        s.im += u[3 * a + k].im * gg[3 * b + k].re - u[3 * a + k].re * gg[3 * b + k].im;
      }
      Q[3 * a + b] = s;
    }
  double* f = F + i * 8;
  f[0] = -0.5 * (Q[1].im + Q[3].im);
  f[1] = -0.5 * (Q[1].re - Q[3].re);
  f[2] = -0.5 * (Q[0].im - Q[4].im);
  f[3] = -0.5 * (Q[2].im + Q[6].im);
  f[4] = -0.5 * (Q[2].re - Q[6].re);
  f[5] = -0.5 * (Q[5].im + Q[7].im);
  f[6] = -0.5 * (Q[5].re - Q[7].re);
  f[7] = -0.5 * (Q[0].im + Q[4].im - 2.0 * Q[8].im) * 0.57735026918962576451;
}

__global__ void __launch_bounds__(256) k_redot_partial(const cplx<double>* __restrict__ a,
                                                       const cplx<double>* __restrict__ b,
                                                       size_t n, double* partials) {
  __shared__ double sh[16];
  double v[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    v[0] += a[i].re * b[i].re + a[i].im * b[i].im;
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(256) k_redot_final(const double* partials, int nblk,
                                                     double* out) {
  __shared__ double sh[16];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v[0] += partials[i];
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) *out = v[0];
}

hipError_t launch_force(const Geo& g, int nsrc, const void* x, const void* lam, const void* y,
                        const void* nu, void* G, hipStream_t s) {
  hipLaunchKernelGGL(k_force, dim3(grid_for(2 * (size_t)g.hv, 256)), dim3(256), 0, s, g, nsrc,
                     (const cplx<double>*)x, (const cplx<double>*)lam, (const cplx<double>*)y,
                     (const cplx<double>*)nu, (cplx<double>*)G);
  return hipGetLastError();
}

hipError_t launch_su3_force(const Geo& g, const void* U, const void* G, double* F, hipStream_t s) {
  const int64_t n = 8 * (int64_t)g.hv;
  hipLaunchKernelGGL(k_su3_force, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                     (const cplx<double>*)U, (const cplx<double>*)G, F);
  return hipGetLastError();
}

hipError_t launch_redot(const void* a, const void* b, size_t n, double* partials, int nblk,
                        double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_redot_partial, dim3(nblk), dim3(256), 0, s, (const cplx<double>*)a,
                     (const cplx<double>*)b, n, partials);
  hipLaunchKernelGGL(k_redot_final, dim3(1), dim3(256), 0, s, partials, nblk, out);
  return hipGetLastError();
}

// ================================================================ probe

// Plain copy with 16-byte accesses: the measured-bandwidth reference and the
// calibration kernel for the memory counters.
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(k_copy16, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, (const uint4*)src,
                     (uint4*)dst, n);
  return hipGetLastError();
}

}  // namespace qx
