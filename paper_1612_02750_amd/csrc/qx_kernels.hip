// gfx950 kernels of libqx.so outside the stencil: packing of gauge fields and
// colour vectors, the device index maps, the fermion force and its su(3)
// projection, a deterministic dot product and the bandwidth probe.
//
// Operator (textbook Kogut-Susskind form of the staggered operator the paper
// names in Sec. 4):
//   (D chi)(x) = 1/2 sum_mu eta_mu(x) [bc U_mu(x) chi(x+mu) - bc U_mu(x-mu)^dag chi(x-mu)]
// The packed links carry eta * bc (folded here at pack time); the stencil
// kernels compute 2D and apply the factor 1/2 (or 1/4 for D_eo D_oe) in
// their epilogues.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/qx.h"
#include "qx_device.h"
#include "qx_dispatch.h"
#include "qx_launch.h"

namespace qx {

// =================================================================== packing

// An FP64 value in the storage type S, rounded once to nearest (ties to even).
// (FP16 is converted straight from FP64: a detour through FP32 would round
// twice, and differ where the FP32 value lands on a binary16 tie.)
template <typename S>
__device__ __forceinline__ S to_store(double x) {
  if constexpr (std::is_same_v<S, __half>)
    return __half_raw{static_cast<_Float16>(x)};
  else
    return (S)x;
}

// Canonical complex128 [4][V][3][3] -> packed links (one region per parity
// and mu, elements in 16-byte chunks, link_elem_offset) with the staggered
// phase and boundary sign folded in.  With 12-real storage the FP64
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
    char* o = reinterpret_cast<char*>(out + (size_t)(p * 4 + mu) * E * g.hv);
#pragma unroll
    for (int e = 0; e < E; ++e)
      *reinterpret_cast<cplx<R>*>(o + link_elem_offset<R, E>(e, g.hv, cb)) = {
          to_store<R>(sg * v[e].re), to_store<R>(sg * v[e].im)};
    if constexpr (RECON == 12) {
      // U in SU(3) <=> rows 0 and 1 orthonormal and row 2 = conj(row0 x row1):
      // the largest deviation from the three conditions, +inf when any of the
      // 18 reals is not finite (fmax would drop a NaN)
      bool fin = true;
#pragma unroll
      for (int e = 0; e < 9; ++e) fin = fin && isfinite(v[e].re) && isfinite(v[e].im);
      const cplx<double> a0 = cmul(v[1], v[5]), b0 = cmul(v[2], v[4]);
      const cplx<double> a1 = cmul(v[2], v[3]), b1 = cmul(v[0], v[5]);
      const cplx<double> a2 = cmul(v[0], v[4]), b2 = cmul(v[1], v[3]);
      const double d0 = fabs(v[6].re - (a0.re - b0.re)) + fabs(v[6].im + (a0.im - b0.im));
      const double d1 = fabs(v[7].re - (a1.re - b1.re)) + fabs(v[7].im + (a1.im - b1.im));
      const double d2 = fabs(v[8].re - (a2.re - b2.re)) + fabs(v[8].im + (a2.im - b2.im));
      double n0 = 0.0, n1 = 0.0, o_re = 0.0, o_im = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        n0 += v[c].re * v[c].re + v[c].im * v[c].im;
        n1 += v[3 + c].re * v[3 + c].re + v[3 + c].im * v[3 + c].im;
        // row0 . conj(row1)
        o_re += v[c].re * v[3 + c].re + v[c].im * v[3 + c].im;
        o_im += v[c].im * v[3 + c].re - v[c].re * v[3 + c].im;
      }
      err = fmax(fmax(fmax(d0, d1), d2),
                 fmax(fmax(fabs(n0 - 1.0), fabs(n1 - 1.0)), fabs(o_re) + fabs(o_im)));
      if (!fin) err = __builtin_inf();
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

// canonical complex128 [nsrc][hv][3] -> FP16 packed: per source [3][hv]
// binary16 pairs, then [hv] FP32 scales.  The scale of a site is the largest
// |re| or |im| of its three colours (as FP32); the stored pairs are the
// components divided by it (zero where the scale is zero).
__global__ void __launch_bounds__(256) k_pack_field_h(int hv, int nsrc,
                                                      const cplx<double>* __restrict__ in,
                                                      char* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nsrc * hv) return;
  const int64_t s = i / hv, cb = i - s * hv;
  cplx<double> v[3];
  double m = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v[c] = in[i * 3 + c];
    m = fmax(m, fmax(fabs(v[c].re), fabs(v[c].im)));
  }
  const float sc = (float)m;
  const double inv = sc > 0.0f ? 1.0 / (double)sc : 0.0;
  // one 16-byte record per site: three half-precision complex numbers (each
  // part the FP64 quotient rounded once to binary16), the scale
  char* rec = out + (s * (int64_t)hv + cb) * 16;
  cplx<__half>* h = reinterpret_cast<cplx<__half>*>(rec);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    h[c] = {__half_raw{static_cast<_Float16>(v[c].re * inv)},
            __half_raw{static_cast<_Float16>(v[c].im * inv)}};
  reinterpret_cast<float*>(rec)[3] = sc;
}

__global__ void __launch_bounds__(256) k_unpack_field_h(int hv, int nsrc,
                                                        const char* __restrict__ in,
                                                        cplx<double>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nsrc * hv) return;
  const char* rec = in + i * 16;  // the site's record (source-major, i = s hv + cb)
  const cplx<__half>* h = reinterpret_cast<const cplx<__half>*>(rec);
  const double sc = (double)reinterpret_cast<const float*>(rec)[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<__half> v = h[c];
    out[i * 3 + c] = {(double)__half2float(v.re) * sc, (double)__half2float(v.im) * sc};
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
    nbr[eo * 8 + mu] = other + s.fwd(mu);
    nbr[eo * 8 + 4 + mu] = other + s.bwd(mu);
  }
}

// Links of the improved operator (one-hop and Naik three-hop terms): for
// every (mu, site x) the one-hop link 9/8 eta bc U_mu(x) and the three-hop
// transporter -1/24 eta bc(x) bc(x+mu) bc(x+2mu) U_mu(x) U_mu(x+mu) U_mu(x+2mu)
// (eta_mu is the same at the three sites), products in FP64.  Regions
// [kind][parity][mu] of 9-element links (link_elem_offset): kind 0 the
// one-hop links, kind 1 the three-hop.
template <typename R>
__global__ void __launch_bounds__(256) k_pack_gauge_naik(Geo g, const cplx<double>* __restrict__ U,
                                                         cplx<R>* __restrict__ out) {
  const int64_t V = 2 * (int64_t)g.hv;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * V) return;
  const int mu = (int)(i / V);
  const int lex = (int)(i - mu * V);
  int x[4];
  {
    int t = lex;
    x[0] = t % g.L0;
    t /= g.L0;
    x[1] = t % g.L1;
    t /= g.L1;
    x[2] = t % g.L2;
    x[3] = t / g.L2;
  }
  const int L[4] = {g.L0, g.L1, g.L2, g.L3};
  const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  const int cb = lex >> 1;
  const double eta = (double)eta_sign(mu, x[0], x[1], x[2]);
  // walk three links along mu
  cplx<double> P[9];
  double sgn = 1.0;
  int y[4] = {x[0], x[1], x[2], x[3]};
  for (int step = 0; step < 3; ++step) {
    const int ly = y[0] + L[0] * (y[1] + L[1] * (y[2] + L[2] * y[3]));
    const cplx<double>* u = U + ((int64_t)mu * V + ly) * 9;
    if (mu == 3 && g.anti_t && y[3] == L[3] - 1) sgn = -sgn;
    if (step == 0) {
#pragma unroll
      for (int e = 0; e < 9; ++e) P[e] = u[e];
      char* o = reinterpret_cast<char*>(out + (size_t)(p * 4 + mu) * 9 * g.hv);
      const double c = 1.125 * eta * sgn;
#pragma unroll
      for (int e = 0; e < 9; ++e)
        *reinterpret_cast<cplx<R>*>(o + link_elem_offset<R, 9>(e, g.hv, cb)) = {
            to_store<R>(c * P[e].re), to_store<R>(c * P[e].im)};
    } else {
      cplx<double> Q[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          cplx<double> t = {0.0, 0.0};
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const cplx<double> m = cmul(P[3 * a + c], u[3 * c + b]);
            t.re += m.re;
            t.im += m.im;
          }
          Q[3 * a + b] = t;
        }
#pragma unroll
      for (int e = 0; e < 9; ++e) P[e] = Q[e];
    }
    y[mu] = y[mu] + 1 == L[mu] ? 0 : y[mu] + 1;
  }
  char* o = reinterpret_cast<char*>(out + (size_t)(8 + p * 4 + mu) * 9 * g.hv);
  const double c = (-1.0 / 24.0) * eta * sgn;
#pragma unroll
  for (int e = 0; e < 9; ++e)
    *reinterpret_cast<cplx<R>*>(o + link_elem_offset<R, 9>(e, g.hv, cb)) = {
        to_store<R>(c * P[e].re), to_store<R>(c * P[e].im)};
}

hipError_t launch_pack_gauge(const Geo& g, const void* U, int prec, int recon, void* packed,
                             unsigned long long* err_bits, hipStream_t s) {
  const size_t n = 8 * (size_t)g.hv;
  if (prec == 2) {
    const unsigned grid = grid_for(n, 256);
    const cplx<double>* u = (const cplx<double>*)U;
    cplx<__half>* o = (cplx<__half>*)packed;
    if (recon == 36)
      hipLaunchKernelGGL(k_pack_gauge_naik<__half>, dim3(grid), dim3(256), 0, s, g, u, o);
    else if (recon == 18)
      hipLaunchKernelGGL((k_pack_gauge<__half, 18>), dim3(grid), dim3(256), 0, s, g, u, o, err_bits);
    else if (recon == 12)
      hipLaunchKernelGGL((k_pack_gauge<__half, 12>), dim3(grid), dim3(256), 0, s, g, u, o, err_bits);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (recon == 36)
    return with_prec(prec, [&]<typename R>() {
      hipLaunchKernelGGL(k_pack_gauge_naik<R>, dim3(grid_for(n, 256)), dim3(256), 0, s, g,
                         (const cplx<double>*)U, (cplx<R>*)packed);
      return hipGetLastError();
    });
  return with_prec_recon(prec, recon, [&]<typename R, int RECON>() {
    if constexpr (RECON == 36) {
      return hipErrorInvalidValue;
    } else {
      hipLaunchKernelGGL((k_pack_gauge<R, RECON>), dim3(grid_for(n, 256)), dim3(256), 0, s, g,
                         (const cplx<double>*)U, (cplx<R>*)packed, err_bits);
      return hipGetLastError();
    }
  });
}

hipError_t launch_pack_field(const Geo& g, int nrhs, int prec, const void* canon, void* packed,
                             hipStream_t s) {
  const size_t n = (size_t)nrhs * g.hv;
  if (prec == 2)
    hipLaunchKernelGGL(k_pack_field_h, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv, nrhs,
                       (const cplx<double>*)canon, (char*)packed);
  else if (prec == 0)
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
  if (prec == 2)
    hipLaunchKernelGGL(k_unpack_field_h, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv, nrhs,
                       (const char*)packed, (cplx<double>*)canon);
  else if (prec == 0)
    hipLaunchKernelGGL(k_unpack_field<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv,
                       nrhs, (const cplx<double>*)packed, (cplx<double>*)canon);
  else
    hipLaunchKernelGGL(k_unpack_field<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv,
                       nrhs, (const cplx<float>*)packed, (cplx<double>*)canon);
  return hipGetLastError();
}

// Per-source statistics of a solve from the device states (no host copy): a
// source that has not finished reports QX_ENOTCONVERGED, and a timed-out grid
// barrier of the persistent engine QX_EHIP for every source.
__global__ void __launch_bounds__(256) k_batch_stats(const SrcState* __restrict__ st, int n,
                                                     const GridSync* __restrict__ gs,
                                                     qx_cg_stats_t* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const SrcState q = st[k];
  qx_cg_stats_t r;
  r.status = q.phase == PH_DONE ? q.status : QX_ENOTCONVERGED;
  if (gs && gs->error) r.status = QX_EHIP;
  r.iters = q.iters;
  r.reliable_updates = q.updates;
  r.true_rel_residual = q.relres;
  r.seconds = 0.0;
  out[k] = r;
}

hipError_t launch_batch_stats(const void* st, int n, const void* gs, void* out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_stats, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s,
                     (const SrcState*)st, n, (const GridSync*)gs, (qx_cg_stats_t*)out);
  return hipGetLastError();
}

hipError_t launch_index_maps(const Geo& g, int32_t* lex_of_eo, int32_t* nbr_eo, hipStream_t s) {
  hipLaunchKernelGGL(k_index_maps, dim3(grid_for(2 * (size_t)g.hv, 256)), dim3(256), 0, s, g,
                     lex_of_eo, nbr_eo);
  return hipGetLastError();
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

// out = s * in over n complex128 values (grid-stride).
__global__ void __launch_bounds__(256) k_scale_c128(size_t n, double sc,
                                                    const cplx<double>* __restrict__ in,
                                                    cplx<double>* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const cplx<double> v = in[i];
    out[i] = {sc * v.re, sc * v.im};
  }
}

hipError_t launch_scale_c128(const void* in, double sc, size_t n, void* out, hipStream_t s) {
  if (!n) return hipSuccess;
  const unsigned grid = (unsigned)std::min<size_t>(grid_for(n, 256), 65536);
  hipLaunchKernelGGL(k_scale_c128, dim3(grid), dim3(256), 0, s, n, sc, (const cplx<double>*)in,
                     (cplx<double>*)out);
  return hipGetLastError();
}

// ================================================================ mesons

// Canonical point sources: b[c][cb][a] = (a == c && cb == cb_src) for the three
// colours c.
__global__ void __launch_bounds__(256) k_point_source(int hv, int cb_src,
                                                      cplx<double>* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * (int64_t)hv) return;
  const int c = (int)(i / (3 * (int64_t)hv));
  const int64_t r = i - c * 3 * (int64_t)hv;
  const int cb = (int)(r / 3), a = (int)(r % 3);
  b[i] = {(a == c && cb == cb_src) ? 1.0 : 0.0, 0.0};
}

constexpr int kMaxMasks = 16;
struct Masks16 {
  int m[kMaxMasks];
};

// One block per timeslice x3: C[k][(x3 - t_src) mod L3] = sum over the sites of
// the timeslice of s_k(x) |G(x)|^2, with |G|^2 = m^2 |x|^2 on even sites and
// |y|^2 on odd sites (x, y packed [3 sources][3 colours][cb]), s_k(x) =
// (-1)^(sum of x_mu over the bits of mask k).  Fixed summation order.
__global__ void __launch_bounds__(256) k_meson_contract(Geo g, const cplx<double>* __restrict__ xp,
                                                        const cplx<double>* __restrict__ yp,
                                                        double m2, int t_src, int nmask, Masks16 mk,
                                                        double* __restrict__ C) {
  __shared__ double sh[kMaxMasks * 16];
  const int x3 = blockIdx.x;
  const int per = g.s3;  // checkerboard sites of one parity per timeslice
  const size_t hv = g.hv;
  double acc[kMaxMasks];
#pragma unroll
  for (int k = 0; k < kMaxMasks; ++k) acc[k] = 0.0;
  for (int j = threadIdx.x; j < 2 * per; j += blockDim.x) {
    const int p = j >= per ? 1 : 0;
    const int cb = x3 * per + (j - p * per);
    Site s;
    site_geometry(g, p, cb, s);
    const cplx<double>* f = p ? yp : xp;
    double d = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) {  // three sources x three colours
      const cplx<double> v = f[(size_t)e * hv + cb];
      d += v.re * v.re + v.im * v.im;
    }
    if (!p) d *= m2;
    const int xs[4] = {s.x0, s.x1, s.x2, s.x3};
#pragma unroll
    for (int k = 0; k < kMaxMasks; ++k) {
      if (k >= nmask) break;
      int e = 0;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu)
        if (mk.m[k] >> mu & 1) e += xs[mu];
      acc[k] += (e & 1) ? -d : d;
    }
  }
  block_sum<kMaxMasks>(acc, sh);
  if (threadIdx.x == 0) {
    const int t = (x3 - t_src + g.L3) % g.L3;
    for (int k = 0; k < nmask; ++k) C[(size_t)k * g.L3 + t] = acc[k];
  }
}

hipError_t launch_point_source(const Geo& g, int cb_src, void* b, hipStream_t s) {
  const size_t n = 9 * (size_t)g.hv;
  hipLaunchKernelGGL(k_point_source, dim3(grid_for(n, 256)), dim3(256), 0, s, g.hv, cb_src,
                     (cplx<double>*)b);
  return hipGetLastError();
}

hipError_t launch_meson_contract(const Geo& g, const void* xp, const void* yp, double mass,
                                 int t_src, int nmask, const int* masks, double* C, hipStream_t s) {
  if (nmask < 1 || nmask > kMaxMasks) return hipErrorInvalidValue;
  Masks16 mk{};
  for (int k = 0; k < nmask; ++k) mk.m[k] = masks[k];
  hipLaunchKernelGGL(k_meson_contract, dim3(g.L3), dim3(256), 0, s, g, (const cplx<double>*)xp,
                     (const cplx<double>*)yp, mass * mass, t_src, nmask, mk, C);
  return hipGetLastError();
}

// ================================================================ probe

// Plain copy with 16-byte accesses, four independent loads in flight per
// thread: the measured-bandwidth reference and the calibration kernel for the
// memory counters.
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Read-only streaming pass: non-temporal 16-byte loads, four in flight per
// thread; the xor of the words of each block goes to out[block % 8192] so that
// nothing is elided.
__global__ void __launch_bounds__(256) k_read16(const uint4* __restrict__ src, size_t n,
                                                unsigned* __restrict__ out) {
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
  const v4u* s = reinterpret_cast<const v4u*>(src);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned acc = 0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4u a = __builtin_nontemporal_load(s + i), b = __builtin_nontemporal_load(s + i + stride),
              c = __builtin_nontemporal_load(s + i + 2 * stride),
              d = __builtin_nontemporal_load(s + i + 3 * stride);
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n; i += stride) {
    const v4u a = __builtin_nontemporal_load(s + i);
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  for (int off = 32; off >= 1; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) atomicXor(out + (blockIdx.x & 8191), acc);
}

hipError_t launch_read(const void* src, size_t bytes, unsigned* out, hipStream_t s) {
  const size_t n = bytes / 16;
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_read16, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, (const uint4*)src, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 16;
  const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 32);
  hipLaunchKernelGGL(k_copy16, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, (const uint4*)src,
                     (uint4*)dst, n);
  return hipGetLastError();
}

}  // namespace qx
