// Standalone staggered operators: the half-Dslash D_{p, 1-p} and the
// even-site operator A = m^2 - D_eo D_oe, for any number of sources.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "qx_device.h"
#include "qx_dispatch.h"
#include "qx_launch.h"

namespace qx {

// out_k = scale * (2D in_k) at the sites of parity pout.  Block: 64 sites and
// LPS * G wavefronts; wavefront w takes hop part w % LPS of the sources
// (w / LPS) * NBT ... + NBT - 1.  LL (LPS 1, G >= 2): the G wavefronts share
// the tile's link loads through LDS (stage_links).
template <typename R, int RECON, int NBT, int LPS, bool LL = false>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>)) k_dslash(Geo g, const cplx<R>* __restrict__ links, int pout,
                                                 const cplx<R>* __restrict__ in,
                                                 cplx<R>* __restrict__ out, int nsrc, R scale,
                                                 int xcd) {
  static_assert(!LL || LPS == 1, "shared links need one wavefront per site");
  cplx<R>* red = reinterpret_cast<cplx<R>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id();
  const int dp = w % LPS, grp = w / LPS;
  const int cb = tile_block(logical_block(xcd), g, xcd) * kTile + lane;
  const size_t hv = g.hv, ss = 3 * hv;
  const int k0 = grp * NBT;
  const int jmax = nsrc - 1 - k0;  // last source slot of the group
  const bool nt = order_nt(xcd);
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  if constexpr (LL) {
    const int ci = cb < g.hv ? cb : g.hv - 1;
    Site s;
    site_geometry(g, pout, ci, s);
    stage_links<RECON>(g, links, pout, ci, s, w, (int)(blockDim.x >> 6),
                       reinterpret_cast<qx_u32x4*>(qx_lds), lane);
    __syncthreads();
    if (cb < g.hv && jmax >= 0)
      stencil_part_ll<R, RECON, NBT, false>(g, links, cb, s,
                                            FieldIn<R>{in + k0 * ss, ss, hv, jmax},
                                            reinterpret_cast<const qx_u32x4*>(qx_lds), acc);
  } else if (cb < g.hv && jmax >= 0) {
    Site s;
    site_geometry(g, pout, cb, s);
    stencil_part<R, RECON, NBT, LPS, false>(g, links, pout, cb, s, dp,
                                     FieldIn<R>{in + k0 * ss, ss, hv, jmax}, acc);
  }
  for_each_item<R, NBT, LPS>(acc, red, dp, grp, lane, [&](int j, int c, cplx<R> v) {
    if (j <= jmax && cb < g.hv)
      st_cplx(out + (k0 + j) * ss + c * hv + cb, cplx<R>{scale * v.re, scale * v.im}, nt);
  });
}

// As k_dslash for FP16 storage (links and colour vectors with per-site
// scales), FP32 arithmetic; each output site is written with its own scale.
template <int RECON, int NBT, int LPS>
__global__ void __launch_bounds__((kMaxThreads<float, NBT>)) k_dslash_h(
    Geo g, const cplx<__half>* __restrict__ links, int pout, const char* __restrict__ in,
    char* __restrict__ out, int nsrc, float scale, int xcd) {
  cplx<float>* red = reinterpret_cast<cplx<float>*>(qx_lds);
  const int lane = threadIdx.x & 63, w = wave_id();
  const int dp = w % LPS, grp = w / LPS;
  const int cb = tile_block(logical_block(xcd), g, xcd) * kTile + lane;
  const size_t hv = g.hv, ss = 16 * hv;
  const int k0 = grp * NBT;
  const int jmax = nsrc - 1 - k0;
  cplx<float> acc[NBT][3];
  zero_acc<float, NBT>(acc);
  if (cb < g.hv && jmax >= 0) {
    Site s;
    site_geometry(g, pout, cb, s);
    stencil_part<float, RECON, NBT, LPS, false>(g, links, pout, cb, s, dp,
                                         FieldInH{in + k0 * ss, hv, jmax}, acc);
  }
  for_each_slot<float, NBT, LPS>(acc, red, dp, grp, lane, [&](int j, const cplx<float>(&v)[3]) {
    if (j > jmax || cb >= g.hv) return;
    const cplx<float> o[3] = {{scale * v[0].re, scale * v[0].im},
                              {scale * v[1].re, scale * v[1].im},
                              {scale * v[2].re, scale * v[2].im}};
    st_field_h(out + (k0 + j) * ss, cb, o);
  });
}

struct Masses16 {
  double m2[16];
};

// out_k = m2_k p_k - 1/4 (2D_eo) t_k at even sites, t = 2 D_oe p (odd sites).
template <typename R, int RECON, int NBT>
__global__ void __launch_bounds__((kMaxThreads<R, NBT>)) k_deo_axpy(Geo g, const cplx<R>* __restrict__ links,
                                                   const cplx<R>* __restrict__ t,
                                                   const cplx<R>* __restrict__ p,
                                                   cplx<R>* __restrict__ out, int nsrc, Masses16 m,
                                                   int xcd) {
  const int lane = threadIdx.x & 63, grp = wave_id();
  const int cb = tile_block(logical_block(xcd), g, xcd) * kTile + lane;
  const size_t hv = g.hv, ss = 3 * hv;
  const int k0 = grp * NBT;
  const int jmax = nsrc - 1 - k0;
  if (cb >= g.hv || jmax < 0) return;
  cplx<R> acc[NBT][3];
  zero_acc<R, NBT>(acc);
  Site s;
  site_geometry(g, 0, cb, s);
  stencil_part<R, RECON, NBT, 1, false>(g, links, 0, cb, s, 0, FieldIn<R>{t + k0 * ss, ss, hv, jmax},
                                        acc);
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    if (j > jmax) continue;
    const R m2 = (R)m.m2[k0 + j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t i = (k0 + j) * ss + c * hv + cb;
      const cplx<R> pv = p[i];
      out[i] = {fmadd(m2, pv.re, (R)-0.25 * acc[j][c].re), fmadd(m2, pv.im, (R)-0.25 * acc[j][c].im)};
    }
  }
}

// As k_deo_axpy for FP16 storage, FP32 arithmetic.
template <int RECON, int NBT>
__global__ void __launch_bounds__((kMaxThreads<float, NBT>)) k_deo_axpy_h(
    Geo g, const cplx<__half>* __restrict__ links, const char* __restrict__ t,
    const char* __restrict__ p, char* __restrict__ out, int nsrc, Masses16 m, int xcd) {
  const int lane = threadIdx.x & 63, grp = wave_id();
  const int cb = tile_block(logical_block(xcd), g, xcd) * kTile + lane;
  const size_t hv = g.hv, ss = 16 * hv;
  const int k0 = grp * NBT;
  const int jmax = nsrc - 1 - k0;
  if (cb >= g.hv || jmax < 0) return;
  cplx<float> acc[NBT][3];
  zero_acc<float, NBT>(acc);
  Site s;
  site_geometry(g, 0, cb, s);
  stencil_part<float, RECON, NBT, 1, false>(g, links, 0, cb, s, 0, FieldInH{t + k0 * ss, hv, jmax},
                                            acc);
  const FieldInH pin{p + k0 * ss, hv, jmax};
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    if (j > jmax) continue;
    const float m2 = (float)m.m2[k0 + j];
    cplx<float> o[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx<float> pv = pin(j, c, cb);
      o[c] = {fmadd(m2, pv.re, -0.25f * acc[j][c].re), fmadd(m2, pv.im, -0.25f * acc[j][c].im)};
    }
    st_field_h(out + (k0 + j) * ss, cb, o);
  }
}

namespace {
// Most sources one launch of this shape can take.
int sources_per_pass(const LaunchShape& sh, size_t csz) {
  int n = (16 / sh.lps) * sh.nbt;
  while (n > 1 && !shape_ok(sh, n, csz)) --n;
  return n;
}
}  // namespace

hipError_t launch_dslash(const Geo& g, int prec, int recon, const void* links, int pout,
                         const void* in, void* out, int nsrc, double scale, LaunchShape sh,
                         hipStream_t s) {
  const size_t csz = cplx_bytes(prec);
  const bool wide = wide_compiled(prec, recon);
  if (!wide) sh = narrow_shape(sh);
  if (!nbt_lps_instantiated(sh.nbt, sh.lps, wide) || !shape_ok(sh, 1, csz)) return hipErrorInvalidValue;
  const size_t field = source_bytes(g, prec);
  const int per = sources_per_pass(sh, csz);
  const unsigned grid = grid_for(g.hv, kTile);
  const size_t link_bytes = (size_t)8 * g.hv * (recon / 2) * link_cplx_bytes(prec);
  for (int k0 = 0; k0 < nsrc; k0 += per) {
    const int n = std::min(per, nsrc - k0);
    const int threads = 64 * sh.lps * shape_groups(sh, n);
    Geo gl = g;
    gl.stream_links = link_bytes > kStreamLinkBytes && shape_groups(sh, n) == 1;
    const size_t lds = shape_lds(sh, n, csz);
    const char* pin = (const char*)in + k0 * field;
    char* po = (char*)out + k0 * field;
    if (prec == 2) {
      hipError_t e = with_recon(recon, [&]<int RECON>() {
        return with_nbt_lps<false>(sh.nbt, sh.lps, [&]<int NBT, int LPS>() {
          hipLaunchKernelGGL((k_dslash_h<RECON, NBT, LPS>), dim3(grid), dim3(threads), lds, s, gl,
                             (const cplx<__half>*)links, pout, pin, po, n, (float)scale, sh.xcd);
          return hipGetLastError();
        });
      });
      if (e != hipSuccess) return e;
      continue;
    }
    hipError_t e = with_prec_recon(prec, recon, [&]<typename R, int RECON>() {
      return with_nbt_lps<(sizeof(R) == 4 && RECON != 36)>(sh.nbt, sh.lps, [&]<int NBT, int LPS>() {
        // several source groups of one wavefront per site share the link loads
        constexpr size_t kLL = kLinkLdsBytes<RECON, R>;
        if constexpr (LPS == 1 && kLL != 0) {
          if (shape_groups(sh, n) >= 2) {
            hipLaunchKernelGGL((k_dslash<R, RECON, NBT, 1, true>), dim3(grid), dim3(threads), kLL,
                               s, gl, (const cplx<R>*)links, pout, (const cplx<R>*)pin,
                               (cplx<R>*)po, n, (R)scale, sh.xcd);
            return hipGetLastError();
          }
        }
        hipLaunchKernelGGL((k_dslash<R, RECON, NBT, LPS>), dim3(grid), dim3(threads), lds, s, gl,
                           (const cplx<R>*)links, pout, (const cplx<R>*)pin, (cplx<R>*)po, n,
                           (R)scale, sh.xcd);
        return hipGetLastError();
      });
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_apply_A(const Geo& g, int prec, int recon, const void* links, int nrhs,
                          const double* m2, const void* in, void* out, void* tmp, LaunchShape sh,
                          hipStream_t s, bool square) {
  hipError_t e = launch_dslash(g, prec, recon, links, 1, in, tmp, nrhs, 1.0, sh, s);
  if (e != hipSuccess) return e;
  const size_t field = source_bytes(g, prec);
  const int per = 16;  // Masses16 holds one pass
  const unsigned grid = grid_for(g.hv, kTile);
  for (int k0 = 0; k0 < nrhs; k0 += per) {
    const int n = std::min(per, nrhs - k0);
    Masses16 m{};
    for (int k = 0; k < n; ++k) m.m2[k] = square ? m2[k0 + k] * m2[k0 + k] : m2[k0 + k];
    const int nbt = narrow_nbt(sh.nbt);  // the A epilogue kernels take at most four
    const int threads = 64 * ((n + nbt - 1) / nbt);
    if (prec == 2) {
      e = with_recon(recon, [&]<int RECON>() {
        return with_nbt(nbt, [&]<int NBT>() {
          hipLaunchKernelGGL((k_deo_axpy_h<RECON, NBT>), dim3(grid), dim3(threads), 0, s, g,
                             (const cplx<__half>*)links, (const char*)tmp + k0 * field,
                             (const char*)in + k0 * field, (char*)out + k0 * field, n, m, sh.xcd);
          return hipGetLastError();
        });
      });
      if (e != hipSuccess) return e;
      continue;
    }
    e = with_prec_recon(prec, recon, [&]<typename R, int RECON>() {
      return with_nbt(nbt, [&]<int NBT>() {
        hipLaunchKernelGGL((k_deo_axpy<R, RECON, NBT>), dim3(grid), dim3(threads), 0, s, g,
                           (const cplx<R>*)links, (const cplx<R>*)((const char*)tmp + k0 * field),
                           (const cplx<R>*)((const char*)in + k0 * field),
                           (cplx<R>*)((char*)out + k0 * field), n, m, sh.xcd);
        return hipGetLastError();
      });
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------ allocation-free operator
//
// The D_oe intermediate of the allocation-free A lives in a file-scope device
// array (one per GPU, held until the process ends).  In host code the array's
// name is not a device address: its address on the current device comes from
// hipGetSymbolAddress, looked up once per device and kept in noalloc_ptr.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_apply_A_noalloc(const Geo& g, int prec, int recon, const void* links, int nrhs,
                                  const double* masses, const void* in, void* out, LaunchShape sh,
                                  hipStream_t s) {
  if ((size_t)nrhs * source_bytes(g, prec) > kNoAllocScratchBytes) return hipErrorInvalidValue;
  void* tmp = nullptr;
  const hipError_t e = noalloc_scratch(&tmp);
  if (e != hipSuccess) return e;
  // every element of the odd intermediate is written by the D_oe launch
  // before A's epilogue reads it: nothing to clear
  return launch_apply_A(g, prec, recon, links, nrhs, masses, in, out, tmp, sh, s, true);
}

}  // namespace qx
