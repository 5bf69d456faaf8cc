// Hybrid-Monte-Carlo molecular dynamics on gfx950, FP64, on the canonical
// layouts (links U [4][V][3][3] complex, momenta p [4][V][8] real, x0 fastest):
// the Wilson plaquette action and its link gradient (staples), the momentum
// and link updates of the leapfrog integrator, and the kinetic energy.  The
// pseudofermion force comes from the solver and k_force.
#include <hip/hip_runtime.h>

#include "qx_device.h"
#include "qx_dispatch.h"
#include "qx_launch.h"
#include "qx_su3.h"

namespace qx {

namespace {

// Lexicographic neighbour x + step * mu (step = +-1) with periodic wrap.
__device__ __forceinline__ int64_t lex_step(const int (&L)[4], const int64_t (&st)[4],
                                            const int (&x)[4], int64_t lex, int mu, int step) {
  const int y = x[mu] + step;
  if (y == L[mu]) return lex + st[mu] - (int64_t)L[mu] * st[mu];
  if (y < 0) return lex + (int64_t)(L[mu] - 1) * st[mu];
  return lex + step * st[mu];
}

__device__ __forceinline__ void coords(const Geo& g, int64_t lex, int (&x)[4], int (&L)[4],
                                       int64_t (&st)[4]) {
  L[0] = g.L0;
  L[1] = g.L1;
  L[2] = g.L2;
  L[3] = g.L3;
  st[0] = 1;
  st[1] = L[0];
  st[2] = st[1] * L[1];
  st[3] = st[2] * L[2];
  int64_t t = lex;
  x[0] = (int)(t % L[0]);
  t /= L[0];
  x[1] = (int)(t % L[1]);
  t /= L[1];
  x[2] = (int)(t % L[2]);
  x[3] = (int)(t / L[2]);
}

__device__ __forceinline__ void load9(const c64* __restrict__ U, int64_t V, int mu, int64_t lex,
                                      c64* m) {
  const c64* p = U + ((int64_t)mu * V + lex) * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = p[e];
}

}  // namespace

// Per-block partial sums of sum_{mu<nu} (1 - Re tr P_munu(x) / 3) over the
// sites of a grid-stride loop; Re tr P = Re <B, A> for A = U_mu(x) U_nu(x+mu),
// B = U_nu(x) U_mu(x+nu).
__global__ void __launch_bounds__(256) k_plaq_partial(Geo g, const c64* __restrict__ U,
                                                      double* __restrict__ partials) {
  __shared__ double sh[16];
  const int64_t V = 2 * (int64_t)g.hv;
  double v[1] = {0.0};
  for (int64_t lex = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; lex < V;
       lex += (int64_t)gridDim.x * blockDim.x) {
    int x[4], L[4];
    int64_t st[4];
    coords(g, lex, x, L, st);
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        c64 a[9], b[9], u1[9], u2[9];
        load9(U, V, mu, lex, u1);
        load9(U, V, nu, lex_step(L, st, x, lex, mu, 1), u2);
        m3_mul(u1, u2, a);
        load9(U, V, nu, lex, u1);
        load9(U, V, mu, lex_step(L, st, x, lex, nu, 1), u2);
        m3_mul(u1, u2, b);
        double tr = 0.0;
#pragma unroll
        for (int e = 0; e < 9; ++e) tr += a[e].re * b[e].re + a[e].im * b[e].im;
        v[0] += 1.0 - tr / 3.0;
      }
  }
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// G_mu(x) (+)= -(beta/3) A_mu(x)^dag, A the sum of the six staples
//   U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu).
__global__ void __launch_bounds__(256) k_gauge_grad(Geo g, const c64* __restrict__ U, double beta,
                                                    c64* __restrict__ G, int accumulate) {
  const int64_t V = 2 * (int64_t)g.hv;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * V) return;
  const int mu = (int)(i / V);
  const int64_t lex = i - mu * V;
  int x[4], L[4];
  int64_t st[4];
  coords(g, lex, x, L, st);
  c64 A[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) A[e] = {0.0, 0.0};
  const int64_t xpmu = lex_step(L, st, x, lex, mu, 1);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    c64 u1[9], u2[9], t[9], s[9];
    // upper staple
    load9(U, V, nu, xpmu, u1);
    load9(U, V, mu, lex_step(L, st, x, lex, nu, 1), u2);
    m3_mul_nd(u1, u2, t);
    load9(U, V, nu, lex, u1);
    m3_mul_nd(t, u1, s);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      A[e].re += s[e].re;
      A[e].im += s[e].im;
    }
    // lower staple: (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu)
    int xm[4] = {x[0], x[1], x[2], x[3]};
    const int64_t xmnu = lex_step(L, st, x, lex, nu, -1);
    xm[nu] = x[nu] == 0 ? L[nu] - 1 : x[nu] - 1;
    load9(U, V, mu, xmnu, u1);
    load9(U, V, nu, lex_step(L, st, xm, xmnu, mu, 1), u2);
    m3_mul(u1, u2, t);
    load9(U, V, nu, xmnu, u1);
    m3_mul_dn(t, u1, s);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      A[e].re += s[e].re;
      A[e].im += s[e].im;
    }
  }
  const double c = -beta / 3.0;
  c64* o = G + i * 9;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      // (A^dag)_ab = conj(A_ba)
      const c64 v = {c * A[3 * b + a].re, -c * A[3 * b + a].im};
      if (accumulate) {
        const c64 w = o[3 * a + b];
        o[3 * a + b] = {w.re + v.re, w.im + v.im};
      } else {
        o[3 * a + b] = v;
      }
    }
}

// p^a -= eps F^a, F^a = Re[i tr(T_a U G^dag)] for every link.
__global__ void __launch_bounds__(256) k_mom_update(int64_t nlinks, const c64* __restrict__ U,
                                                    const c64* __restrict__ G, double eps,
                                                    double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlinks) return;
  c64 u[9], gg[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    u[e] = U[i * 9 + e];
    gg[e] = G[i * 9 + e];
  }
  double f[8];
  su3_project(u, gg, f);
#pragma unroll
  for (int a = 0; a < 8; ++a) p[i * 8 + a] -= eps * f[a];
}

// U <- exp(i eps P) U for every link, P = sum_a p^a T_a.
__global__ void __launch_bounds__(256) k_link_update(int64_t nlinks, const double* __restrict__ p,
                                                     double eps, c64* __restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlinks) return;
  double pa[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) pa[a] = p[i * 8 + a];
  c64 E[9], u[9], r[9];
  su3_exp(pa, eps, E);
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[i * 9 + e];
  m3_mul(E, u, r);
#pragma unroll
  for (int e = 0; e < 9; ++e) U[i * 9 + e] = r[e];
}

// Per-block partial sums of v[i]^2 over n doubles (grid-stride).
__global__ void __launch_bounds__(256) k_sumsq_partial(const double* __restrict__ v, int64_t n,
                                                       double* __restrict__ partials) {
  __shared__ double sh[16];
  double s[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s[0] += v[i] * v[i];
  block_sum<1>(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// out = sum of nblk partials in a fixed order (one block).
__global__ void __launch_bounds__(256) k_sum_final(const double* __restrict__ partials, int nblk,
                                                   double* __restrict__ out) {
  __shared__ double sh[16];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v[0] += partials[i];
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) *out = v[0];
}

// ------------------------------------------------------------------ host

hipError_t launch_plaquette_sum(const Geo& g, const void* U, double* partials, int nblk,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_plaq_partial, dim3(nblk), dim3(256), 0, s, g, (const c64*)U, partials);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partials, nblk, out);
  return hipGetLastError();
}

hipError_t launch_gauge_grad(const Geo& g, const void* U, double beta, void* G, int accumulate,
                             hipStream_t s) {
  const size_t n = 8 * (size_t)g.hv;
  hipLaunchKernelGGL(k_gauge_grad, dim3(grid_for(n, 256)), dim3(256), 0, s, g, (const c64*)U,
                     beta, (c64*)G, accumulate);
  return hipGetLastError();
}

hipError_t launch_mom_update(const Geo& g, const void* U, const void* G, double eps, double* p,
                             hipStream_t s) {
  const int64_t n = 8 * (int64_t)g.hv;
  hipLaunchKernelGGL(k_mom_update, dim3(grid_for(n, 256)), dim3(256), 0, s, n, (const c64*)U,
                     (const c64*)G, eps, p);
  return hipGetLastError();
}

hipError_t launch_link_update(const Geo& g, const double* p, double eps, void* U, hipStream_t s) {
  const int64_t n = 8 * (int64_t)g.hv;
  hipLaunchKernelGGL(k_link_update, dim3(grid_for(n, 256)), dim3(256), 0, s, n, p, eps, (c64*)U);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* v, int64_t n, double* partials, int nblk, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nblk), dim3(256), 0, s, v, n, partials);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partials, nblk, out);
  return hipGetLastError();
}

}  // namespace qx
