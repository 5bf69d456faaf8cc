// FP64 SU(3) helpers of the force and molecular-dynamics kernels: 3x3 complex
// products, the projection of a link gradient onto the eight generators, and
// the exponential of i eps P for a traceless Hermitian P.
#pragma once

#include "qx_internal.h"

namespace qx {

typedef cplx<double> c64;

// c = a b
__device__ __forceinline__ void m3_mul(const c64* a, const c64* b, c64* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c64 s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s.re += a[3 * i + k].re * b[3 * k + j].re - a[3 * i + k].im * b[3 * k + j].im;
        s.im += a[3 * i + k].re * b[3 * k + j].im + a[3 * i + k].im * b[3 * k + j].re;
      }
      c[3 * i + j] = s;
    }
}

// c = a b^dag
__device__ __forceinline__ void m3_mul_nd(const c64* a, const c64* b, c64* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c64 s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // a[i][k] * conj(b[j][k])
        s.re += a[3 * i + k].re * b[3 * j + k].re + a[3 * i + k].im * b[3 * j + k].im;
        s.im += a[3 * i + k].im * b[3 * j + k].re - a[3 * i + k].re * b[3 * j + k].im;
      }
      c[3 * i + j] = s;
    }
}

// c = a^dag b
__device__ __forceinline__ void m3_mul_dn(const c64* a, const c64* b, c64* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      c64 s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // conj(a[k][i]) * b[k][j]
        s.re += a[3 * k + i].re * b[3 * k + j].re + a[3 * k + i].im * b[3 * k + j].im;
        s.im += a[3 * k + i].re * b[3 * k + j].im - a[3 * k + i].im * b[3 * k + j].re;
      }
      c[3 * i + j] = s;
    }
}

// F^a = Re[i tr(T_a Q)] = -1/2 Im[sum_ij (lambda_a)_ij Q_ji], Q = U G^dag: the
// derivative of S(exp(i w T_a) U) at w = 0 for the link gradient
// G = dS/dRe U + i dS/dIm U, written out for the eight Gell-Mann matrices.
__device__ __forceinline__ void su3_project(const c64* u, const c64* g, double* f) {
  c64 Q[9];
  m3_mul_nd(u, g, Q);
  f[0] = -0.5 * (Q[1].im + Q[3].im);
  f[1] = -0.5 * (Q[1].re - Q[3].re);
  f[2] = -0.5 * (Q[0].im - Q[4].im);
  f[3] = -0.5 * (Q[2].im + Q[6].im);
  f[4] = -0.5 * (Q[2].re - Q[6].re);
  f[5] = -0.5 * (Q[5].im + Q[7].im);
  f[6] = -0.5 * (Q[5].re - Q[7].re);
  f[7] = -0.5 * (Q[0].im + Q[4].im - 2.0 * Q[8].im) * 0.57735026918962576451;
}

// E = exp(i eps P), P = sum_a p^a lambda_a / 2, by scaling and squaring: the
// argument is halved until its Frobenius norm is at most 1/2, the exponential
// of that summed to the 16th power by Horner's rule (truncation below 1e-19
// relative), then squared back.
__device__ __forceinline__ void su3_exp(const double* p, double eps, c64* E) {
  const double r3 = 0.57735026918962576451;  // 1 / sqrt(3)
  // H = P (Hermitian); X = i eps H
  const double h00 = 0.5 * (p[2] + r3 * p[7]), h11 = 0.5 * (-p[2] + r3 * p[7]);
  const double h22 = -r3 * p[7];
  const c64 h01 = {0.5 * p[0], -0.5 * p[1]}, h02 = {0.5 * p[3], -0.5 * p[4]};
  const c64 h12 = {0.5 * p[5], -0.5 * p[6]};
  c64 X[9];
  // i eps h: (a + i b) -> (-eps b + i eps a)
  X[0] = {0.0, eps * h00};
  X[4] = {0.0, eps * h11};
  X[8] = {0.0, eps * h22};
  X[1] = {-eps * h01.im, eps * h01.re};
  X[2] = {-eps * h02.im, eps * h02.re};
  X[5] = {-eps * h12.im, eps * h12.re};
  X[3] = {eps * h01.im, eps * h01.re};  // i eps conj(h01)
  X[6] = {eps * h02.im, eps * h02.re};
  X[7] = {eps * h12.im, eps * h12.re};
  double nrm = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) nrm += X[e].re * X[e].re + X[e].im * X[e].im;
  nrm = sqrt(nrm);
  int s = 0;
  while (nrm > 0.5 && s < 40) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
#pragma unroll
  for (int e = 0; e < 9; ++e) X[e] = {X[e].re * sc, X[e].im * sc};
  // Horner: E = 1 + X (1 + X/2 (1 + X/3 (... (1 + X/16))))
  c64 T[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) E[e] = {(e % 4 == 0) ? 1.0 : 0.0, 0.0};
  for (int k = 16; k >= 1; --k) {
    m3_mul(X, E, T);
    const double inv = 1.0 / k;
#pragma unroll
    for (int e = 0; e < 9; ++e) E[e] = {T[e].re * inv + ((e % 4 == 0) ? 1.0 : 0.0), T[e].im * inv};
  }
  for (int i = 0; i < s; ++i) {
    m3_mul(E, E, T);
#pragma unroll
    for (int e = 0; e < 9; ++e) E[e] = T[e];
  }
}

}  // namespace qx
