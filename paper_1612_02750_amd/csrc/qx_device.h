// Device-side building blocks of the gfx950 kernels: even-odd geometry computed
// on the fly, link loads with optional 12-real reconstruction, the per-site
// staggered stencil for several sources, and deterministic wave/block
// reductions.
#pragma once

#include <hip/hip_fp16.h>

#include <type_traits>

#include "qx_internal.h"

// Dynamic LDS of the stencil kernels (16-byte aligned).
extern __shared__ double2 qx_lds[];

namespace qx {

// ------------------------------------------------------------ complex math

// c += a * b
template <typename R>
__device__ __forceinline__ void cfma(cplx<R>& c, const cplx<R>& a, const cplx<R>& b) {
  c.re = fma(a.re, b.re, c.re);
  c.re = fma(-a.im, b.im, c.re);
  c.im = fma(a.re, b.im, c.im);
  c.im = fma(a.im, b.re, c.im);
}

// c -= conj(a) * b
template <typename R>
__device__ __forceinline__ void cfms_conj(cplx<R>& c, const cplx<R>& a, const cplx<R>& b) {
  c.re = fma(-a.re, b.re, c.re);
  c.re = fma(-a.im, b.im, c.re);
  c.im = fma(-a.re, b.im, c.im);
  c.im = fma(a.im, b.re, c.im);
}

template <typename R>
__device__ __forceinline__ cplx<R> cmul(const cplx<R>& a, const cplx<R>& b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// ----------------------------------------------------------------- geometry

// Coordinates of the site (parity p, checkerboard index cb) and the
// checkerboard indices of its eight neighbours (which have parity 1 - p).
// In lexicographic order with x fastest and L0 even, cb = lex >> 1, so the
// x neighbours stay in the same row of L0/2 entries (shift 0 or +-1 by the
// parity of x) and the y, z, t neighbours are cb +- s1, s2, s3 with wrap.
struct Site {
  int x0, x1, x2, x3;
  int f0, f1, f2, f3;  // checkerboard index of x + mu
  int b0, b1, b2, b3;  // checkerboard index of x - mu
  int g0, g1, g2, g3;  // checkerboard index of x + 3 mu (improved operator only)
  int c0, c1, c2, c3;  // checkerboard index of x - 3 mu (improved operator only)
  // neighbour of hop h: h < 4 x + mu_h, h < 8 x - mu_{h-4}, h < 12 x + 3 mu_{h-8},
  // else x - 3 mu_{h-12}; h known at compile time
  template <int H>
  __host__ __device__ __forceinline__ int nbr() const {
    if constexpr (H == 0) return f0;
    else if constexpr (H == 1) return f1;
    else if constexpr (H == 2) return f2;
    else if constexpr (H == 3) return f3;
    else if constexpr (H == 4) return b0;
    else if constexpr (H == 5) return b1;
    else if constexpr (H == 6) return b2;
    else if constexpr (H == 7) return b3;
    else if constexpr (H == 8) return g0;
    else if constexpr (H == 9) return g1;
    else if constexpr (H == 10) return g2;
    else if constexpr (H == 11) return g3;
    else if constexpr (H == 12) return c0;
    else if constexpr (H == 13) return c1;
    else if constexpr (H == 14) return c2;
    else return c3;
  }
  __host__ __device__ __forceinline__ int fwd(int mu) const {
    return mu == 0 ? f0 : mu == 1 ? f1 : mu == 2 ? f2 : f3;
  }
  __host__ __device__ __forceinline__ int bwd(int mu) const {
    return mu == 0 ? b0 : mu == 1 ? b1 : mu == 2 ? b2 : b3;
  }
};

__host__ __device__ __forceinline__ void site_geometry(const Geo& g, int p, int cb, Site& s) {
  const int r = cb / g.Lh;
  const int x0h = cb - r * g.Lh;
  const int r2 = r / g.L1;
  const int x1 = r - r2 * g.L1;
  const int x3 = r2 / g.L2;
  const int x2 = r2 - x3 * g.L2;
  const int x0 = 2 * x0h + ((p + x1 + x2 + x3) & 1);
  s.x0 = x0;
  s.x1 = x1;
  s.x2 = x2;
  s.x3 = x3;
  const int row = r * g.Lh;
  const int x0p = (x0 + 1 == g.L0) ? 0 : x0 + 1;
  const int x0m = (x0 == 0) ? g.L0 - 1 : x0 - 1;
  s.f0 = row + (x0p >> 1);
  s.b0 = row + (x0m >> 1);
  s.f1 = (x1 + 1 == g.L1) ? cb - (g.L1 - 1) * g.s1 : cb + g.s1;
  s.b1 = (x1 == 0) ? cb + (g.L1 - 1) * g.s1 : cb - g.s1;
  s.f2 = (x2 + 1 == g.L2) ? cb - (g.L2 - 1) * g.s2 : cb + g.s2;
  s.b2 = (x2 == 0) ? cb + (g.L2 - 1) * g.s2 : cb - g.s2;
  s.f3 = (x3 + 1 == g.L3) ? cb - (g.L3 - 1) * g.s3 : cb + g.s3;
  s.b3 = (x3 == 0) ? cb + (g.L3 - 1) * g.s3 : cb - g.s3;
}

// The x +- 3 mu neighbours of a site (the Naik hops), with periodic wrap on
// any even extent (on an extent of 2 or 4 they land on x -+ mu or x +- mu).
__host__ __device__ __forceinline__ void three_hop_geometry(const Geo& g, int cb, Site& s) {
  const int row = cb - (s.x0 >> 1);
  s.g0 = row + (((s.x0 + 3) % g.L0) >> 1);
  s.c0 = row + (((s.x0 - 3) % g.L0 + g.L0) % g.L0 >> 1);
  s.g1 = cb + ((s.x1 + 3) % g.L1 - s.x1) * g.s1;
  s.c1 = cb + (((s.x1 - 3) % g.L1 + g.L1) % g.L1 - s.x1) * g.s1;
  s.g2 = cb + ((s.x2 + 3) % g.L2 - s.x2) * g.s2;
  s.c2 = cb + (((s.x2 - 3) % g.L2 + g.L2) % g.L2 - s.x2) * g.s2;
  s.g3 = cb + ((s.x3 + 3) % g.L3 - s.x3) * g.s3;
  s.c3 = cb + (((s.x3 - 3) % g.L3 + g.L3) % g.L3 - s.x3) * g.s3;
}

// Staggered phase eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}).
__host__ __device__ __forceinline__ int eta_sign(int mu, int x0, int x1, int x2) {
  int e = 0;
  if (mu >= 1) e += x0;
  if (mu >= 2) e += x1;
  if (mu >= 3) e += x2;
  return (e & 1) ? -1 : 1;
}

// eta_mu(x) times the boundary sign of the link U_mu(x): the factor folded
// into the packed links.
__host__ __device__ __forceinline__ int link_sign(const Geo& g, int mu, int x0, int x1, int x2, int x3) {
  const int s = eta_sign(mu, x0, x1, x2);
  return (mu == 3 && g.anti_t && x3 == g.L3 - 1) ? -s : s;
}

// Block index in the order that gives each XCD a contiguous range of tiles.
// Workgroups are dealt round-robin to the eight XCDs (blockIdx % 8), each with
// its own L2; with this remapping XCD k works on the k-th eighth of the
// checkerboard range, so the t and z neighbours of its sites mostly live in
// the same L2.
// xcd_block(b, G) is that remapping for dispatch index b of a G-block grid
// (a bijection of [0, G)).
__host__ __device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G >> 3, r = G & 7;
  const int x = b & 7, j = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

__device__ __forceinline__ int logical_block(int xcd_order) {
  const int b = blockIdx.x;
  if (!xcd_order) return b;
  return xcd_block(b, gridDim.x);
}

// Largest divisor of L that is at most cap.
__host__ __device__ __forceinline__ int divisor_upto(int L, int cap) {
  int d = cap < L ? cap : L;
  while (d > 1 && L % d) --d;
  return d;
}

// Checkerboard block (64 sites) visited at position bl of a lattice's block
// range.  Orders 0 and 1 visit blocks in checkerboard order.  Orders 2 and 3
// walk the (z, t) planes in tiles of tz x tt planes (2 x 8 and 4 x 4, cut to
// divisors of L2 and L3), z fastest inside a tile: the t neighbours of a site
// are then visited a few planes apart instead of a whole t-slice apart, so
// the colour vectors of many sources stay in an XCD's L2 between their eight
// uses.  The tiling needs whole blocks per (z, t) plane (Lh * L1 a multiple
// of 64) and falls back to checkerboard order otherwise.  A bijection of
// [0, hv / 64) onto itself.
//
// Orders 4 and 5 give each of the eight XCDs a slab of the lattice and walk it
// plane by plane, so that the blocks an XCD runs at the same time work on
// neighbouring (z, t) planes and the colour vectors those planes share stay in
// its L2: order 4 cuts z into eight slabs and walks t (slowest), then z, then
// the blocks of a (z, t) plane; order 5 cuts t and walks z.  With the
// XCD-contiguous dispatch (logical_block) slab k is the range XCD k runs.  They
// need whole blocks per (z, t) plane and the cut extent divisible by 8, and
// fall back to checkerboard order otherwise.  Stencil kernels under orders 4
// and 5 also store their outputs non-temporally (st_cplx).
__host__ __device__ __forceinline__ int tile_block(int bl, const Geo& g, int order) {
  if (order >= 4) {
    const int cut = order == 4 ? g.L2 : g.L3;
    if ((g.s2 & 63) || (cut & 7)) return bl;
    const int P = g.s2 >> 6, w = cut >> 3;
    const int per = (g.hv >> 6) >> 3;  // blocks of one slab
    const int k = bl / per, j = bl - k * per;
    const int a = j / (w * P), b = k * w + (j / P) % w;
    const int z = order == 4 ? b : a, t = order == 4 ? a : b;
    return (z + g.L2 * t) * P + j % P;
  }
  if (order < 2 || (g.s2 & 63)) return bl;
  const int P = g.s2 >> 6;  // blocks per (z, t) plane
  const int tz = divisor_upto(g.L2, order == 2 ? 2 : 4);
  const int tt = divisor_upto(g.L3, order == 2 ? 8 : 4);
  const int k = bl % P;
  int r = bl / P;
  const int zi = r % tz;
  r /= tz;
  const int ti = r % tt;
  r /= tt;
  const int nz = g.L2 / tz;
  const int z = (r % nz) * tz + zi, t = (r / nz) * tt + ti;
  return (z + g.L2 * t) * P + k;
}

// ------------------------------------------------------------------- links

// Element idx of an array whose base is the same across the wavefront.  The
// byte offset is formed in 32 bits (arrays here hold fewer than 2^28
// elements), so the load takes the scalar-base + 32-bit-lane-offset form and
// costs one VGPR of address instead of a 64-bit pointer per element.  NT: a
// non-temporal load, which streams past the caches.
// The access goes through a global-address-space pointer: a generic pointer
// would make it a flat access, which has no scalar-base form and takes a
// 64-bit address per lane.  Every array read or written through these
// helpers is in device memory.
#define QX_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const QX_GLOBAL T* as_global(const void* p) {
  return (const QX_GLOBAL T*)p;
}
// Element idx of a T array in device memory, the byte offset formed in 32
// bits (scalar base + 32-bit lane offset addressing).
template <typename T>
__device__ __forceinline__ const QX_GLOBAL T* global_elem(const void* base, unsigned idx) {
  return (const QX_GLOBAL T*)((const QX_GLOBAL char*)base + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ QX_GLOBAL T* as_global_w(void* p) {
  return (QX_GLOBAL T*)p;
}

template <bool NT, typename R>
__device__ __forceinline__ cplx<R> ld_cplx(const cplx<R>* __restrict__ base, unsigned idx) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  const QX_GLOBAL v2* q = global_elem<v2>(base, idx);
  v2 t;
  if constexpr (NT)
    t = __builtin_nontemporal_load(q);
  else
    t = *q;
  return {t.x, t.y};
}

// Element idx of an array of complex numbers stored as S, returned in the
// compute type R (FP16 storage widens to FP32).
template <bool NT, typename R, typename S>
__device__ __forceinline__ cplx<R> ld_cplx_as(const cplx<S>* __restrict__ base, unsigned idx) {
  if constexpr (std::is_same_v<S, __half>) {
    const QX_GLOBAL unsigned* p = global_elem<unsigned>(base, idx);
    unsigned w;
    if constexpr (NT)
      w = __builtin_nontemporal_load(p);
    else
      w = *p;
    __half2 h;
    __builtin_memcpy(&h, &w, sizeof w);
    const float2 f = __half22float2(h);
    return {(R)f.x, (R)f.y};
  } else {
    return ld_cplx<NT>(base, idx);
  }
}

// Wave index of the calling thread, as a scalar.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Packed links: one region per (parity, mu) of E elements (e = 3 * row +
// column; E = 9 for 18 reals, 6 for 12 reals: rows 0 and 1) for each of the
// hv links, E * C * hv bytes for C-byte complex numbers.  Inside a region the
// elements are grouped in chunks of W = 16 / C consecutive elements (FP64 1,
// FP32 2, FP16 4); chunk J occupies bytes [16 J hv, 16 (J + 1) hv) (or less for
// a last, partial chunk) as [cb][elements of the chunk], so that a link is read
// with 16-byte loads in every precision.  FP64 keeps the plain [e][cb] order.
template <typename LS, int E>
__host__ __device__ constexpr size_t link_elem_offset(int e, size_t hv, size_t cb) {
  constexpr int C = (int)sizeof(cplx<LS>), K = 16, W = K / C;
  const int J = e / W, n = (E - J * W) < W ? (E - J * W) : W;
  return (size_t)J * K * hv + cb * (size_t)(n * C) + (size_t)(e % W) * C;
}

// NW 32-bit words at base + off (off formed in 32 bits, as in ld_cplx).
template <int NW, bool NT>
__device__ __forceinline__ void ld_words(const char* __restrict__ base, unsigned off,
                                         unsigned (&w)[NW]) {
  if constexpr (NW == 1) {
    const QX_GLOBAL unsigned* q = as_global<unsigned>(base + off);
    if constexpr (NT)
      w[0] = __builtin_nontemporal_load(q);
    else
      w[0] = *q;
  } else {
    typedef unsigned vw __attribute__((ext_vector_type(NW)));
    const QX_GLOBAL vw* q = as_global<vw>(base + off);
    vw t;
    if constexpr (NT)
      t = __builtin_nontemporal_load(q);
    else
      t = *q;
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = t[i];
  }
}

// The complex number stored as LS in words w[0 .. sizeof(cplx<LS>) / 4), as R.
template <typename R, typename LS>
__device__ __forceinline__ cplx<R> cplx_from_words(const unsigned* w) {
  if constexpr (std::is_same_v<LS, __half>) {
    __half2 h;
    __builtin_memcpy(&h, w, sizeof h);
    const float2 f = __half22float2(h);
    return {(R)f.x, (R)f.y};
  } else {
    cplx<LS> v;
    __builtin_memcpy(&v, w, sizeof v);
    return {(R)v.re, (R)v.im};
  }
}

// Elements of chunks J, J + 1, ... of one link (layout above).
template <typename R, typename LS, bool NT, int E, int J>
__device__ __forceinline__ void load_link_chunks(cplx<R> (&u)[9], const char* __restrict__ region,
                                                 unsigned idx, size_t hv) {
  constexpr int C = (int)sizeof(cplx<LS>), K = 16, W = K / C;
  if constexpr (J * W < E) {
    constexpr int N = (E - J * W) < W ? (E - J * W) : W;
    unsigned w[N * C / 4];
    ld_words<N * C / 4, NT>(region + (size_t)J * K * hv, idx * (unsigned)(N * C), w);
#pragma unroll
    for (int n = 0; n < N; ++n) u[J * W + n] = cplx_from_words<R, LS>(w + n * (C / 4));
    load_link_chunks<R, LS, NT, E, J + 1>(u, region, idx, hv);
  }
}

// Fused multiply-add in the type of its operands.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a b - c d for complex a, b, c, d, every step an explicit multiply or fused
// multiply-add, so that no kernel's contraction of products and sums changes
// the rounding (the same link gives the same bits in every kernel).
template <typename R>
__device__ __forceinline__ cplx<R> cmul_sub(const cplx<R>& a, const cplx<R>& b, const cplx<R>& c,
                                            const cplx<R>& d) {
  R re = a.re * b.re;
  re = fmadd(-a.im, b.im, re);
  re = fmadd(-c.re, d.re, re);
  re = fmadd(c.im, d.im, re);
  R im = a.re * b.im;
  im = fmadd(a.im, b.re, im);
  im = fmadd(-c.re, d.im, im);
  im = fmadd(-c.im, d.re, im);
  return {re, im};
}

// Row 2 of a 12-real link from rows 0 and 1: for W = s U with U in SU(3) and
// s = +-1, row2(W) = s * conj(row0(W) x row1(W)).
template <typename R>
__device__ __forceinline__ void reconstruct_row2(cplx<R> (&u)[9], int sign) {
  const R s = (R)sign;
  const cplx<R> c0 = cmul_sub(u[1], u[5], u[2], u[4]);
  const cplx<R> c1 = cmul_sub(u[2], u[3], u[0], u[5]);
  const cplx<R> c2 = cmul_sub(u[0], u[4], u[1], u[3]);
  u[6] = {s * c0.re, -s * c0.im};
  u[7] = {s * c1.re, -s * c1.im};
  u[8] = {s * c2.re, -s * c2.im};
}

// Link idx of the region that starts at base (element 0 of direction mu of one
// parity).  Links are read once per half-Dslash: when they cannot stay in the
// Infinity Cache anyway they are loaded non-temporally (NT), so that the
// caches keep the colour vectors, each read by eight neighbouring sites.
// LS: the storage type of the links (R, or FP16 widened to R = float).
template <typename R, int RECON, bool NT, typename LS>
__device__ __forceinline__ void load_link(cplx<R> (&u)[9], const cplx<LS>* __restrict__ base,
                                          unsigned idx, size_t hv, int sign) {
  constexpr int E = RECON == 12 ? 6 : 9;
  if constexpr (sizeof(cplx<LS>) == 16) {
    // one element per chunk: the plain [e][cb] order
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = ld_cplx<NT>(base + e * hv, idx);
  } else {
    load_link_chunks<R, LS, NT, E, 0>(u, reinterpret_cast<const char*>(base), idx, hv);
  }
  if constexpr (RECON == 12) reconstruct_row2(u, sign);
}

// ---------------------------------------------------------------- stencil
//
// The eight hops of an output site x are h = 0..3 (forward, mu = h) and
// h = 4..7 (backward, mu = h - 4):
//   forward  mu: + W_mu(x)        in(x + mu)
//   backward mu: - W_mu(x - mu)^dag in(x - mu)
// with W = eta * bc * U the packed links, so the full sum is 2 D in.  A
// stencil kernel may split the hops of a site over LPS wavefronts (wave part
// dp takes the hops h with h % LPS == dp) and the sources over groups of NBT;
// every link a wavefront loads is applied to all of its active sources.

// Loader of the input vectors of a stencil: in_j(site, colour) for the
// sources j of the calling thread, from one packed field.
//
// Every loader serves the NBT source slots of a thread: slots past the last
// source it may read (jmax, uniform) read that source again, so that a
// stencil can load every slot of a hop unconditionally.
template <typename R>
struct FieldIn {
  const cplx<R>* __restrict__ p;  // first source of the thread
  size_t ss, hv;                  // source stride (3 hv), colour stride (hv)
  int jmax;                       // last readable slot
  __device__ __forceinline__ cplx<R> operator()(int j, int c, int site) const {
    const int jj = j < jmax ? j : jmax;
    return ld_cplx<false>(p + jj * ss + c * hv, (unsigned)site);
  }
};

// Colour vectors of FP32/FP64 sources as FieldIn, for a wavefront that covers
// the 64 consecutive sites [cb0, cb0 + 64) of a tile: the x and y neighbours
// that fall inside the tile are taken from the lane that loaded that index
// (ds_bpermute) instead of being loaded again.  Every lane first loads the
// colour vectors at its own index of the input parity (`own`, stencil_hops):
// one of a site's two x neighbours has that index and the other lies in the
// same row, and the y neighbours of all but the tile's first or last row are
// other lanes' own indices.  Lanes whose neighbour is outside the tile (a
// row split by the tile boundary, the first and last rows' y hops, the y
// wrap-around) load it.  The values are the same bits as FieldIn's.
template <typename R>
struct FieldInXY {
  const cplx<R>* __restrict__ p;  // first source of the thread
  size_t ss, hv;
  int jmax;  // last readable slot
  int cb0;   // first site of the wavefront's tile
  __device__ __forceinline__ cplx<R> operator()(int j, int c, int site) const {
    const int jj = j < jmax ? j : jmax;
    return ld_cplx<false>(p + jj * ss + c * hv, (unsigned)site);
  }
};
template <typename In>
struct is_xy_input : std::false_type {};
template <typename R>
struct is_xy_input<FieldInXY<R>> : std::true_type {};

// The lane's own-index colour vectors of every slot (for FieldInXY).
template <typename R, int NBT>
struct OwnVals {
  cplx<R> v[NBT][3];
  bool ok;  // loaded: the wavefront holds both x or both y hops
};

__device__ __forceinline__ float lane_shfl(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double lane_shfl(double v, int src) { return __shfl(v, src, 64); }

// FP16 colour vectors: per source [hv] records of 16 bytes, one per site:
// the three colours as half-precision complex numbers (12 bytes) and the
// site's FP32 scale; element = half * scale.  A site is one 16-byte load.
typedef unsigned qx_u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ cplx<float> h2_scaled(unsigned w, float sc) {
  __half2 h;
  __builtin_memcpy(&h, &w, sizeof h);
  const float2 f = __half22float2(h);
  return {f.x * sc, f.y * sc};
}

struct FieldInH {
  const char* __restrict__ p;  // first source of the thread
  size_t hv;
  int jmax;  // last readable slot
  __device__ __forceinline__ cplx<float> operator()(int j, int c, int site) const {
    const int jj = j < jmax ? j : jmax;
    // the three colours of a site read the same record: one load after CSE
    const qx_u32x4 r = *global_elem<qx_u32x4>(p + (size_t)jj * 16 * hv, (unsigned)site);
    return h2_scaled(c == 0 ? r.x : c == 1 ? r.y : r.z, __uint_as_float(r.w));
  }
};

// *p = v, non-temporally when nt (outputs the next pass reads from far away).
template <typename R>
__device__ __forceinline__ void st_cplx(cplx<R>* p, const cplx<R>& v, bool nt) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  v2 t;
  t.x = v.re;
  t.y = v.im;
  QX_GLOBAL v2* q = as_global_w<v2>(p);
  if (nt)
    __builtin_nontemporal_store(t, q);
  else
    *q = t;
}

// Store the colour vector v of site cb into an FP16 source (layout of
// FieldInH): scale = the largest |re| or |im| of v, pairs = v / scale.
__device__ __forceinline__ void st_field_h(char* __restrict__ src, int cb,
                                           const cplx<float> (&v)[3]) {
  float m = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
  const float inv = m > 0.0f ? 1.0f / m : 0.0f;
  qx_u32x4 r;
  unsigned w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const __half2 h = __floats2half2_rn(v[c].re * inv, v[c].im * inv);
    __builtin_memcpy(&w[c], &h, sizeof w[c]);
  }
  r.x = w[0];
  r.y = w[1];
  r.z = w[2];
  r.w = __float_as_uint(m);
  reinterpret_cast<qx_u32x4*>(src)[cb] = r;
}

// ------------------------------------------------- links shared through LDS
//
// When a block's wavefronts serve different source groups of the same 64
// sites (one wavefront per group and site), each would load every link of
// the tile itself: the same bytes through the vector memory pipeline once per
// group.  Instead the wavefronts share the loads: wavefront w of G loads the
// links of the hops h with h % G == w into LDS, the block meets at one
// barrier, and every wavefront reads all eight hops' links from LDS.  Chunk J
// of the link of hop h for lane l sits at ll[(h * NC + J) * 64 + l], 16 bytes
// (a partial last chunk in its first words), in the storage format of the
// link regions (link_elem_offset), so the values are the same bits as
// load_link's.
template <typename LS, int E>
constexpr int link_chunks() {
  return (int)((E * sizeof(cplx<LS>) + 15) / 16);
}

// LDS bytes of a tile's staged one-hop links (eight hops, 64 lanes), or 0
// where they are not staged (three-hop links, or more than 64 KB).
template <int RECON, typename LS>
constexpr size_t kLinkLdsBytes =
    RECON == 36 || 8 * link_chunks<LS, RECON == 12 ? 6 : 9>() * 64 * 16 > 65536
        ? 0
        : (size_t)8 * link_chunks<LS, RECON == 12 ? 6 : 9>() * 64 * 16;

template <typename LS, int E, bool NT, int J>
__device__ __forceinline__ void stage_link_chunks(qx_u32x4* __restrict__ ll, const char* region,
                                                  unsigned idx, size_t hv) {
  constexpr int C = (int)sizeof(cplx<LS>), K = 16, W = K / C;
  if constexpr (J * W < E) {
    constexpr int N = (E - J * W) < W ? (E - J * W) : W;
    unsigned w[N * C / 4];
    ld_words<N * C / 4, NT>(region + (size_t)J * K * hv, idx * (unsigned)(N * C), w);
    qx_u32x4 t = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < N * C / 4; ++i) t[i] = w[i];
    ll[J * 64] = t;
    stage_link_chunks<LS, E, NT, J + 1>(ll, region, idx, hv);
  }
}

// The links of hop H of the calling lane's output site into LDS (layout above).
template <int H, int RECON, bool NT, typename LS>
__device__ __forceinline__ void stage_hop_link(const Geo& g, const cplx<LS>* __restrict__ lf,
                                               const cplx<LS>* __restrict__ lb, int cb,
                                               const Site& s, qx_u32x4* ll, int lane) {
  constexpr int E = RECON == 12 ? 6 : 9, NC = link_chunks<LS, E>();
  constexpr int mu = H & 3;
  constexpr bool fwd = (H & 4) == 0;
  const cplx<LS>* base = (fwd ? lf : lb) + (size_t)mu * E * (size_t)g.hv;
  stage_link_chunks<LS, E, NT, 0>(ll + H * NC * 64 + lane, reinterpret_cast<const char*>(base),
                                  (unsigned)(fwd ? cb : s.template nbr<H>()), (size_t)g.hv);
}

// The eight hops' links of output parity pout for the tile, shared by the G
// wavefronts of the block (w: the caller's wavefront).  Every lane takes
// part (a lane past the lattice passes a clamped site); the caller then
// synchronises the block before any wavefront reads ll.
template <int RECON, typename LS>
__device__ __forceinline__ void stage_links(const Geo& g, const cplx<LS>* __restrict__ links,
                                            int pout, int cb, const Site& s, int w, int G,
                                            qx_u32x4* ll, int lane) {
  static_assert(RECON != 36, "one-hop links only");
  constexpr int E = RECON == 12 ? 6 : 9;
  const size_t hv = (size_t)g.hv;
  const cplx<LS>* lf = links + (size_t)pout * 4 * E * hv;
  const cplx<LS>* lb = links + (size_t)(1 - pout) * 4 * E * hv;
  unsigned mine = 0;  // the hops h = w, w + G, ... of this wavefront
  for (int h = w; h < 8; h += G) mine |= 1u << h;
#define QX_STAGE(H)                                                                  \
  if (mine >> (H) & 1u) {                                                            \
    if (g.stream_links)                                                              \
      stage_hop_link<H, RECON, true>(g, lf, lb, cb, s, ll, lane);                    \
    else                                                                             \
      stage_hop_link<H, RECON, false>(g, lf, lb, cb, s, ll, lane);                   \
  }
  QX_STAGE(0);
  QX_STAGE(1);
  QX_STAGE(2);
  QX_STAGE(3);
  QX_STAGE(4);
  QX_STAGE(5);
  QX_STAGE(6);
  QX_STAGE(7);
#undef QX_STAGE
}

// Link of hop H from LDS (stage_links), as load_link returns it.
template <typename R, int RECON, typename LS>
__device__ __forceinline__ void lds_link(cplx<R> (&u)[9], const qx_u32x4* __restrict__ ll, int H,
                                         int lane, int sign) {
  constexpr int E = RECON == 12 ? 6 : 9, NC = link_chunks<LS, E>();
  constexpr int C = (int)sizeof(cplx<LS>), W = 16 / C;
#pragma unroll
  for (int J = 0; J < NC; ++J) {
    const qx_u32x4 t = ll[(H * NC + J) * 64 + lane];
    const unsigned w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int n = 0; n < W; ++n)
      if (J * W + n < E) u[J * W + n] = cplx_from_words<R, LS>(w + n * (C / 4));
  }
  if constexpr (RECON == 12) reconstruct_row2(u, sign);
}

// acc[j] += hop H applied to in_j for every slot j < NBT.  The colour vectors
// of all slots are loaded before any product is formed and no slot is
// skipped: a per-slot test would put every slot's loads behind its own branch
// and let a wavefront have only one slot's loads in flight.  Callers mask
// unused slots when they store.
// Hops 8..15 (RECON == 36) are the three-hop terms, with the links at lf3/lb3.
// LL: the one-hop links come from LDS (stage_links) instead of memory.
template <int H, typename R, int RECON, int NBT, bool NT, bool LL, typename In, typename LS>
__device__ __forceinline__ void stencil_hop(const Geo& g, const cplx<LS>* __restrict__ lf,
                                            const cplx<LS>* __restrict__ lb,
                                            const cplx<LS>* __restrict__ lf3,
                                            const cplx<LS>* __restrict__ lb3, int cb, const Site& s,
                                            const In& in, const OwnVals<R, NBT>& own,
                                            const qx_u32x4* __restrict__ ll,
                                            cplx<R> (&acc)[NBT][3]) {
  constexpr int E = RECON == 12 ? 6 : 9;
  constexpr int mu = H & 3;
  constexpr bool fwd = (H & 4) == 0;
  constexpr bool three = H >= 8;
  const size_t hv = (size_t)g.hv;
  int sign = 1;
  if constexpr (RECON == 12) {
    // Forward link U_mu(x); backward link U_mu(x - mu), which has the same
    // eta (eta_mu does not depend on x_mu) and the antiperiodic sign when
    // (x - mu)_3 = L3 - 1, i.e. x3 = 0 for mu = t.
    const int e = eta_sign(mu, s.x0, s.x1, s.x2);
    const bool flip = mu == 3 && g.anti_t && (fwd ? s.x3 == g.L3 - 1 : s.x3 == 0);
    sign = flip ? -e : e;
  }
  const int nb = s.template nbr<H>();
  cplx<R> v[NBT][3];
  const auto load_all = [&]() {
#pragma unroll
    for (int j = 0; j < NBT; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) v[j][c] = in(j, c, nb);
  };
  if constexpr (is_xy_input<In>::value && !three && mu < 2) {
    if (own.ok) {
      // in-tile neighbours from the lane that holds them, the rest loaded
      const unsigned o = (unsigned)(nb - in.cb0);
      const bool inside = o < 64u;
      const int src = inside ? (int)o : (int)(threadIdx.x & 63);
#pragma unroll
      for (int j = 0; j < NBT; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          v[j][c] = {lane_shfl(own.v[j][c].re, src), lane_shfl(own.v[j][c].im, src)};
      if (!inside) load_all();
    } else {
      load_all();
    }
  } else {
    load_all();
  }
  cplx<R> u[9];
  if constexpr (LL && !three) {
    lds_link<R, RECON, LS>(u, ll, H, (int)(threadIdx.x & 63), sign);
  } else {
    const cplx<LS>* base = three ? (fwd ? lf3 : lb3) : (fwd ? lf : lb);
    load_link<R, RECON, NT>(u, base + (size_t)mu * E * hv, (unsigned)(fwd ? cb : nb), hv, sign);
  }
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    if constexpr (fwd) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cfma(acc[j][a], u[3 * a + 0], v[j][0]);
        cfma(acc[j][a], u[3 * a + 1], v[j][1]);
        cfma(acc[j][a], u[3 * a + 2], v[j][2]);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cfms_conj(acc[j][a], u[0 + a], v[j][0]);
        cfms_conj(acc[j][a], u[3 + a], v[j][1]);
        cfms_conj(acc[j][a], u[6 + a], v[j][2]);
      }
    }
  }
}

// acc[j] += the hops of part dp (of LPS) applied to in_j, j < NBT.
// Each hop is its own instantiation, guarded by a wavefront-uniform test.
// PAIRED (the solver's passes): the hops of a direction are taken one after
// the other (x+, x-, y+, y-, z+, z-, t+, t-), so that a wavefront with
// FieldInXY input uses the own-index values it loaded for both x (or both y)
// hops; every engine's stencils sum their hops in this order, so the engines
// round alike.  Otherwise (the standalone operator) the order is x+, y+, z+,
// t+, x-, ..., which the compiler schedules with fewer registers there.
template <typename R, int RECON, int NBT, int LPS, bool NT, bool PAIRED, bool LL = false,
          typename In, typename LS>
__device__ __forceinline__ void stencil_hops(const Geo& g, const cplx<LS>* __restrict__ lf,
                                             const cplx<LS>* __restrict__ lb,
                                             const cplx<LS>* __restrict__ lf3,
                                             const cplx<LS>* __restrict__ lb3, int cb, const Site& s,
                                             int dp, const In& in, cplx<R> (&acc)[NBT][3],
                                             const qx_u32x4* __restrict__ ll = nullptr) {
  OwnVals<R, NBT> own;
  own.ok = false;
  if constexpr (is_xy_input<In>::value) {
    // hop h goes to part h % LPS: with LPS <= 4 parts 0 and 1 hold both x
    // hops and both y hops (with LPS 8 each part holds one hop: no gain)
    own.ok = LPS == 1 || (LPS <= 4 && dp < 2);
    if (own.ok) {
      const int ci = cb < (int)g.hv ? cb : (int)g.hv - 1;
#pragma unroll
      for (int j = 0; j < NBT; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) own.v[j][c] = in(j, c, ci);
    }
  }
#define QX_HOP(H)                               \
  if (LPS == 1 || (H) % LPS == dp)              \
  stencil_hop<H, R, RECON, NBT, NT, LL>(g, lf, lb, lf3, lb3, cb, s, in, own, ll, acc)
  if constexpr (PAIRED) {
    QX_HOP(0);
    QX_HOP(4);
    QX_HOP(1);
    QX_HOP(5);
    QX_HOP(2);
    QX_HOP(6);
    QX_HOP(3);
    QX_HOP(7);
  } else {
    QX_HOP(0);
    QX_HOP(1);
    QX_HOP(2);
    QX_HOP(3);
    QX_HOP(4);
    QX_HOP(5);
    QX_HOP(6);
    QX_HOP(7);
  }
  if constexpr (RECON == 36) {
    QX_HOP(8);
    QX_HOP(9);
    QX_HOP(10);
    QX_HOP(11);
    QX_HOP(12);
    QX_HOP(13);
    QX_HOP(14);
    QX_HOP(15);
  }
#undef QX_HOP
}

// The same for the links of output parity pout; whether the links stream past
// the caches is decided once per launch (Geo::stream_links).  The caller runs
// it only for sites of the lattice (every slot of the thread is computed).
template <typename R, int RECON, int NBT, int LPS, bool PAIRED = true, typename In, typename LS>
__device__ __forceinline__ void stencil_part(const Geo& g, const cplx<LS>* __restrict__ links,
                                             int pout, int cb, const Site& s, int dp, const In& in,
                                             cplx<R> (&acc)[NBT][3]) {
  constexpr int E = RECON == 12 ? 6 : 9;
  const size_t hv = (size_t)g.hv;
  // link regions [parity][mu] (link_elem_offset); the improved operator's three-hop links follow
  // the one-hop ones in the same layout
  const cplx<LS>* lf = links + (size_t)pout * 4 * E * hv;
  const cplx<LS>* lb = links + (size_t)(1 - pout) * 4 * E * hv;
  const cplx<LS>* lf3 = links + (size_t)(2 + pout) * 4 * E * hv;
  const cplx<LS>* lb3 = links + (size_t)(3 - pout) * 4 * E * hv;
  if constexpr (RECON == 36) {
    Site s3 = s;
    three_hop_geometry(g, cb, s3);
    if (g.stream_links)
      stencil_hops<R, RECON, NBT, LPS, true, PAIRED>(g, lf, lb, lf3, lb3, cb, s3, dp, in, acc);
    else
      stencil_hops<R, RECON, NBT, LPS, false, PAIRED>(g, lf, lb, lf3, lb3, cb, s3, dp, in, acc);
  } else {
    if (g.stream_links)
      stencil_hops<R, RECON, NBT, LPS, true, PAIRED>(g, lf, lb, lf3, lb3, cb, s, dp, in, acc);
    else
      stencil_hops<R, RECON, NBT, LPS, false, PAIRED>(g, lf, lb, lf3, lb3, cb, s, dp, in, acc);
  }
}

// stencil_part (one wavefront per site: all eight hops) with the links read
// from LDS, where stage_links put them before the block's barrier.
template <typename R, int RECON, int NBT, bool PAIRED = true, typename In, typename LS>
__device__ __forceinline__ void stencil_part_ll(const Geo& g, const cplx<LS>* __restrict__ links,
                                                int cb, const Site& s, const In& in,
                                                const qx_u32x4* __restrict__ ll,
                                                cplx<R> (&acc)[NBT][3]) {
  static_assert(RECON != 36, "one-hop links only");
  const cplx<LS>* none = nullptr;
  (void)links;
  stencil_hops<R, RECON, NBT, 1, false, PAIRED, true>(g, none, none, none, none, cb, s, 0, in, acc,
                                                      ll);
}

template <typename R, int NBT>
__device__ __forceinline__ void zero_acc(cplx<R> (&acc)[NBT][3]) {
#pragma unroll
  for (int j = 0; j < NBT; ++j)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[j][a] = {(R)0, (R)0};
}

// Visit every reduced item of the block's stencil: f(j, c, v) is called for
// item (source slot j, colour c) with the sum v over the LPS hop parts, in the
// wavefront that owns it (part (3 j + c) % LPS).  Wave w of the block is
// (part dp = w % LPS, group grp = w / LPS).  Without hop splitting f sees
// acc[j][c] directly; with it the parts meet in LDS, one slot j at a time, so
// red holds G * LPS * 3 * 64 complex numbers.  All threads of the block must
// call it (it synchronises when LPS > 1).
template <typename R, int NBT, int LPS, typename F>
__device__ __forceinline__ void for_each_item(const cplx<R> (&acc)[NBT][3], cplx<R>* red, int dp,
                                              int grp, int lane, F&& f) {
  if constexpr (LPS == 1) {
#pragma unroll
    for (int j = 0; j < NBT; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) f(j, c, acc[j][c]);
  } else {
    cplx<R>* mine = red + (size_t)(grp * LPS + dp) * 3 * 64;
    const cplx<R>* base = red + (size_t)grp * LPS * 3 * 64;
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (j > 0) __syncthreads();  // the previous slot has been read
#pragma unroll
      for (int c = 0; c < 3; ++c) mine[c * 64 + lane] = acc[j][c];
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if ((j * 3 + c) % LPS != dp) continue;
        cplx<R> t = {(R)0, (R)0};
#pragma unroll
        for (int q = 0; q < LPS; ++q) {
          const cplx<R> v = base[((size_t)q * 3 + c) * 64 + lane];
          t.re += v.re;
          t.im += v.im;
        }
        f(j, c, t);
      }
    }
  }
}

// As for_each_item, with a value ld(j, c) per item (an epilogue operand in
// device memory) loaded for all the thread's items before the first slot's
// barrier, so that the slots' loads overlap instead of each waiting behind
// the previous slot's barrier: f(j, c, v, loaded).
template <typename R, int NBT, int LPS, typename L, typename F>
__device__ __forceinline__ void for_each_item_ld(const cplx<R> (&acc)[NBT][3], cplx<R>* red,
                                                 int dp, int grp, int lane, L&& ld, F&& f) {
  using T = decltype(ld(0, 0));
  T pre[NBT][3];
#pragma unroll
  for (int j = 0; j < NBT; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (LPS == 1 || (j * 3 + c) % LPS == dp) pre[j][c] = ld(j, c);
  for_each_item<R, NBT, LPS>(acc, red, dp, grp, lane,
                             [&](int j, int c, cplx<R> v) { f(j, c, v, pre[j][c]); });
}

// As for_each_item, but all three colours of a source slot meet in one
// wavefront (part j % LPS), for outputs that need the whole colour vector of
// a site at once (FP16 storage with a per-site scale): f(j, v[3]).
template <typename R, int NBT, int LPS, typename F>
__device__ __forceinline__ void for_each_slot(const cplx<R> (&acc)[NBT][3], cplx<R>* red, int dp,
                                              int grp, int lane, F&& f) {
  if constexpr (LPS == 1) {
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      const cplx<R> v[3] = {acc[j][0], acc[j][1], acc[j][2]};
      f(j, v);
    }
  } else {
    cplx<R>* mine = red + (size_t)(grp * LPS + dp) * 3 * 64;
    const cplx<R>* base = red + (size_t)grp * LPS * 3 * 64;
#pragma unroll
    for (int j = 0; j < NBT; ++j) {
      if (j > 0) __syncthreads();
#pragma unroll
      for (int c = 0; c < 3; ++c) mine[c * 64 + lane] = acc[j][c];
      __syncthreads();
      if (j % LPS != dp) continue;
      cplx<R> v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cplx<R> t = {(R)0, (R)0};
#pragma unroll
        for (int q = 0; q < LPS; ++q) {
          const cplx<R> w = base[((size_t)q * 3 + c) * 64 + lane];
          t.re += w.re;
          t.im += w.im;
        }
        v[c] = t;
      }
      f(j, v);
    }
  }
}

// Threads per stencil block allowed by the register budget (see max_waves).
template <typename R, int NBT>
constexpr int kMaxThreads = sizeof(R) * NBT > 8 ? 512 : 1024;

// Is the stencil output of this block order stored non-temporally?
__host__ __device__ __forceinline__ bool order_nt(int order) { return order >= 4; }

// ------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of v over the block for NB independent values, fixed order (wave
// butterflies, then waves in index order), result valid in thread 0.
// `sh` must hold NB * 16 doubles.
template <int NB>
__device__ __forceinline__ void block_sum(double (&v)[NB], double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double t = wave_sum(v[k]);
    if (lane == 0) sh[k * 16 + w] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      double t = 0;
      for (int i = 0; i < nw; ++i) t += sh[k * 16 + i];
      v[k] = t;
    }
  }
  __syncthreads();
}

// Per-source sums over a stencil block: thread (wave w, lane) holds v[j] for
// source grp * NBT + j of its group (grp = w / LPS).  The totals for the G*NBT
// sources of the block land in tot_sh[k], fixed summation order.  sh must hold
// 16 * NBT * 16 doubles.
template <int NBT>
__device__ __forceinline__ void group_sum(const double (&v)[NBT], int nwaves_per_group, int grp,
                                          int wig, int ngroups, double* sh, double* tot_sh) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < NBT; ++j) {
    const double t = wave_sum(v[j]);
    if (lane == 0) sh[(grp * NBT + j) * 16 + wig] = t;
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < ngroups * NBT) {
    double t = 0;
    for (int i = 0; i < nwaves_per_group; ++i) t += sh[k * 16 + i];
    tot_sh[k] = t;
  }
  __syncthreads();
}

}  // namespace qx
