// Host build of the library's device geometry (qx_device.h): the even-odd
// coordinates, the one- and three-hop neighbour indices, the folded link signs
// (eta times the boundary sign), the (z, t)-tiled block order and the
// XCD-contiguous block remapping, evaluated on the CPU so that tests without a
// GPU can compare them with brute-force enumeration.  The functions called here
// are the __host__ __device__ ones the kernels call; nothing is re-implemented.
#include <stdint.h>

#include <vector>

#include "qx_device.h"

using qx::Geo;
using qx::Site;

namespace {

Geo geo_of(const int32_t L[4], int anti) {
  Geo g{};
  g.L0 = L[0];
  g.L1 = L[1];
  g.L2 = L[2];
  g.L3 = L[3];
  g.Lh = L[0] / 2;
  g.hv = (int)((int64_t)L[0] * L[1] * L[2] * L[3] / 2);
  g.s1 = g.Lh;
  g.s2 = g.Lh * L[1];
  g.s3 = g.Lh * L[1] * L[2];
  g.anti_t = anti;
  return g;
}

}  // namespace

extern "C" {

// For every site in even-odd order eo = p * V/2 + cb: its lexicographic index,
// the eo indices of x + mu (0..3), x - mu (4..7), x + 3 mu (8..11) and x - 3 mu
// (12..15), and the sign folded into the packed link U_mu(x) (4 per site).
int qxg_maps(const int32_t L[4], int anti, int32_t* lex_of_eo, int32_t* nbr, int32_t* sign) {
  const Geo g = geo_of(L, anti);
  for (int p = 0; p < 2; ++p)
    for (int cb = 0; cb < g.hv; ++cb) {
      const int64_t eo = (int64_t)p * g.hv + cb;
      Site s;
      qx::site_geometry(g, p, cb, s);
      qx::three_hop_geometry(g, cb, s);
      lex_of_eo[eo] = 2 * cb + (s.x0 & 1);
      const int other = (1 - p) * g.hv;
      for (int mu = 0; mu < 4; ++mu) {
        nbr[eo * 16 + mu] = other + s.fwd(mu);
        nbr[eo * 16 + 4 + mu] = other + s.bwd(mu);
      }
      nbr[eo * 16 + 8] = other + s.g0;
      nbr[eo * 16 + 9] = other + s.g1;
      nbr[eo * 16 + 10] = other + s.g2;
      nbr[eo * 16 + 11] = other + s.g3;
      nbr[eo * 16 + 12] = other + s.c0;
      nbr[eo * 16 + 13] = other + s.c1;
      nbr[eo * 16 + 14] = other + s.c2;
      nbr[eo * 16 + 15] = other + s.c3;
      for (int mu = 0; mu < 4; ++mu) sign[eo * 4 + mu] = qx::link_sign(g, mu, s.x0, s.x1, s.x2, s.x3);
    }
  return 0;
}

// tile_block(bl) for every block bl of the half lattice (hv / 64 blocks).
int qxg_tile_perm(const int32_t L[4], int order, int32_t* out) {
  const Geo g = geo_of(L, 0);
  const int nb = g.hv / 64;
  for (int bl = 0; bl < nb; ++bl) out[bl] = qx::tile_block(bl, g, order);
  return nb;
}

// xcd_block(b, G) for b in [0, G).
int qxg_xcd_perm(int G, int32_t* out) {
  for (int b = 0; b < G; ++b) out[b] = qx::xcd_block(b, G);
  return G;
}

// Exhaustive bijection check of tile_block: every L2, L3 even in [2, maxL],
// P = (L0 / 2) L1 / 64 blocks per (z, t) plane in [1, maxP], orders 0 to 5.
// Returns the number of (geometry, order) pairs that fail.
int64_t qxg_tile_bijection_failures(int maxL, int maxP) {
  int64_t bad = 0;
  std::vector<int> seen;
  for (int P = 1; P <= maxP; ++P)
    for (int L2 = 2; L2 <= maxL; L2 += 2)
      for (int L3 = 2; L3 <= maxL; L3 += 2) {
        // L0 = 2 * 64 P / L1 with L1 = 2: s2 = Lh * L1 = 64 P
        const int32_t L[4] = {64 * P, 2, L2, L3};
        const Geo g = geo_of(L, 0);
        const int nb = g.hv / 64;
        for (int order = 0; order < 6; ++order) {
          seen.assign(nb, 0);
          bool ok = true;
          for (int bl = 0; bl < nb && ok; ++bl) {
            const int t = qx::tile_block(bl, g, order);
            if (t < 0 || t >= nb || seen[t]++) ok = false;
          }
          if (!ok) ++bad;
        }
      }
  return bad;
}

}  // extern "C"
