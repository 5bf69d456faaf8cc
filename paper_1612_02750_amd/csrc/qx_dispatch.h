// Compile-time dispatch of the kernel templates from runtime parameters.
#pragma once

#include <hip/hip_runtime.h>

namespace qx {

inline unsigned grid_for(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

// recon: link storage, 18 or 12 reals per link, or 36 for the improved
// operator (one-hop and three-hop links of 18 reals each).
template <typename F>
hipError_t with_prec_recon(int prec, int recon, F&& f) {
  if (prec == 0 && recon == 18) return f.template operator()<double, 18>();
  if (prec == 0 && recon == 12) return f.template operator()<double, 12>();
  if (prec == 1 && recon == 18) return f.template operator()<float, 18>();
  if (prec == 1 && recon == 12) return f.template operator()<float, 12>();
  if (prec == 0 && recon == 36) return f.template operator()<double, 36>();
  if (prec == 1 && recon == 36) return f.template operator()<float, 36>();
  return hipErrorInvalidValue;
}

template <typename F>
hipError_t with_recon(int recon, F&& f) {
  if (recon == 18) return f.template operator()<18>();
  if (recon == 12) return f.template operator()<12>();
  if (recon == 36) return f.template operator()<36>();
  return hipErrorInvalidValue;
}

template <typename F>
hipError_t with_prec(int prec, F&& f) {
  if (prec == 0) return f.template operator()<double>();
  if (prec == 1) return f.template operator()<float>();
  return hipErrorInvalidValue;
}

// (sources per thread, wavefronts per site) pairs that are instantiated.  The
// wide pairs (six and twelve sources per thread) only where WIDE is set: the
// FP32 one-hop stencils of the standalone Dslash and of the launch-per-pass
// solver (wide_compiled); FP64 accumulators for that many sources do not fit
// the registers, and the other kernels serve few sources per system.
template <bool WIDE, typename F>
hipError_t with_nbt_lps(int nbt, int lps, F&& f) {
  if constexpr (WIDE) {
    switch (nbt * 16 + lps) {
      case 6 * 16 + 1: return f.template operator()<6, 1>();
      case 6 * 16 + 2: return f.template operator()<6, 2>();
      case 12 * 16 + 1: return f.template operator()<12, 1>();
      case 12 * 16 + 2: return f.template operator()<12, 2>();
      default: break;
    }
  }
  switch (nbt * 16 + lps) {
    case 1 * 16 + 1: return f.template operator()<1, 1>();
    case 1 * 16 + 2: return f.template operator()<1, 2>();
    case 1 * 16 + 4: return f.template operator()<1, 4>();
    case 1 * 16 + 8: return f.template operator()<1, 8>();
    case 2 * 16 + 1: return f.template operator()<2, 1>();
    case 2 * 16 + 2: return f.template operator()<2, 2>();
    case 2 * 16 + 4: return f.template operator()<2, 4>();
    case 4 * 16 + 1: return f.template operator()<4, 1>();
    case 4 * 16 + 2: return f.template operator()<4, 2>();
    default: return hipErrorInvalidValue;
  }
}

// Are the wide pairs compiled for links of this precision and storage?
inline bool wide_compiled(int prec, int recon) { return prec == 1 && recon != 36; }

// wide: the kernel has the wide pairs (wide_compiled, and the caller's path).
inline bool nbt_lps_instantiated(int nbt, int lps, bool wide) {
  return (nbt == 1 && (lps == 1 || lps == 2 || lps == 4 || lps == 8)) ||
         (nbt == 2 && (lps == 1 || lps == 2 || lps == 4)) || (nbt == 4 && (lps == 1 || lps == 2)) ||
         (wide && (nbt == 6 || nbt == 12) && (lps == 1 || lps == 2));
}

template <typename F>
hipError_t with_nbt(int nbt, F&& f) {
  if (nbt == 1) return f.template operator()<1>();
  if (nbt == 2) return f.template operator()<2>();
  if (nbt == 4) return f.template operator()<4>();
  return hipErrorInvalidValue;
}

// At most four sources per thread (the kernels without wide pairs: the FP64
// reliable-update stencils, the A epilogue of the standalone operator).
inline int narrow_nbt(int nbt) { return nbt > 4 ? 4 : nbt; }

}  // namespace qx
