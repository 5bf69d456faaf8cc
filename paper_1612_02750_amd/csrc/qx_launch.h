// Host-callable launchers of the gfx950 kernels (internal to libqx.so).
#pragma once

#include "qx_internal.h"

namespace qx {

struct LaunchShape {
  int block = 256;  // threads per block
  int xcd = 1;      // XCD-contiguous block order
};

// Bytes of one complex number of the given precision (QX_PREC_F64 = 0 -> 16, F32 -> 8).
inline size_t cplx_bytes(int prec) { return prec == 0 ? 16 : 8; }

hipError_t launch_pack_gauge(const Geo& g, const void* U, int prec, int recon, void* packed,
                             unsigned long long* err_bits, hipStream_t s);
hipError_t launch_pack_field(const Geo& g, int nrhs, int prec, const void* canon, void* packed,
                             hipStream_t s);
hipError_t launch_unpack_field(const Geo& g, int nrhs, int prec, const void* packed, void* canon,
                               hipStream_t s);
hipError_t launch_index_maps(const Geo& g, int32_t* lex_of_eo, int32_t* nbr_eo, hipStream_t s);

// out = scale * (2D) in, from parity 1 - pout to pout, nsrc sources (any count).
hipError_t launch_dslash(const Geo& g, int prec, int recon, const void* links, int pout,
                         const void* in, void* out, int nsrc, double scale, LaunchShape sh,
                         hipStream_t s);
// out_k = m2[k] in_k - D_eo D_oe in_k (tmp: odd scratch).
hipError_t launch_apply_A(const Geo& g, int prec, int recon, const void* links, int nrhs,
                          const double* m2, const void* in, void* out, void* tmp, LaunchShape sh,
                          hipStream_t s);

// ------------------------------------------------------------------ engine

// One solver launch configuration: the systems (device table), their source
// states, the inner precision and link storage, the FP64 link storage, the
// number of sources each thread handles (nb), and the launch shape.
struct EngineCfg {
  int prec_lo = 0, recon_lo = 18, recon_hi = 18, nb = 1;
  LaunchShape shape;
  int nsys = 0, nblk_total = 0, nsrc_total = 0;
  const SysDesc* d_sys = nullptr;
  SrcState* d_st = nullptr;
};

bool engine_supported(const EngineCfg& c);
hipError_t engine_init(const EngineCfg& c, int zero_xhi, hipStream_t s);
hipError_t engine_iteration(const EngineCfg& c, hipStream_t s);
hipError_t engine_reliable_update(const EngineCfg& c, hipStream_t s);

// ------------------------------------------------------------------ force

hipError_t launch_force(const Geo& g, int nsrc, const void* x, const void* lam, const void* y,
                        const void* nu, void* G, hipStream_t s);
hipError_t launch_su3_force(const Geo& g, const void* U, const void* G, double* F, hipStream_t s);
// out = sum_i Re(conj(a_i) b_i) over n complex128 values (two deterministic passes).
hipError_t launch_redot(const void* a, const void* b, size_t n, double* partials, int nblk,
                        double* out, hipStream_t s);

// dst = src, bytes a multiple of 16.
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace qx
