// CG engine dispatch: picks the (inner precision, link storage) instantiation
// of the launch sequences (qx_engine_kernels.h, instantiated per pair in
// qx_engine_inst.hip).  The engine itself is described there.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "qx_dispatch.h"
#include "qx_engine_impl.h"
#include "qx_launch.h"

namespace qx {

// The iteration's instantiation: inner arithmetic and vectors R, inner links
// LS (R, or binary16 under FP32 vectors).
template <typename F>
hipError_t with_iteration_types(const EngineCfg& c, F&& f) {
  if (!c.links16)
    return with_prec_recon(c.prec_lo, c.recon_lo, [&]<typename R, int RECON>() {
      return f.template operator()<R, RECON, R>();
    });
  if (c.prec_lo != 1) return hipErrorInvalidValue;
  return with_recon(c.recon_lo,
                    [&]<int RECON>() { return f.template operator()<float, RECON, __half>(); });
}

bool engine_supported(const EngineCfg& c) {
  const bool ok_lo = (c.prec_lo == 0 || c.prec_lo == 1) && (!c.links16 || c.prec_lo == 1) &&
                     (c.recon_lo == 18 || c.recon_lo == 12 || c.recon_lo == 36);
  const bool ok_hi = c.recon_hi == 18 || c.recon_hi == 12 || c.recon_hi == 36;
  // the FP64 reliable-update stencils take narrow_nbt sources per thread, one wavefront each
  const LaunchShape rsh{narrow_nbt(c.shape.nbt), 1, 0};
  const bool wide = wide_compiled(c.prec_lo, c.recon_lo) && !c.links16;
  const bool ok_shape = nbt_lps_instantiated(c.shape.nbt, c.shape.lps, wide) &&
                        shape_ok(c.shape, c.nsrc_max, cplx_bytes(c.prec_lo)) &&
                        shape_groups(rsh, c.nsrc_max) <= max_waves(rsh.nbt, 16);
  return ok_lo && ok_hi && ok_shape && c.nsrc_max >= 1 && c.nsrc_max <= 64 && c.nsys >= 1 &&
         c.nblk_total >= 1 && c.nvblk_total >= 1;
}

hipError_t engine_init(const EngineCfg& c, int zero_xhi, hipStream_t s) {
  return with_prec(c.prec_lo, [&]<typename R>() { return init_impl<R>(c, zero_xhi, s); });
}

hipError_t engine_iteration(const EngineCfg& c, int parity, hipStream_t s) {
  return with_iteration_types(c, [&]<typename R, int RECON, typename LS>() {
    return iteration_impl<R, RECON, LS>(c, parity, s);
  });
}

hipError_t engine_reliable_update(const EngineCfg& c, bool last, hipStream_t s) {
  return with_prec_recon(c.prec_lo, c.recon_hi, [&]<typename R, int RECON>() {
    return reliable_update_impl<R, RECON>(c, last, s);
  });
}

namespace {
int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n = 0;
  }
  return n;
}
}  // namespace

int engine_persistent_capacity(const EngineCfg& c) {
  int per_cu = 0;
  hipError_t e = with_iteration_types(c, [&]<typename R, int RECON, typename LS>() {
    per_cu = persistent_per_cu_impl<R, RECON, LS>(c);
    return hipSuccess;
  });
  if (e != hipSuccess) return 0;
  return per_cu * cu_count();
}

hipError_t engine_persistent(const EngineCfg& c, int iters, GridSync* gs, int grid,
                             hipStream_t s) {
  // barrier waits give up after 2 s of the constant-rate device clock
  static long long timeout = 0;
  if (!timeout) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    timeout = 2000LL * khz;
  }
  return with_iteration_types(c, [&]<typename R, int RECON, typename LS>() {
    return persistent_impl<R, RECON, LS>(c, iters, gs, grid, timeout, s);
  });
}

}  // namespace qx
