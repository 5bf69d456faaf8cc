// Instantiates the CG engine's kernels and launch sequences for one (inner
// precision, link storage) pair, given at compile time as QX_R (float or
// double) and QX_RECON (12, 18 or 36); with QX_LINKS16 the inner links are
// binary16 (QX_R float), and only the iteration sequences are instantiated
// (the initialisation and the reliable update read no inner links).  The
// build compiles this file once per combination so they compile in parallel.
#include "qx_engine_kernels.h"

#if !defined(QX_R) || !defined(QX_RECON)
#error "compile with -DQX_R=<float|double> -DQX_RECON=<12|18|36> [-DQX_LINKS16]"
#endif

namespace qx {

#ifdef QX_LINKS16
template hipError_t iteration_impl<float, QX_RECON, __half>(const EngineCfg&, int, hipStream_t);
template int persistent_per_cu_impl<float, QX_RECON, __half>(const EngineCfg&);
template hipError_t persistent_impl<float, QX_RECON, __half>(const EngineCfg&, int, GridSync*, int,
                                                              long long, hipStream_t);
#else
template hipError_t iteration_impl<QX_R, QX_RECON, QX_R>(const EngineCfg&, int, hipStream_t);
template int persistent_per_cu_impl<QX_R, QX_RECON, QX_R>(const EngineCfg&);
template hipError_t persistent_impl<QX_R, QX_RECON, QX_R>(const EngineCfg&, int, GridSync*, int,
                                                           long long, hipStream_t);
template hipError_t reliable_update_impl<QX_R, QX_RECON>(const EngineCfg&, bool, hipStream_t);
#if QX_RECON == 18
template hipError_t init_impl<QX_R>(const EngineCfg&, int, hipStream_t);
#endif
#endif

}  // namespace qx
