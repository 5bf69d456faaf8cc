// Host launch sequences of the CG engine for one (inner precision, link
// storage) pair; LS is the storage type of the inner links.  Defined in
// qx_engine_kernels.h, instantiated per pair in qx_engine_inst.hip,
// dispatched from qx_engine.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "qx_internal.h"
#include "qx_launch.h"

namespace qx {

template <typename R>
hipError_t init_impl(const EngineCfg& c, int zero_xhi, hipStream_t s);
template <typename R, int RECON, typename LS>
hipError_t iteration_impl(const EngineCfg& c, int parity, hipStream_t s);
template <typename Rlo, int RECON>
hipError_t reliable_update_impl(const EngineCfg& c, bool last, hipStream_t s);
template <typename R, int RECON, typename LS>
int persistent_per_cu_impl(const EngineCfg& c);
template <typename R, int RECON, typename LS>
hipError_t persistent_impl(const EngineCfg& c, int iters, GridSync* gs, int grid,
                           long long timeout, hipStream_t s);

}  // namespace qx
