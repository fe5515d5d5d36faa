// lbm_sweeps.hpp -- host entry points of the fused sweeps (k_fused, k_fused_pc).
//
// Their kernels have many instantiations (storage x gathered x body force x one plane x K), so
// they are compiled apart from the rest of the library: lbm_sweep.hip is built once per storage
// type, with -DLBM_SWEEP_S=<0..3>, and the build compiles those units in parallel.  Callers see
// only these declarations.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_kernels.hpp"

namespace lbm {

// One step of the single-role fused sweep (k_fused) from F, B into Fo, Bo.  gathered: B holds
// bbar itself (after set_fields / set_state) instead of the scattered bbar*.  slots: work-groups
// resident at once.  accel: body-force field (3 planes of the compute type) or null.  Returns 0,
// or -1 when the grid does not fit.
template <int S>
int launch_fused(const typename Storage<S>::T *F, const typename Storage<S>::T *B, typename Storage<S>::T *Fo,
                 typename Storage<S>::T *Bo, const typename Storage<S>::C *Tf, typename Storage<S>::C Tconst,
                 const Geo &g, const StepConst<typename Storage<S>::C> &k, const Codec &cd, unsigned *flag,
                 bool gathered, int slots, hipStream_t stream, const typename Storage<S>::C *accel = nullptr);

// One step of the producer/consumer sweep (k_fused_pc; S = 1, 2, 3 and B scattered), as above.
// With walls (g.walls) it steps the interior planes 1 .. nz-2 only and needs wsrc, the source
// planes (NSRC planes of n values) holding at least planes 0 and nz-1; returns -1 without it.
template <int S>
int launch_fused_pc(const typename Storage<S>::T *F, const typename Storage<S>::T *B, typename Storage<S>::T *Fo,
                    typename Storage<S>::T *Bo, const typename Storage<S>::C *Tf, typename Storage<S>::C Tconst,
                    const Geo &g, const StepConst<typename Storage<S>::C> &k, const Codec &cd, unsigned *flag, int slots,
                    hipStream_t stream, const typename Storage<S>::C *accel = nullptr,
                    const typename Storage<S>::C *wsrc = nullptr);

// Work-groups of each sweep that one CU holds at once (the runtime's occupancy of the steady-state
// kernel of storage S); per_cu_pc is left alone for S = 0.
template <int S> hipError_t sweep_occupancy(int *per_cu, int *per_cu_pc);

}  // namespace lbm
