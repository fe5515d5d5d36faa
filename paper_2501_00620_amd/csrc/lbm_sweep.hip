// lbm_sweep.hip -- the fused sweeps of one storage type (LBM_SWEEP_S = 0: FP64, 1: FP32, 2: FP16
// deviations, 3: BF16 deviations): their launch functions and kernel instantiations, declared in
// lbm_sweeps.hpp.  The build compiles this file once per storage type.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_fused_pc.hpp"
#include "lbm_sweeps.hpp"

#ifndef LBM_SWEEP_S
#error "lbm_sweep.hip is compiled with -DLBM_SWEEP_S=<storage type 0..3>"
#endif

namespace lbm {

template <int S>
int launch_fused(const typename Storage<S>::T *F, const typename Storage<S>::T *B, typename Storage<S>::T *Fo,
                 typename Storage<S>::T *Bo, const typename Storage<S>::C *Tf, typename Storage<S>::C Tconst,
                 const Geo &g, const StepConst<typename Storage<S>::C> &k, const Codec &cd, unsigned *flag,
                 bool gathered, int slots, hipStream_t stream, const typename Storage<S>::C *accel) {
    using TL = typename TileFor<S>::type;
    const FusedGeo fg = fused_geometry<S>(g, slots);
    const long long blocks = (long long)fg.tiles_x * fg.tiles_y * fg.nchunks;
    if (blocks > 2147483647LL) return -1;
    const dim3 grid((unsigned)blocks), block(TL::NT);
    const bool hask = k.K != 0;
    // one z plane: the instantiation with the in-plane gather and gradient (the serving kernel
    // sweeps such lattices with the same arithmetic)
    auto go = [&](auto G, auto H, auto T1) {
        if (accel || k.force_u)
            hipLaunchKernelGGL((k_fused<S, decltype(G)::value, decltype(H)::value, decltype(T1)::value, true>), grid,
                               block, 0, stream, F, B, Fo, Bo, Tf, Tconst, g, k, cd, flag, fg, accel);
        else
            hipLaunchKernelGGL((k_fused<S, decltype(G)::value, decltype(H)::value, decltype(T1)::value, false>), grid,
                               block, 0, stream, F, B, Fo, Bo, Tf, Tconst, g, k, cd, flag, fg, accel);
    };
    using tt = std::true_type;
    using ff = std::false_type;
    const bool thin1 = g.nz == 1;
    if (gathered) {
        if (hask) thin1 ? go(tt{}, tt{}, tt{}) : go(tt{}, tt{}, ff{});
        else thin1 ? go(tt{}, ff{}, tt{}) : go(tt{}, ff{}, ff{});
    } else {
        if (hask) thin1 ? go(ff{}, tt{}, tt{}) : go(ff{}, tt{}, ff{});
        else thin1 ? go(ff{}, ff{}, tt{}) : go(ff{}, ff{}, ff{});
    }
    return 0;
}

// Resident work-groups per CU of the producer/consumer sweep: one (its LDS).  With walls the
// chunks cover the interior planes 1 .. nz-2, and wsrc holds the source planes of planes 0 and
// nz-1 (NSRC planes of n values).
template <int S>
int launch_fused_pc(const typename Storage<S>::T *F, const typename Storage<S>::T *B, typename Storage<S>::T *Fo,
                    typename Storage<S>::T *Bo, const typename Storage<S>::C *Tf, typename Storage<S>::C Tconst,
                    const Geo &g, const StepConst<typename Storage<S>::C> &k, const Codec &cd, unsigned *flag, int slots,
                    hipStream_t stream, const typename Storage<S>::C *accel, const typename Storage<S>::C *wsrc) {
    if (g.walls && (g.nz < 3 || !wsrc)) return -1;
    Geo gi = g;
    if (g.walls) gi.nz = g.nz - 2;
    const FusedGeo fg = fused_geometry_t<PcTile>(gi, slots);
    const long long blocks = (long long)fg.tiles_x * fg.tiles_y * fg.nchunks;
    if (blocks > 2147483647LL) return -1;
    const dim3 grid((unsigned)blocks), block(PC_THREADS);
    auto go = [&](auto H, auto FO, auto M) {
        if (g.walls)
            hipLaunchKernelGGL((k_fused_pc<S, decltype(H)::value, decltype(FO)::value, decltype(M)::value, true>), grid,
                               block, 0, stream, F, B, Fo, Bo, Tf, Tconst, g, k, cd, flag, fg, accel, wsrc);
        else
            hipLaunchKernelGGL((k_fused_pc<S, decltype(H)::value, decltype(FO)::value, decltype(M)::value, false>), grid,
                               block, 0, stream, F, B, Fo, Bo, Tf, Tconst, g, k, cd, flag, fg, accel, wsrc);
    };
    using tt = std::true_type;
    using ff = std::false_type;
    auto with_mrt = [&](auto H, auto FO) { k.ghost != 0 ? go(H, FO, tt{}) : go(H, FO, ff{}); };
    auto with_force = [&](auto H) { accel || k.force_u ? with_mrt(H, tt{}) : with_mrt(H, ff{}); };
    k.K != 0 ? with_force(tt{}) : with_force(ff{});
    return 0;
}

template <int S> hipError_t sweep_occupancy(int *per_cu, int *per_cu_pc) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fused<S, false, false, false, false>,
                                                                TileFor<S>::type::NT, 0);
    if constexpr (S != 0) {
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu_pc, k_fused_pc<S, false, false, false, false>,
                                                             PC_THREADS, 0);
    }
    return e;
}

constexpr int SW = LBM_SWEEP_S;
template int launch_fused<SW>(const Storage<SW>::T *, const Storage<SW>::T *, Storage<SW>::T *, Storage<SW>::T *,
                              const Storage<SW>::C *, Storage<SW>::C, const Geo &, const StepConst<Storage<SW>::C> &,
                              const Codec &, unsigned *, bool, int, hipStream_t, const Storage<SW>::C *);
#if LBM_SWEEP_S != 0
template int launch_fused_pc<SW>(const Storage<SW>::T *, const Storage<SW>::T *, Storage<SW>::T *, Storage<SW>::T *,
                                 const Storage<SW>::C *, Storage<SW>::C, const Geo &, const StepConst<Storage<SW>::C> &,
                                 const Codec &, unsigned *, int, hipStream_t, const Storage<SW>::C *,
                                 const Storage<SW>::C *);
#endif
template hipError_t sweep_occupancy<SW>(int *, int *);

}  // namespace lbm
