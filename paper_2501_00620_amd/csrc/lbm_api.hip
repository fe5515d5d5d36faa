// lbm_api.hip -- host side of the C ABI declared in include/lbm.h.
//
// One lattice = device buffers of the kernels in lbm_kernels.hpp plus a HIP stream.  Every
// step of the method runs in those kernels; the host only validates arguments, chooses the
// codec scales from device reductions, and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>

#include "../../include/lbm.h"
#include "lbm_fused.hpp"
#include "lbm_fused_pc.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernels.hpp"
#include "lbm_proj.hpp"
#include "lbm_sweeps.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

namespace lbm {
int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}
}  // namespace lbm

namespace {

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(LBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t store_bytes(int storage) { return storage == LBM_F64 ? 8 : storage == LBM_F32 ? 4 : 2; }
size_t compute_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }

}  // namespace




namespace {

Geo geo(const lbm_lattice *h) { return Geo{h->p.nx, h->p.ny, h->p.nz, h->n, h->walls}; }

int blocks_for(int n) { return (n + BLOCK - 1) / BLOCK; }
int red_blocks(int n) {
    int b = blocks_for(n);
    return b < RED_MAX_BLOCKS ? b : RED_MAX_BLOCKS;
}

// Codec references: ref_i = w_i rho_ref, bbar_ref = (T_ref - 1/3) I; unit scales until chosen.
void codec_defaults(lbm_lattice *h) {
    const double w[Q] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                         1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                         1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    for (int i = 0; i < Q; i++) h->codec.ref[i] = w[i] * h->p.rho_ref;
    for (int c = 0; c < NB; c++) h->codec.ref[Q + c] = c < 3 ? h->p.T_ref - 1.0 / 3.0 : 0.0;
    for (int k = 0; k < NFIELD; k++) h->codec.scale[k] = h->codec.inv[k] = 1.0f;
}

// One power-of-two scale per stored array (the 19 populations; the 6 bbar components): the
// largest deviation in the array maps to at most HMAX/1024 (fp16), leaving 1024x headroom for
// growth before saturation.  The scale only moves binary16's 30-octave window: values stay
// normal (relative precision 2^-11) down to about 1e-6 of the array's initial largest
// deviation, and below that the absolute error is under 1e-9 of it, so per-field scales would
// buy no precision; one scale per array lets the sweep keep two constants in scalar registers
// instead of fifty.  A field that starts without deviation counts as a deviation of 1e-3 of its
// reference magnitude (1e-3 for bbar).  bfloat16 has the exponent range of binary32, so its
// codes hold the deviations themselves (unit scale).
void choose_scales(lbm_lattice *h, const double *absmax) {
    if (h->p.storage != LBM_F16DEV) {
        for (int k = 0; k < NFIELD; k++) h->codec.scale[k] = h->codec.inv[k] = 1.0f;
        return;
    }
    const double target = 65504.0 / 1024.0;
    double mg[2] = {0.0, 0.0};  // populations, bbar
    for (int k = 0; k < NFIELD; k++) {
        double floor_dev = k < Q ? 1e-3 * std::fabs(h->codec.ref[k]) : 1e-3;
        if (floor_dev <= 0) floor_dev = 1e-3;
        const double m = absmax[k] > floor_dev ? absmax[k] : floor_dev;
        double &g = mg[k < Q ? 0 : 1];
        g = m > g ? m : g;
    }
    for (int k = 0; k < NFIELD; k++) {
        const int e = (int)std::ceil(std::log2(mg[k < Q ? 0 : 1] / target));
        const double sc = std::ldexp(1.0, e);
        h->codec.scale[k] = (float)sc;
        h->codec.inv[k] = (float)(1.0 / sc);
    }
}

// FP16 scales of a projected lattice: each plane's initial deviation is bounded by the sum of its
// members' (class sums; transverse-weighted for G), the variance planes by their components'.
// Then the same power-of-two choice as choose_scales.  Fields: class sum c at c, its G at
// NC + c, variance plane k at Q + k.
template <int D> void choose_scales_proj(lbm_lattice *h, const double *absmax) {
    using PS = ProjSet<D>;
    const bool th = h->p.mode == LBM_THERMAL;
    double am[NFIELD], fl[NFIELD];
    for (int k = 0; k < NFIELD; k++) am[k] = 0.0, fl[k] = 1e-3;
    for (int i = 0; i < Q; i++) {
        const int c = PS::CLS[i];
        am[c] += absmax[i];
        if (th && et2<D>(i) > 0) am[PS::NC + c] += et2<D>(i) * absmax[i];
    }
    for (int c = 0; c < PS::NC; c++) {
        fl[c] = 1e-3 * class_w<D>(c) * h->p.rho_ref;
        if (c < PS::NG) fl[PS::NC + c] = 1e-3 * class_gw<D>(c) * h->p.rho_ref;
    }
    if constexpr (D == 2) {
        am[Q + 0] = absmax[Q + 0];
        am[Q + 1] = absmax[Q + 1];
        am[Q + 2] = absmax[Q + 3];
        am[Q + 3] = absmax[Q + 2];
    } else {
        am[Q + 0] = absmax[Q + 0];
        am[Q + 1] = absmax[Q + 1] + absmax[Q + 2];
    }
    const double target = 65504.0 / 1024.0;
    for (int k = 0; k < NFIELD; k++) {
        const double m = am[k] > fl[k] ? am[k] : fl[k];
        const double sc = std::ldexp(1.0, (int)std::ceil(std::log2(m / target)));
        h->codec.scale[k] = (float)sc;
        h->codec.inv[k] = (float)(1.0 / sc);
    }
}

template <typename Fn> int dispatch_storage(int storage, Fn &&fn) {
    switch (storage) {
    case LBM_F64: return fn(std::integral_constant<int, 0>{});
    case LBM_F32: return fn(std::integral_constant<int, 1>{});
    case LBM_F16DEV: return fn(std::integral_constant<int, 2>{});
    case LBM_BF16DEV: return fn(std::integral_constant<int, 3>{});
    }
    return fail(LBM_ERR_ARG, "unknown storage %d", storage);
}

// Projected lattices (lbm_set_projection): any storage, D = 2 or 1, energy-conserving or not.
template <typename Fn> int dispatch_proj(const lbm_lattice *h, Fn &&fn) {
    using D2 = std::integral_constant<int, 2>;
    using D1 = std::integral_constant<int, 1>;
    const bool th = h->p.mode == LBM_THERMAL;
    return dispatch_storage(h->p.storage, [&](auto SI) -> int {
        if (h->proj == 2)
            return th ? fn(SI, D2{}, std::true_type{}) : fn(SI, D2{}, std::false_type{});
        return th ? fn(SI, D1{}, std::true_type{}) : fn(SI, D1{}, std::false_type{});
    });
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBM_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
    return LBM_OK;
}

// Fold block partials into h->red_out[0..K) and copy to host.
template <bool MAX> int finish_reduction(lbm_lattice *h, int nblocks, int K, double *host) {
    hipLaunchKernelGGL(k_reduce_final<MAX>, dim3(1), dim3(BLOCK), 0, h->stream, h->partial, nblocks, K, h->red_out);
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(host, h->red_out, sizeof(double) * K, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int clear_flag(lbm_lattice *h) {
    HIP_TRY(hipMemsetAsync(h->flag, 0, sizeof(unsigned), h->stream));
    return LBM_OK;
}

int read_clear_flag(lbm_lattice *h, unsigned *val) {
    HIP_TRY(hipMemcpyAsync(val, h->flag, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (*val) HIP_TRY(hipMemsetAsync(h->flag, 0, sizeof(unsigned), h->stream));
    return LBM_OK;
}

// ---- one step ----------------------------------------------------------------------------------
// The two-pass step's source planes, allocated on its first use (the fused step keeps the
// sources in LDS, and the readout uses the idle population buffer).
int ensure_src(lbm_lattice *h) {
    if (h->src) return LBM_OK;
    const hipError_t e = hipMalloc(&h->src, compute_bytes(h->p.storage) * NSRC * (size_t)h->n);
    if (e != hipSuccess) {
        h->src = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, "source planes: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

// The two-pass step's launches on the current state: the predictor over planes [z0, z1) into
// the source planes, and the collision over planes [c0, c1) (both ends plane indices; the wall
// kernel on planes 0 and nz-1 when the lattice has walls).
template <int S> struct TwoPass {
    using T = typename Storage<S>::T;
    using C = typename Storage<S>::C;
    lbm_lattice *h;
    Geo g;
    StepConst<C> k;
    const T *F, *B;
    T *Fo, *Bo;
    C *src;
    explicit TwoPass(lbm_lattice *hh)
        : h(hh), g(geo(hh)), k(step_const<C>(hh)), F((const T *)hh->F[hh->cur]), B((const T *)hh->B[hh->cur]),
          Fo((T *)hh->F[1 - hh->cur]), Bo((T *)hh->B[1 - hh->cur]), src((C *)hh->src) {}
    int nxy() const { return h->p.nx * h->p.ny; }
    template <bool G> void predict(int z0, int z1) const {
        const int s0 = z0 * nxy(), count = (z1 - z0) * nxy();
        hipLaunchKernelGGL((k_predict<S, G>), dim3(blocks_for(count)), dim3(BLOCK), 0, h->stream, F, B, src,
                           (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, s0, count);
    }
    template <bool G, bool M, bool W> void collide(int z0, int z1) const {
        const int s0 = z0 * nxy(), count = (z1 - z0) * nxy();
        hipLaunchKernelGGL((k_collide<S, G, M, W>), dim3(blocks_for(count)), dim3(BLOCK), 0, h->stream, F, B, src, Fo,
                           Bo, (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, h->flag, (const C *)h->accel, s0,
                           count);
    }
    // The wall planes 0 and nz-1, stepped with the wall kernel, and the sources of the planes
    // next to them (which the split sweep's gradients of planes 1 and nz-2 read too).  For a
    // state whose bbar is held scattered: the split sweep's steps, never the first after
    // set_fields / set_state.
    template <bool M> void wall_planes() const {
        const int nz = h->p.nz;
        if (nz <= 6) {
            predict<false>(0, nz);
        } else {
            predict<false>(0, 3);
            predict<false>(nz - 3, nz);
        }
        collide<false, M, true>(0, 1);
        collide<false, M, true>(nz - 1, nz);
    }
};

template <int S> int step_two_pass(lbm_lattice *h) {
    if (int rc = ensure_src(h)) return rc;
    const TwoPass<S> tp(h);
    const int nz = h->p.nz;
    auto launch = [&](auto GI, auto MI) {
        constexpr bool G = decltype(GI)::value, M = decltype(MI)::value;
        tp.template predict<G>(0, nz);
        if (!h->walls) {
            tp.template collide<G, M, false>(0, nz);
        } else {
            // interior planes with the periodic kernel; the two wall planes with the wall kernel
            tp.template collide<G, M, false>(1, nz - 1);
            tp.template collide<G, M, true>(0, 1);
            tp.template collide<G, M, true>(nz - 1, nz);
        }
    };
    auto with_mrt = [&](auto GI) {
        if (h->tau_ghost > 0.0) launch(GI, std::true_type{}); else launch(GI, std::false_type{});
    };
    if (h->gathered) with_mrt(std::true_type{}); else with_mrt(std::false_type{});
    int rc = check_launch();
    if (rc) return rc;
    h->cur = 1 - h->cur;
    h->gathered = false;
    return LBM_OK;
}

// The producer/consumer sweep steps float and 16-bit lattices that march in z, once bbar is held
// scattered (the first step after the state was set gathers it from global memory in the
// single-role sweep, or two-pass with walls); lbm_set_kernel(2) keeps the single-role sweep
// throughout.
bool use_fused_pc(const lbm_lattice *h) {
    return (h->kernel == 0 || h->kernel == 3) && !h->gathered && fused_pc_supported(geo(h), h->p.storage);
}

template <int S> int step_fused(lbm_lattice *h) {
    using T = typename Storage<S>::T;
    using C = typename Storage<S>::C;
    const Geo g = geo(h);
    const StepConst<C> k = step_const<C>(h);
    int rc = 0;
    if constexpr (S != 0) {
        if (use_fused_pc(h)) {
            if (h->walls) {
                // the wall planes and their neighbours' sources first (two-pass kernels), then the
                // interior planes; each writes population slots the other does not
                if ((rc = ensure_src(h))) return rc;
                const TwoPass<S> tp(h);
                if (h->tau_ghost > 0.0) tp.template wall_planes<true>(); else tp.template wall_planes<false>();
                if ((rc = check_launch())) return rc;
            }
            rc = launch_fused_pc<S>((const T *)h->F[h->cur], (const T *)h->B[h->cur], (T *)h->F[1 - h->cur],
                                    (T *)h->B[1 - h->cur], (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, h->flag,
                                    h->slots_pc, h->stream, (const C *)h->accel, (const C *)h->src);
            if (rc) return fail(LBM_ERR_HIP, "fused launch failed");
            rc = check_launch();
            if (rc) return rc;
            h->cur = 1 - h->cur;
            return LBM_OK;
        }
    }
    rc = launch_fused<S>((const T *)h->F[h->cur], (const T *)h->B[h->cur], (T *)h->F[1 - h->cur],
                         (T *)h->B[1 - h->cur], (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, h->flag,
                         h->gathered, h->slots, h->stream, (const C *)h->accel);
    if (rc) return fail(LBM_ERR_HIP, "fused launch failed");
    rc = check_launch();
    if (rc) return rc;
    h->cur = 1 - h->cur;
    h->gathered = false;
    return LBM_OK;
}

// One step of a projected lattice: in-plane predictor sources, then gradient, collision and the
// push of the class sums.
int step_proj(lbm_lattice *h) {
    return dispatch_proj(h, [&](auto SI, auto DI, auto TI) -> int {
        constexpr int S = decltype(SI)::value, D = decltype(DI)::value;
        constexpr bool TH = decltype(TI)::value;
        using T = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const Geo g = geo(h);
        const StepConst<C> k = step_const<C>(h);
        const T *F = (const T *)h->F[h->cur];
        const T *B = (const T *)h->B[h->cur];
        const dim3 grid(blocks_for(h->n)), block(BLOCK);
        if (h->kernel != 1) {  // one launch per step (lbm_set_kernel(1) keeps the two-pass form)
            using TL = ProjTile<D>;
            const dim3 tiles((h->p.nx + TL::TX - 1) / TL::TX, (h->p.ny + TL::TY - 1) / TL::TY);
            T *Fo = (T *)h->F[1 - h->cur];
            T *Bo = (T *)h->B[1 - h->cur];
            if (h->gathered)
                hipLaunchKernelGGL((k_proj_fused<S, D, TH, true>), tiles, dim3(TL::NT), 0, h->stream, F, B, Fo, Bo,
                                   (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, h->flag);
            else
                hipLaunchKernelGGL((k_proj_fused<S, D, TH, false>), tiles, dim3(TL::NT), 0, h->stream, F, B, Fo, Bo,
                                   (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, h->flag);
        } else if (h->gathered) {
            hipLaunchKernelGGL((k_proj_predict<S, D, TH, true>), grid, block, 0, h->stream, F, B, (C *)h->src,
                               (const C *)h->Tf, (C)h->Tconst, g, k, h->codec);
            hipLaunchKernelGGL((k_proj_collide<S, D, TH, true>), grid, block, 0, h->stream, F, B, (const C *)h->src,
                               (T *)h->F[1 - h->cur], (T *)h->B[1 - h->cur], (const C *)h->Tf, (C)h->Tconst, g, k,
                               h->codec, h->flag);
        } else {
            hipLaunchKernelGGL((k_proj_predict<S, D, TH, false>), grid, block, 0, h->stream, F, B, (C *)h->src,
                               (const C *)h->Tf, (C)h->Tconst, g, k, h->codec);
            hipLaunchKernelGGL((k_proj_collide<S, D, TH, false>), grid, block, 0, h->stream, F, B, (const C *)h->src,
                               (T *)h->F[1 - h->cur], (T *)h->B[1 - h->cur], (const C *)h->Tf, (C)h->Tconst, g, k,
                               h->codec, h->flag);
        }
        int rc = check_launch();
        if (rc) return rc;
        h->cur = 1 - h->cur;
        h->gathered = false;
        return LBM_OK;
    });
}

// One step of the standard lattice Boltzmann comparator (Sec. I, Eq. 4): BGK and push.
template <int S> int step_std(lbm_lattice *h) {
    using T = typename Storage<S>::T;
    using C = typename Storage<S>::C;
    auto launch = [&](auto WI, int s0, int count) {
        hipLaunchKernelGGL((k_std<S, decltype(WI)::value>), dim3(blocks_for(count)), dim3(BLOCK), 0, h->stream,
                           (const T *)h->F[h->cur], (T *)h->F[1 - h->cur], (const C *)h->Tf, (C)h->Tconst, geo(h),
                           step_const<C>(h), h->codec, h->flag, (const C *)h->accel, s0, count);
    };
    if (!h->walls) {
        launch(std::false_type{}, 0, h->n);
    } else {  // interior planes with the periodic kernel, the two wall planes with the wall kernel
        const int nxy = h->p.nx * h->p.ny;
        launch(std::false_type{}, nxy, (h->p.nz - 2) * nxy);
        launch(std::true_type{}, 0, nxy);
        launch(std::true_type{}, (h->p.nz - 1) * nxy, nxy);
    }
    int rc = check_launch();
    if (rc) return rc;
    // bbar carries nothing in this model: both buffers hold its reference (zero deviation) since
    // set_fields
    h->cur = 1 - h->cur;
    h->gathered = false;
    return LBM_OK;
}

// Whether the next step is a fused one: the producer/consumer sweep when it takes the lattice
// (a ghost rate and walls included), else the single-role sweep, which relaxes with a single rate
// on a periodic lattice.
bool use_fused(const lbm_lattice *h) {
    if (h->kernel == 1) return false;
    if (use_fused_pc(h)) return true;
    return h->tau_ghost <= 0.0 && !h->walls && fused_supported(geo(h), h->p.storage);
}

}  // namespace

// ===============================================================================================
extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

int lbm_create(const lbm_params *p, void *hip_stream, lbm_handle *out) {
    if (!p || !out) return fail(LBM_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_ERR_ARG, "lattice size must be >= 1");
    const long long n = (long long)p->nx * p->ny * p->nz;
    if (n > 2147483647LL) return fail(LBM_ERR_ARG, "lattice has more than 2^31-1 sites");
    if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(LBM_ERR_ARG, "tau must be > 0");
    if (p->storage < 0 || p->storage > 3) return fail(LBM_ERR_ARG, "unknown storage %d", p->storage);
    if (p->mode != LBM_THERMAL && p->mode != LBM_ISO && p->mode != LBM_STANDARD)
        return fail(LBM_ERR_ARG, "unknown mode %d", p->mode);
    if (!(p->rho_ref > 0.0)) return fail(LBM_ERR_ARG, "rho_ref must be > 0");
    lbm_lattice *h = new (std::nothrow) lbm_lattice();
    if (!h) return fail(LBM_ERR_OOM, "host allocation failed");
    h->p = *p;
    h->n = (int)n;
    h->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(LBM_ERR_HIP, "hipGetDevice failed");
    }
    const size_t sb = store_bytes(p->storage);
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; b++) {
        e = hipMalloc(&h->F[b], sb * Q * (size_t)n);
        if (e == hipSuccess) e = hipMalloc(&h->B[b], sb * NB * (size_t)n);
    }
    // shapes beyond the fused sweep's range step with the two-pass kernel, which needs its
    // source planes (others allocate them if lbm_set_kernel asks for the two-pass kernel)
    if (e == hipSuccess && !fused_supported(geo(h), p->storage))
        e = hipMalloc(&h->src, compute_bytes(p->storage) * NSRC * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&h->partial, sizeof(double) * 2 * RED_MAX_BLOCKS * RED_K);
    if (e == hipSuccess) e = hipMalloc((void **)&h->red_out, sizeof(double) * RED_K);
    if (e == hipSuccess) e = hipMalloc((void **)&h->flag, sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(h->flag, 0, sizeof(unsigned));
    if (e != hipSuccess) {
        lbm_destroy(h);
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, "allocation: %s", hipGetErrorString(e));
    }
    // resident fused work-groups: CUs x work-groups per CU (the runtime's occupancy of the
    // steady-state kernel of this storage)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
        int per_cu = 0;
        (void)dispatch_storage(p->storage, [&](auto SI) -> int {
            int per_cu_pc = 0;
            if (sweep_occupancy<decltype(SI)::value>(&per_cu, &per_cu_pc) != hipSuccess) per_cu = per_cu_pc = 1;
            h->slots_pc = cus * (per_cu_pc > 0 ? per_cu_pc : 1);
            return LBM_OK;
        });
        h->slots = cus * (per_cu > 0 ? per_cu : 1);
    }
    codec_defaults(h);
    *out = h;
    return LBM_OK;
}

void lbm_destroy(lbm_handle h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (int b = 0; b < 2; b++) {
        if (h->F[b]) (void)hipFree(h->F[b]);
        if (h->B[b]) (void)hipFree(h->B[b]);
    }
    if (h->src) (void)hipFree(h->src);
    if (h->accel) (void)hipFree(h->accel);
    if (h->Tf) (void)hipFree(h->Tf);
    if (h->partial) (void)hipFree(h->partial);
    if (h->red_out) (void)hipFree(h->red_out);
    if (h->flag) (void)hipFree(h->flag);
    delete h;
}

int lbm_set_kernel(lbm_handle h, int kernel) {
    if (!h || kernel < 0 || kernel > 3) return fail(LBM_ERR_ARG, "bad kernel choice");
    const bool fused = kernel == 2 || kernel == 3;
    if (fused && h->proj < 3) return fail(LBM_ERR_ARG, "projected lattices step with their own kernels");
    if (fused && !fused_supported(geo(h), h->p.storage))
        return fail(LBM_ERR_ARG, "fused sweep does not support this lattice shape");
    if (kernel == 2 && h->tau_ghost > 0.0)
        return fail(LBM_ERR_ARG, "the single-role fused sweep relaxes with a single rate (a ghost rate is set)");
    if (kernel == 2 && h->walls) return fail(LBM_ERR_ARG, "the single-role fused sweep is periodic (walls are set)");
    if (kernel == 3 && !fused_pc_supported(geo(h), h->p.storage))
        return fail(LBM_ERR_ARG, "the producer/consumer sweep takes float or 16-bit storage and nz >= 3");
    h->kernel = kernel;
    return LBM_OK;
}

int lbm_set_walls(lbm_handle h, int on, const double *u_bottom, const double *u_top) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (!on) {
        h->walls = 0;
        for (int c = 0; c < 6; c++) h->uw[c] = 0.0;
        return LBM_OK;
    }
    if (h->p.nz < 3) return fail(LBM_ERR_ARG, "walls need nz >= 3 (got %d)", h->p.nz);
    if (h->proj < 3) return fail(LBM_ERR_ARG, "projected lattices have no walls");
    if (h->kernel == 2)
        return fail(LBM_ERR_ARG, "the single-role fused sweep is periodic (lbm_set_kernel chose it)");
    double uw[6] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < 3; c++) {
        if (u_bottom) uw[c] = u_bottom[c];
        if (u_top) uw[3 + c] = u_top[c];
    }
    for (int c = 0; c < 6; c++)
        if (!std::isfinite(uw[c])) return fail(LBM_ERR_ARG, "wall velocity not finite");
    if (uw[2] != 0.0 || uw[5] != 0.0) return fail(LBM_ERR_ARG, "a wall cannot move along its normal (z)");
    // the step after a change reads the new walls; bbar already gathered stays valid
    h->walls = 1;
    for (int c = 0; c < 6; c++) h->uw[c] = uw[c];
    return LBM_OK;
}

int lbm_set_projection(lbm_handle h, int dims) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (dims == h->proj) return LBM_OK;
    if (dims != 1 && dims != 2 && dims != 3) return fail(LBM_ERR_ARG, "dims must be 1, 2 or 3");
    if (dims == 2 && h->p.nz != 1) return fail(LBM_ERR_ARG, "a D2Q9 projection needs nz = 1");
    if (dims == 1 && (h->p.ny != 1 || h->p.nz != 1)) return fail(LBM_ERR_ARG, "a D1Q3 projection needs ny = nz = 1");
    if (dims < 3) {
        if (h->p.mode == LBM_STANDARD) return fail(LBM_ERR_ARG, "the standard comparator is not projected");
        if (h->kernel == 2 || h->kernel == 3)
            return fail(LBM_ERR_ARG, "projected lattices step with their own two-pass kernels");
        if (h->walls || h->accel || h->force_uniform || h->tau_ghost > 0.0)
            return fail(LBM_ERR_ARG, "projected lattices have no walls, body force or ghost rate");
    }
    HIP_TRY(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
    for (int b = 0; b < 2; b++) {
        if (h->F[b]) (void)hipFree(h->F[b]);
        if (h->B[b]) (void)hipFree(h->B[b]);
        h->F[b] = h->B[b] = nullptr;
    }
    if (h->src) (void)hipFree(h->src);
    h->src = nullptr;
    h->has_state = false;
    h->proj = dims;
    int nf = Q, nb = NB, nsrc = NSRC;
    if (dims < 3) {
        const bool th = h->p.mode == LBM_THERMAL;
        nf = dims == 2 ? (th ? ProjLayout<2, true>::NF : ProjLayout<2, false>::NF)
                       : (th ? ProjLayout<1, true>::NF : ProjLayout<1, false>::NF);
        nb = dims == 2 ? (th ? ProjLayout<2, true>::NBP : ProjLayout<2, false>::NBP)
                       : (th ? ProjLayout<1, true>::NBP : ProjLayout<1, false>::NBP);
        nsrc = dims == 2 ? ProjSet<2>::NSP : ProjSet<1>::NSP;
    }
    const size_t sb = store_bytes(h->p.storage), n = h->n;
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; b++) {
        e = hipMalloc(&h->F[b], sb * nf * n);
        if (e == hipSuccess) e = hipMalloc(&h->B[b], sb * nb * n);
    }
    // the two-pass and projected steps keep their source planes; the fused sweep needs none
    if (e == hipSuccess && (dims < 3 || !fused_supported(geo(h), h->p.storage)))
        e = hipMalloc(&h->src, compute_bytes(h->p.storage) * nsrc * n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, "allocation: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

int lbm_get_projection(lbm_handle h, int *dims, int *nf, int *nb) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    int f = Q, b = NB;
    if (h->proj < 3) {
        const bool th = h->p.mode == LBM_THERMAL;
        f = h->proj == 2 ? (th ? ProjLayout<2, true>::NF : ProjLayout<2, false>::NF)
                         : (th ? ProjLayout<1, true>::NF : ProjLayout<1, false>::NF);
        b = h->proj == 2 ? (th ? ProjLayout<2, true>::NBP : ProjLayout<2, false>::NBP)
                         : (th ? ProjLayout<1, true>::NBP : ProjLayout<1, false>::NBP);
    }
    if (dims) *dims = h->proj;
    if (nf) *nf = f;
    if (nb) *nb = b;
    return LBM_OK;
}

int lbm_set_body_force(lbm_handle h, const void *accel, int dtype, int on_device) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->accel) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        (void)hipFree(h->accel);
        h->accel = nullptr;
    }
    h->force_uniform = 0;
    for (int c = 0; c < 3; c++) h->acc_u[c] = 0.0;
    if (!accel) return LBM_OK;
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_ERR_ARG, "unknown dtype %d", dtype);
    if (h->proj < 3) return fail(LBM_ERR_ARG, "projected lattices have no body force");
    const size_t count = 3 * (size_t)h->n, eb = dtype == LBM_DTYPE_F64 ? 8 : 4;
    HIP_TRY(hipMalloc(&h->accel, compute_bytes(h->p.storage) * count));
    void *stage = nullptr;
    const void *src = accel;
    if (!on_device) {
        HIP_TRY(hipMalloc(&stage, eb * count));
        hipError_t e = hipMemcpyAsync(stage, accel, eb * count, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return fail(LBM_ERR_HIP, "copy of the body force: %s", hipGetErrorString(e));
        }
        src = stage;
    }
    const unsigned blocks = (unsigned)((count + BLOCK - 1) / BLOCK);
    int rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
        using C = typename Storage<decltype(SI)::value>::C;
        if (dtype == LBM_DTYPE_F64)
            hipLaunchKernelGGL((k_cast<double, C>), dim3(blocks), dim3(BLOCK), 0, h->stream, (const double *)src,
                               (C *)h->accel, count);
        else
            hipLaunchKernelGGL((k_cast<float, C>), dim3(blocks), dim3(BLOCK), 0, h->stream, (const float *)src,
                               (C *)h->accel, count);
        return check_launch();
    });
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (stage) (void)hipFree(stage);
    if (!rc && e != hipSuccess) rc = fail(LBM_ERR_HIP, "body force: %s", hipGetErrorString(e));
    return rc;
}

int lbm_set_body_force_uniform(lbm_handle h, const double *accel) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (accel) {
        for (int c = 0; c < 3; c++)
            if (!std::isfinite(accel[c])) return fail(LBM_ERR_ARG, "body force not finite");
        if (h->proj < 3) return fail(LBM_ERR_ARG, "projected lattices have no body force");
    }
    if (int rc = lbm_set_body_force(h, nullptr, 0, 0)) return rc;  // drops a field
    if (!accel) return LBM_OK;
    h->force_uniform = 1;
    for (int c = 0; c < 3; c++) h->acc_u[c] = accel[c];
    return LBM_OK;
}

int lbm_set_ghost_relaxation(lbm_handle h, double tau_ghost) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (!(tau_ghost > 0.0) || !std::isfinite(tau_ghost)) return fail(LBM_ERR_ARG, "tau_ghost must be > 0");
    if (h->p.mode == LBM_STANDARD) return fail(LBM_ERR_ARG, "the standard comparator relaxes with a single rate");
    if (h->proj < 3 && tau_ghost != h->p.tau) return fail(LBM_ERR_ARG, "projected lattices relax with a single rate");
    if (h->kernel == 2 && tau_ghost != h->p.tau)
        return fail(LBM_ERR_ARG, "the single-role fused sweep relaxes with a single rate (lbm_set_kernel chose it)");
    h->tau_ghost = tau_ghost == h->p.tau ? -1.0 : tau_ghost;
    return LBM_OK;
}

long lbm_steps_done(lbm_handle h) { return h ? h->steps : -1; }

size_t lbm_lattice_bytes(const lbm_params *p) {
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1 || p->storage < 0 || p->storage > 3) return 0;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    const Geo g{p->nx, p->ny, p->nz, (int)std::min<size_t>(n, 2147483647)};
    const bool two_pass = !fused_supported(g, p->storage);  // the two-pass step adds its sources
    return 2 * (size_t)NFIELD * store_bytes(p->storage) * n + (two_pass ? NSRC * compute_bytes(p->storage) * n : 0) +
           sizeof(double) * (2 * RED_MAX_BLOCKS * RED_K + RED_K) + sizeof(unsigned) +
           (p->mode == LBM_ISO || p->mode == LBM_STANDARD ? compute_bytes(p->storage) * n : 0);
}

int lbm_sync(lbm_handle h) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_set_fields(lbm_handle h, const void *rho, const void *u, const void *T, int dtype, int on_device) {
    if (!h || !rho || !u || !T) return fail(LBM_ERR_ARG, "null argument");
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_ERR_ARG, "unknown dtype %d", dtype);
    const size_t n = h->n, eb = dtype == LBM_DTYPE_F64 ? 8 : 4;
    // stage host inputs on the device
    void *stage = nullptr;
    const void *dr = rho, *du = u, *dT = T;
    if (!on_device) {
        HIP_TRY(hipMalloc(&stage, eb * 5 * n));
        char *s = (char *)stage;
        hipError_t e = hipMemcpyAsync(s, rho, eb * n, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s + eb * n, u, eb * 3 * n, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s + eb * 4 * n, T, eb * n, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return fail(LBM_ERR_HIP, "copy of fields: %s", hipGetErrorString(e));
        }
        dr = s;
        du = s + eb * n;
        dT = s + eb * 4 * n;
    }
    int rc = LBM_OK;
    const Geo g = geo(h);
    const int rb = red_blocks(h->n);
    double absmax[NFIELD + 1];
    codec_defaults(h);
    // a range flag left by steps of the previous state is not this state's
    if (int e = clear_flag(h)) {
        if (stage) (void)hipFree(stage);
        return e;
    }
    if (dtype == LBM_DTYPE_F64)
        hipLaunchKernelGGL(k_absmax_fields<double>, dim3(rb), dim3(BLOCK), 0, h->stream, (const double *)dr,
                           (const double *)du, (const double *)dT, g, h->p.rho_ref, h->p.T_ref, h->partial);
    else
        hipLaunchKernelGGL(k_absmax_fields<float>, dim3(rb), dim3(BLOCK), 0, h->stream, (const float *)dr,
                           (const float *)du, (const float *)dT, g, h->p.rho_ref, h->p.T_ref, h->partial);
    rc = check_launch();
    if (!rc) rc = finish_reduction<true>(h, rb, NFIELD + 1, absmax);
    if (!rc && absmax[NFIELD] > 0) rc = fail(LBM_ERR_ARG, "fields contain rho <= 0 or non-finite values");
    if (!rc) {
        if (h->proj < 3 && h->p.storage == LBM_F16DEV) {
            if (h->proj == 2) choose_scales_proj<2>(h, absmax); else choose_scales_proj<1>(h, absmax);
        } else {
            choose_scales(h, absmax);
        }
        // ISO: keep a per-site temperature field only if it is not uniform
        if (h->Tf) {
            (void)hipFree(h->Tf);
            h->Tf = nullptr;
        }
        bool keepT = false;
        if (h->p.mode == LBM_ISO || h->p.mode == LBM_STANDARD) {
            // uniform check on the host is cheap for host inputs; device inputs are kept as a field
            if (!on_device) {
                if (dtype == LBM_DTYPE_F64) {
                    const double *t = (const double *)T;
                    for (size_t i = 1; i < n && !keepT; i++) keepT = t[i] != t[0];
                    h->Tconst = t[0] - h->p.T_ref;
                } else {
                    const float *t = (const float *)T;
                    for (size_t i = 1; i < n && !keepT; i++) keepT = t[i] != t[0];
                    h->Tconst = (double)t[0] - h->p.T_ref;
                }
            } else {
                keepT = true;
            }
            if (keepT) {
                hipError_t e = hipMalloc(&h->Tf, compute_bytes(h->p.storage) * n);
                if (e != hipSuccess) rc = fail(LBM_ERR_OOM, "temperature field: %s", hipGetErrorString(e));
            }
        }
    }
    if (!rc && h->proj < 3) {
        rc = dispatch_proj(h, [&](auto SI, auto DI, auto TI) -> int {
            constexpr int S = decltype(SI)::value, D = decltype(DI)::value;
            constexpr bool TH = decltype(TI)::value;
            using TT = typename Storage<S>::T;
            using C = typename Storage<S>::C;
            if (dtype == LBM_DTYPE_F64)
                hipLaunchKernelGGL((k_proj_init<S, D, TH, double>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                                   (const double *)dr, (const double *)du, (const double *)dT, g, h->p.rho_ref,
                                   h->p.T_ref, (TT *)h->F[0], (TT *)h->B[0], (C *)h->Tf, h->flag, h->codec);
            else
                hipLaunchKernelGGL((k_proj_init<S, D, TH, float>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                                   (const float *)dr, (const float *)du, (const float *)dT, g, h->p.rho_ref,
                                   h->p.T_ref, (TT *)h->F[0], (TT *)h->B[0], (C *)h->Tf, h->flag, h->codec);
            return check_launch();
        });
    } else if (!rc) {
        rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
            constexpr int S = decltype(SI)::value;
            using TT = typename Storage<S>::T;
            using C = typename Storage<S>::C;
            if (h->p.mode == LBM_STANDARD) {
                if (dtype == LBM_DTYPE_F64)
                    hipLaunchKernelGGL((k_init_std<S, double>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                                       (const double *)dr, (const double *)du, (const double *)dT, g, h->codec,
                                       h->p.rho_ref, h->p.T_ref, (TT *)h->F[0], (TT *)h->B[0], (C *)h->Tf, h->flag);
                else
                    hipLaunchKernelGGL((k_init_std<S, float>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                                       (const float *)dr, (const float *)du, (const float *)dT, g, h->codec,
                                       h->p.rho_ref, h->p.T_ref, (TT *)h->F[0], (TT *)h->B[0], (C *)h->Tf, h->flag);
                // the other bbar buffer too: zero bits are a zero deviation in every storage
                const hipError_t e = hipMemsetAsync(h->B[1], 0, store_bytes(h->p.storage) * NB * n, h->stream);
                if (e != hipSuccess) return fail(LBM_ERR_HIP, "clearing bbar: %s", hipGetErrorString(e));
            } else if (dtype == LBM_DTYPE_F64)
                hipLaunchKernelGGL((k_init<S, double>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                                   (const double *)dr, (const double *)du, (const double *)dT, g, h->codec,
                                   h->p.rho_ref, h->p.T_ref, (TT *)h->F[0], (TT *)h->B[0], (C *)h->Tf, h->flag);
            else
                hipLaunchKernelGGL((k_init<S, float>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                                   (const float *)dr, (const float *)du, (const float *)dT, g, h->codec,
                                   h->p.rho_ref, h->p.T_ref, (TT *)h->F[0], (TT *)h->B[0], (C *)h->Tf, h->flag);
            return check_launch();
        });
    }
    unsigned sat = 0;
    if (!rc) rc = read_clear_flag(h, &sat);
    if (stage) (void)hipFree(stage);
    if (rc) return rc;
    if (h->proj < 3 && (sat & 2u)) return fail(LBM_ERR_ARG, "a projected lattice takes no transverse velocity");
    h->cur = 0;
    h->gathered = true;
    h->has_state = true;
    h->steps = 0;
    if (sat) return fail(LBM_ERR_RANGE, "16-bit encode saturated during set_fields");
    return LBM_OK;
}

int lbm_step(lbm_handle h, long n_steps) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (n_steps < 0) return fail(LBM_ERR_ARG, "n_steps < 0");
    if (!h->has_state) return fail(LBM_ERR_STATE, "step before set_fields/set_state");
    const bool standard = h->p.mode == LBM_STANDARD;
    for (long i = 0; i < n_steps; i++) {
        int rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
            constexpr int S = decltype(SI)::value;
            if (h->proj < 3) return step_proj(h);
            // per step: the first step after the state was set may take another kernel
            return standard ? step_std<S>(h) : use_fused(h) ? step_fused<S>(h) : step_two_pass<S>(h);
        });
        if (rc) return rc;
        h->steps++;
    }
    return LBM_OK;
}

// Tail of lbm_get_moments: copy host outputs from the staging buffer, synchronise, free it.
int finish_moments(lbm_lattice *h, int rc, void *rho, void *u, void *T, const char *dr, const char *du,
                   const char *dT, size_t eb, void *stage, int on_device) {
    const size_t n = h->n;
    if (!rc && !on_device) {
        hipError_t e = hipSuccess;
        if (rho) e = hipMemcpyAsync(rho, dr, eb * n, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, eb * 3 * n, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && T) e = hipMemcpyAsync(T, dT, eb * n, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "copy of moments: %s", hipGetErrorString(e));
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "moments: %s", hipGetErrorString(e));
    }
    if (stage) (void)hipFree(stage);
    return rc;
}

int lbm_get_moments(lbm_handle h, void *rho, void *u, void *T, int dtype, int on_device) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (!h->has_state) return fail(LBM_ERR_STATE, "no state");
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return fail(LBM_ERR_ARG, "unknown dtype %d", dtype);
    const size_t n = h->n, eb = dtype == LBM_DTYPE_F64 ? 8 : 4;
    void *stage = nullptr;
    char *dr = (char *)rho, *du = (char *)u, *dT = (char *)T;
    if (!on_device) {
        HIP_TRY(hipMalloc(&stage, eb * 5 * n));
        dr = rho ? (char *)stage : nullptr;
        du = u ? (char *)stage + eb * n : nullptr;
        dT = T ? (char *)stage + eb * 4 * n : nullptr;
    }
    const Geo g = geo(h);
    if (h->proj < 3) {
        int rc = dispatch_proj(h, [&](auto SI, auto DI, auto TI) -> int {
            constexpr int S = decltype(SI)::value, D = decltype(DI)::value;
            constexpr bool TH = decltype(TI)::value;
            using TT = typename Storage<S>::T;
            using C = typename Storage<S>::C;
            const StepConst<C> k = step_const<C>(h);
            const TT *F = (const TT *)h->F[h->cur];
            const TT *B = (const TT *)h->B[h->cur];
            const dim3 grid(blocks_for(h->n)), block(BLOCK);
            auto launch = [&](auto GI, auto OI) {
                constexpr bool G = decltype(GI)::value;
                using OUT = typename decltype(OI)::type;
                hipLaunchKernelGGL((k_proj_predict<S, D, TH, G>), grid, block, 0, h->stream, F, B, (C *)h->src,
                                   (const C *)h->Tf, (C)h->Tconst, g, k, h->codec);
                hipLaunchKernelGGL((k_proj_readout<S, D, TH, G, OUT>), grid, block, 0, h->stream, F, B,
                                   (const C *)h->src, (const C *)h->Tf, (C)h->Tconst, g, k, h->codec, h->p.T_ref,
                                   (OUT *)dr, (OUT *)du, (OUT *)dT);
            };
            struct Dd { using type = double; };
            struct Ff { using type = float; };
            if (h->gathered) {
                if (dtype == LBM_DTYPE_F64) launch(std::true_type{}, Dd{}); else launch(std::true_type{}, Ff{});
            } else {
                if (dtype == LBM_DTYPE_F64) launch(std::false_type{}, Dd{}); else launch(std::false_type{}, Ff{});
            }
            return check_launch();
        });
        return finish_moments(h, rc, rho, u, T, dr, du, dT, eb, stage, on_device);
    }
    int rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const StepConst<C> k = step_const<C>(h);
        const TT *F = (const TT *)h->F[h->cur];
        const TT *B = (const TT *)h->B[h->cur];
        // the predictor sources of the readout go to the idle population buffer: between steps
        // it holds nothing, and its 19 planes of storage type hold the 9 of compute type
        static_assert(NSRC * sizeof(C) <= Q * sizeof(TT), "source planes exceed the idle buffer");
        C *src = (C *)h->F[1 - h->cur];
        const dim3 grid(blocks_for(h->n)), block(BLOCK);
        auto launch = [&](auto GI, auto OI) {
            constexpr bool G = decltype(GI)::value;
            using OUT = typename decltype(OI)::type;
            if (h->p.mode == LBM_STANDARD) {
                hipLaunchKernelGGL((k_readout_std<S, OUT>), grid, block, 0, h->stream, F, (const C *)h->Tf,
                                   (C)h->Tconst, g, k, h->codec, h->p.T_ref, (OUT *)dr, (OUT *)du, (OUT *)dT,
                                   (const C *)h->accel);
                return;
            }
            hipLaunchKernelGGL((k_predict<S, G>), grid, block, 0, h->stream, F, B, src, (const C *)h->Tf, (C)h->Tconst, g, k,
                               h->codec, 0, h->n);
            hipLaunchKernelGGL((k_readout<S, G, OUT>), grid, block, 0, h->stream, F, B, (const C *)src, (const C *)h->Tf,
                               (C)h->Tconst, g, k, h->codec, h->p.T_ref, (OUT *)dr, (OUT *)du, (OUT *)dT, (const C *)h->accel);
        };
        struct D { using type = double; };
        struct Fl { using type = float; };
        if (h->gathered) {
            if (dtype == LBM_DTYPE_F64) launch(std::true_type{}, D{}); else launch(std::true_type{}, Fl{});
        } else {
            if (dtype == LBM_DTYPE_F64) launch(std::false_type{}, D{}); else launch(std::false_type{}, Fl{});
        }
        return check_launch();
    });
    return finish_moments(h, rc, rho, u, T, dr, du, dT, eb, stage, on_device);
}

int lbm_get_state(lbm_handle h, void *F, void *b, int on_device) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (!h->has_state) return fail(LBM_ERR_STATE, "no state");
    const size_t n = h->n;
    void *stage = nullptr;
    double *dF = (double *)F, *dB = (double *)b;
    if (!on_device) {
        HIP_TRY(hipMalloc(&stage, sizeof(double) * NFIELD * n));
        dF = F ? (double *)stage : nullptr;
        dB = b ? (double *)stage + Q * n : nullptr;
    }
    const Geo g = geo(h);
    int nf = Q, nbp = NB;
    (void)lbm_get_projection(h, nullptr, &nf, &nbp);
    int rc = h->proj < 3 ? dispatch_proj(h, [&](auto SI, auto DI, auto TI) -> int {
        constexpr int S = decltype(SI)::value, D = decltype(DI)::value;
        constexpr bool TH = decltype(TI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const TT *Fs = (const TT *)h->F[h->cur];
        const TT *Bs = (const TT *)h->B[h->cur];
        const double th_ref = h->p.T_ref - 1.0 / 3.0;
        if (h->gathered)
            hipLaunchKernelGGL((k_proj_decode<S, D, TH, true>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream, Fs,
                               Bs, g, h->codec, (C)h->p.rho_ref, th_ref, dF, dB);
        else
            hipLaunchKernelGGL((k_proj_decode<S, D, TH, false>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream, Fs,
                               Bs, g, h->codec, (C)h->p.rho_ref, th_ref, dF, dB);
        return check_launch();
    }) : dispatch_storage(h->p.storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const TT *Fs = (const TT *)h->F[h->cur];
        const TT *Bs = (const TT *)h->B[h->cur];
        if (h->gathered)
            hipLaunchKernelGGL((k_decode_state<S, true>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream, Fs, Bs, g,
                               h->codec, (C)h->p.rho_ref, dF, dB);
        else
            hipLaunchKernelGGL((k_decode_state<S, false>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream, Fs, Bs, g,
                               h->codec, (C)h->p.rho_ref, dF, dB);
        return check_launch();
    });
    if (!rc && !on_device) {
        hipError_t e = hipSuccess;
        if (F) e = hipMemcpyAsync(F, dF, sizeof(double) * nf * n, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && b) e = hipMemcpyAsync(b, dB, sizeof(double) * nbp * n, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "copy of state: %s", hipGetErrorString(e));
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "get_state: %s", hipGetErrorString(e));
    }
    if (stage) (void)hipFree(stage);
    return rc;
}

int lbm_get_stored(lbm_handle h, void *F, void *b, int *b_is_gathered, int on_device) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->proj < 3) return fail(LBM_ERR_ARG, "not available on a projected lattice");
    if (!h->has_state) return fail(LBM_ERR_STATE, "no state");
    const size_t n = h->n;
    void *stage = nullptr;
    double *dF = (double *)F, *dB = (double *)b;
    if (!on_device) {
        HIP_TRY(hipMalloc(&stage, sizeof(double) * NFIELD * n));
        dF = F ? (double *)stage : nullptr;
        dB = b ? (double *)stage + Q * n : nullptr;
    }
    const Geo g = geo(h);
    int rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        using TT = typename Storage<S>::T;
        hipLaunchKernelGGL((k_decode_stored<S>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream,
                           (const TT *)h->F[h->cur], (const TT *)h->B[h->cur], g, h->codec, dF, dB);
        return check_launch();
    });
    if (!rc && !on_device) {
        hipError_t e = hipSuccess;
        if (F) e = hipMemcpyAsync(F, dF, sizeof(double) * Q * n, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && b) e = hipMemcpyAsync(b, dB, sizeof(double) * NB * n, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "copy of stored state: %s", hipGetErrorString(e));
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "get_stored: %s", hipGetErrorString(e));
    }
    if (stage) (void)hipFree(stage);
    if (!rc && b_is_gathered) *b_is_gathered = h->gathered ? 1 : 0;
    return rc;
}

int lbm_set_state(lbm_handle h, const void *F, const void *b, int on_device) {
    if (!h || !F || !b) return fail(LBM_ERR_ARG, "null argument");
    if (h->proj < 3) return fail(LBM_ERR_ARG, "not available on a projected lattice");
    if ((h->p.mode == LBM_ISO || h->p.mode == LBM_STANDARD) && !h->has_state)
        return fail(LBM_ERR_STATE, "ISO and STANDARD mode: set_fields first (it provides the temperature field)");
    const size_t n = h->n;
    void *stage = nullptr;
    const double *dF = (const double *)F, *dB = (const double *)b;
    if (!on_device) {
        HIP_TRY(hipMalloc(&stage, sizeof(double) * NFIELD * n));
        hipError_t e = hipMemcpyAsync(stage, F, sizeof(double) * Q * n, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((double *)stage + Q * n, b, sizeof(double) * NB * n, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return fail(LBM_ERR_HIP, "copy of state: %s", hipGetErrorString(e));
        }
        dF = (const double *)stage;
        dB = (const double *)stage + Q * n;
    }
    const Geo g = geo(h);
    const int rb = red_blocks(h->n);
    double absmax[NFIELD + 1];
    codec_defaults(h);
    if (int e = clear_flag(h)) {
        if (stage) (void)hipFree(stage);
        return e;
    }
    hipLaunchKernelGGL(k_absmax_state<0>, dim3(rb), dim3(BLOCK), 0, h->stream, dF, dB, g, h->codec, h->partial);
    int rc = check_launch();
    if (!rc) rc = finish_reduction<true>(h, rb, NFIELD + 1, absmax);
    if (!rc && absmax[NFIELD] > 0) rc = fail(LBM_ERR_ARG, "state contains non-finite values");
    if (!rc) {
        choose_scales(h, absmax);
        rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
            constexpr int S = decltype(SI)::value;
            using TT = typename Storage<S>::T;
            hipLaunchKernelGGL((k_encode_state<S>), dim3(blocks_for(h->n)), dim3(BLOCK), 0, h->stream, dF, dB, g,
                               h->codec, (TT *)h->F[0], (TT *)h->B[0], h->flag);
            return check_launch();
        });
    }
    unsigned sat = 0;
    if (!rc) rc = read_clear_flag(h, &sat);
    if (stage) (void)hipFree(stage);
    if (rc) return rc;
    h->cur = 0;
    h->gathered = true;
    h->has_state = true;
    h->steps = 0;
    if (sat) return fail(LBM_ERR_RANGE, "16-bit encode saturated during set_state");
    return LBM_OK;
}

int lbm_get_codec(lbm_handle h, double *scales25, double *refs25) {
    if (!h || !scales25 || !refs25) return fail(LBM_ERR_ARG, "null argument");
    if (h->p.storage != LBM_F16DEV && h->p.storage != LBM_BF16DEV) return fail(LBM_ERR_ARG, "not a 16-bit storage");
    for (int k = 0; k < NFIELD; k++) {
        scales25[k] = h->codec.scale[k];
        refs25[k] = h->codec.ref[k];
    }
    return LBM_OK;
}

int lbm_get_raw(lbm_handle h, void *F_codes, void *b_codes, int on_device) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (h->p.storage != LBM_F16DEV && h->p.storage != LBM_BF16DEV) return fail(LBM_ERR_ARG, "not a 16-bit storage");
    if (!h->has_state || !h->gathered || h->cur != 0) return fail(LBM_ERR_STATE, "raw codes only right after set_fields/set_state");
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (F_codes) HIP_TRY(hipMemcpyAsync(F_codes, h->F[0], 2 * Q * (size_t)h->n, kind, h->stream));
    if (b_codes) HIP_TRY(hipMemcpyAsync(b_codes, h->B[0], 2 * NB * (size_t)h->n, kind, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_invariants(lbm_handle h, double out[5]) {
    if (!h || !out) return fail(LBM_ERR_ARG, "null argument");
    if (h->proj < 3) return fail(LBM_ERR_ARG, "not available on a projected lattice");
    if (!h->has_state) return fail(LBM_ERR_STATE, "no state");
    const Geo g = geo(h);
    const int rb = red_blocks(h->n);
    int rc = dispatch_storage(h->p.storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const TT *F = (const TT *)h->F[h->cur];
        const TT *B = (const TT *)h->B[h->cur];
        if (h->gathered)
            hipLaunchKernelGGL((k_invariants<S, true>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, h->p.T_ref - 1.0 / 3.0, h->partial);
        else
            hipLaunchKernelGGL((k_invariants<S, false>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, h->p.T_ref - 1.0 / 3.0, h->partial);
        return check_launch();
    });
    if (!rc) rc = finish_reduction<false>(h, rb, 5, out);
    return rc;
}

int lbm_health(lbm_handle h, long counts[2], double *max_u) {
    if (!h) return fail(LBM_ERR_ARG, "null handle");
    if (!h->has_state) return fail(LBM_ERR_STATE, "no state");
    const Geo g = geo(h);
    const int rb = red_blocks(h->n);
    double *pmax = h->partial + (size_t)RED_MAX_BLOCKS * RED_K;
    int rc = h->proj < 3 ? dispatch_proj(h, [&](auto SI, auto DI, auto TI) -> int {
        constexpr int S = decltype(SI)::value, D = decltype(DI)::value;
        constexpr bool TH = decltype(TI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const TT *F = (const TT *)h->F[h->cur];
        const TT *B = (const TT *)h->B[h->cur];
        if (h->gathered)
            hipLaunchKernelGGL((k_proj_health<S, D, TH, true>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, h->partial, pmax);
        else
            hipLaunchKernelGGL((k_proj_health<S, D, TH, false>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, h->partial, pmax);
        return check_launch();
    }) : dispatch_storage(h->p.storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const TT *F = (const TT *)h->F[h->cur];
        const TT *B = (const TT *)h->B[h->cur];
        if (h->gathered)
            hipLaunchKernelGGL((k_health<S, true>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, h->partial, pmax);
        else
            hipLaunchKernelGGL((k_health<S, false>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, h->partial, pmax);
        return check_launch();
    });
    double sums[2] = {0, 0}, mx = 0;
    if (!rc) rc = finish_reduction<false>(h, rb, 2, sums);
    if (!rc) {
        hipLaunchKernelGGL(k_reduce_final<true>, dim3(1), dim3(BLOCK), 0, h->stream, pmax, rb, 1, h->red_out);
        rc = check_launch();
        if (!rc) {
            hipError_t e = hipMemcpyAsync(&mx, h->red_out, sizeof(double), hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) rc = fail(LBM_ERR_HIP, "health: %s", hipGetErrorString(e));
        }
    }
    // the range flag of 16-bit codes that overflowed since the state was set or last checked
    unsigned range = 0;
    if (!rc) rc = read_clear_flag(h, &range);
    if (rc) return rc;
    if (counts) {
        counts[0] = (long)sums[0];
        counts[1] = (long)sums[1];
    }
    if (max_u) *max_u = mx;
    if (range & 1u)
        return fail(LBM_ERR_RANGE, "16-bit code overflow since the last check (stored as +-inf); %ld non-finite sites, "
                    "%ld sites with rho <= 0", (long)sums[0], (long)sums[1]);
    if (sums[0] > 0 || sums[1] > 0) return fail(LBM_ERR_DIVERGED, "%ld non-finite sites, %ld sites with rho <= 0", (long)sums[0], (long)sums[1]);
    return LBM_OK;
}

}  // extern "C"
