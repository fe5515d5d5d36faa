// lbm_noalloc.hip -- lbm_invariants_noalloc: the global invariants of lbm_invariants computed
// without any device allocation, and without synchronising when the result goes to device
// memory, for callers that cannot allocate (code under HIP graph capture, serving loops, hosts
// that forbid hipMalloc).
//
// The reduction's partial sums live in `scratch`, a file-scope device array: each GPU the
// library runs on holds one copy until the process ends, and every call on that GPU shares it.
// Its size does not grow with the lattice: the reduction launches at most RED_MAX_BLOCKS
// work-groups, each striding over the lattice, and one work-group folds their partials.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"
#include "lbm_kernels.hpp"

using namespace lbm;

namespace {

// RED_MAX_BLOCKS partials of RED_K doubles, then the 5 results of a call with a host output.
constexpr size_t NOALLOC_PARTIALS = (size_t)RED_MAX_BLOCKS * RED_K;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_PARTIALS + 8;  // 256 KiB + 64 B per GPU
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

// Device addresses of `scratch`, one per GPU, taken once with that GPU current.  In host code
// the array's name is only a stand-in; kernels and copies take these addresses.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

int scratch_address(int dev, double **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(LBM_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(LBM_ERR_HIP, "hipGetSymbolAddress(scratch) failed");
        }
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

int reduce_invariants(lbm_lattice *h, double *ptr, double *out, int on_device) {
    const Geo g{h->p.nx, h->p.ny, h->p.nz, h->n, h->walls};
    const int want = (h->n + BLOCK - 1) / BLOCK;
    const int rb = want < RED_MAX_BLOCKS ? want : RED_MAX_BLOCKS;
    if ((size_t)rb * RED_K > NOALLOC_PARTIALS) return set_error(LBM_ERR_ARG, "reduction exceeds the static scratch");
    auto launch = [&](auto SI) {
        constexpr int S = decltype(SI)::value;
        using TT = typename Storage<S>::T;
        using C = typename Storage<S>::C;
        const TT *F = (const TT *)h->F[h->cur];
        const TT *B = (const TT *)h->B[h->cur];
        const double th_ref = h->p.T_ref - 1.0 / 3.0;
        if (h->gathered)
            hipLaunchKernelGGL((k_invariants<S, true>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, th_ref, ptr);
        else
            hipLaunchKernelGGL((k_invariants<S, false>), dim3(rb), dim3(BLOCK), 0, h->stream, F, B, g, h->codec,
                               (C)h->p.rho_ref, th_ref, ptr);
    };
    switch (h->p.storage) {
    case LBM_F64: launch(std::integral_constant<int, 0>{}); break;
    case LBM_F32: launch(std::integral_constant<int, 1>{}); break;
    case LBM_F16DEV: launch(std::integral_constant<int, 2>{}); break;
    default: launch(std::integral_constant<int, 3>{}); break;
    }
    double *res = on_device ? out : ptr + NOALLOC_PARTIALS;
    hipLaunchKernelGGL(k_reduce_final<false>, dim3(1), dim3(BLOCK), 0, h->stream, ptr, rb, 5, res);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LBM_ERR_HIP, hipGetErrorString(e));
    if (!on_device) {
        e = hipMemcpyAsync(out, res, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return set_error(LBM_ERR_HIP, hipGetErrorString(e));
    }
    return LBM_OK;
}

}  // namespace

extern "C" int lbm_invariants_noalloc(lbm_handle h, double *out, int on_device) {
    if (!h || !out) return set_error(LBM_ERR_ARG, "null argument");
    if (h->proj < 3) return set_error(LBM_ERR_ARG, "not available on a projected lattice");
    if (!h->has_state) return set_error(LBM_ERR_STATE, "no state");
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return set_error(LBM_ERR_HIP, "hipGetDevice failed");
    if (prev != h->device && hipSetDevice(h->device) != hipSuccess)
        return set_error(LBM_ERR_HIP, "hipSetDevice to the lattice's device failed");
    double *ptr = nullptr;
    int rc = scratch_address(h->device, &ptr);
    if (!rc) rc = reduce_invariants(h, ptr, out, on_device);
    if (prev != h->device) (void)hipSetDevice(prev);
    return rc;
}
