// lbm_internal.hpp -- the lattice object behind an lbm_handle, shared by the C-ABI and the
// serving runtime (both in liblbm.so).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

struct lbm_lattice {
    lbm_params p{};
    hipStream_t stream = nullptr;
    int n = 0;
    void *F[2] = {nullptr, nullptr};
    void *B[2] = {nullptr, nullptr};
    void *src = nullptr;
    void *Tf = nullptr;       // ISO temperature field (compute type), or null when uniform
    double Tconst = 0.0;      // ISO uniform temperature, stored as theta = T - T_ref
    int cur = 0;
    bool gathered = true;
    bool has_state = false;
    long steps = 0;
    lbm::Codec codec{};
    double *partial = nullptr;  // 2 * RED_MAX_BLOCKS * RED_K (sum and max partials)
    double *red_out = nullptr;  // RED_K
    unsigned *flag = nullptr;   // saturation flag
    int kernel = 0;
    int slots = 256;            // fused work-groups resident at once (one per CU)
    double tau_ghost = -1.0;    // relaxation time of Table I rows 11-19 (<= 0: the single rate)
    void *accel = nullptr;      // body-force acceleration, 3 planes of the compute type, or null
    int walls = 0;              // 1: walls normal to z bound the lattice (lbm_set_walls)
    double uw[6] = {0, 0, 0, 0, 0, 0};  // velocities of the bottom and top walls
    int proj = 3;               // 3: D3Q19; 2, 1: the projected lattice of lbm_set_projection
};

namespace lbm {
// Sets the calling thread's lbm_last_error() message; returns code.
int set_error(int code, const char *msg);
}  // namespace lbm
