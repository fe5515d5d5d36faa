// lbm_internal.hpp -- the lattice object behind an lbm_handle, shared by the C-ABI and the
// serving runtime (both in liblbm.so).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

struct lbm_lattice {
    lbm_params p{};
    hipStream_t stream = nullptr;
    int device = 0;           // the HIP device the lattice was created on
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
    int slots_pc = 256;         // the same for the producer/consumer sweep
    double tau_ghost = -1.0;    // relaxation time of Table I rows 11-19 (<= 0: the single rate)
    void *accel = nullptr;      // body-force acceleration, 3 planes of the compute type, or null
    int force_uniform = 0;      // 1: a uniform body-force acceleration acc_u (no field)
    double acc_u[3] = {0, 0, 0};
    int walls = 0;              // 1: walls normal to z bound the lattice (lbm_set_walls)
    double uw[6] = {0, 0, 0, 0, 0, 0};  // velocities of the bottom and top walls
    int proj = 3;               // 3: D3Q19; 2, 1: the projected lattice of lbm_set_projection
};

namespace lbm {
// Sets the calling thread's lbm_last_error() message; returns code.
int set_error(int code, const char *msg);

// omega = 1/(tau + 1/2) in the compute precision C, chosen so that 1 - omega is exact in C as
// well: the update (1 - omega) d + omega feq then hands the momentum on with a coefficient of
// exactly 1 (two separately rounded constants could sum to 1 + 3e-8 in single precision,
// which compounds step after step).  For omega >= 1/2, 1 - omega is exact for any omega of C
// (Sterbenz); below, omega is rounded to a multiple of 2^-digits, the spacing of C in [1/2, 1).
template <typename C> inline double compute_omega(double tau) {
    const double omega = 1.0 / (tau + 0.5);
    if (omega >= 0.5) return (double)(C)omega;
    const int digits = std::numeric_limits<C>::digits;
    return std::ldexp(std::nearbyint(std::ldexp(omega, digits)), -digits);
}

// Step constants of a lattice (Eq. 55 and the deviation references) in the compute precision C.
template <typename C> inline StepConst<C> step_const(const lbm_lattice *h) {
    StepConst<C> k;
    const double omega = compute_omega<C>(h->p.tau);
    k.omega = (C)omega;
    k.half_omega = (C)(0.5 * omega);
    k.fcoef = (C)(1.0 - 0.5 * omega);
    k.rho_ref = (C)h->p.rho_ref;
    k.theta_ref = (C)(h->p.T_ref - 1.0 / 3.0);
    k.K = (C)(h->p.rho_ref * (h->p.T_ref - 1.0 / 3.0));
    k.om1 = (C)(1.0 - omega);  // exact: omega is a value of C (compute_omega)
    k.ghost = h->tau_ghost > 0.0 ? (C)(1.0 - (1.0 / (h->tau_ghost + 0.5)) / omega) : C(0);
    for (int c = 0; c < 3; c++) {
        k.uwb[c] = (C)h->uw[c];
        k.uwt[c] = (C)h->uw[3 + c];
        k.au[c] = (C)h->acc_u[c];
    }
    k.force_u = h->force_uniform && !h->accel;
    k.iso = h->p.mode == LBM_ISO;
    return k;
}

}  // namespace lbm
