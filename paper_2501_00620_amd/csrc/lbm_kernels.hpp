// lbm_kernels.hpp -- HIP kernels of liblbm (gfx950): initialisation, the two-pass step,
// readout, state codec and FP64 diagnostics reductions.
//
// Device layout of one lattice (n = nx*ny*nz sites, x fastest):
//   F[2]  : 19 planes of n stored values (ping-pong), post-stream populations fbar_i(x)
//   B[2]  : 6 planes of n stored values, bbar in one of two forms:
//             gathered  -- bbar(x) itself (after set_fields / set_state)
//             scattered -- the post-collision bbar*(x) of the previous step, not yet carried
//                          along; the step (and every readout) gathers
//                          bbar(x) = sum_i fbar_i(x) bbar*(x - e_i) / rho(x)   (Eq. 66)
//                          using the post-stream populations fbar_i(x) = fbar*_i(x - e_i)
//                          as weights.
//   src   : 9 planes of n compute-type values, the predictor sources rho*b (6) and u* (3).
// The step pushes fbar*_i(x) to x + e_i and stores bbar*(x) at x, so the populations are always
// held post-stream and bbar becomes scattered after the first step.
//
// Walls (Geo::walls): two planes normal to z, half-way outside planes 0 and nz - 1 (the channels
// of Sec. III A and C); x and y stay periodic.  A population pushed through a wall lands in the
// opposite slot of its own site (half-way bounce-back) with the moving-wall momentum
// -6 w_i rho e_i.u_w; its gather weight takes the site's own bbar* (a reversal maps the second
// moment onto itself).  Beyond a wall the gradient sources are the wall-adjacent plane's rho b
// (mirrored) and the second-order extrapolation of rho b u* (grad_add_wall).
#pragma once

#include <type_traits>

#include "lbm_device.hpp"

namespace lbm {

constexpr int BLOCK = 256;

struct Geo {
    int nx, ny, nz;
    int n;          // sites
    int walls = 0;  // 1: walls bound z (see the header), 0: periodic
};

// Bit 0: the site is next to the wall below plane 0; bit 1: next to the wall above plane nz - 1.
__device__ __forceinline__ int wall_bits(const Geo &g, int z) {
    return g.walls ? (int)(z == 0) | ((int)(z == g.nz - 1) << 1) : 0;
}

// Population I arriving at a site with wall bits zw came back through a wall (x - e_I is beyond).
template <int I> __device__ __forceinline__ bool arrives_from_wall(int zw) {
    return (EZ[I] == 1 && (zw & 1)) || (EZ[I] == -1 && (zw & 2));
}
// Population I leaving a site with wall bits zw goes into a wall (x + e_I is beyond).
template <int I> __device__ __forceinline__ bool leaves_into_wall(int zw) {
    return (EZ[I] == -1 && (zw & 1)) || (EZ[I] == 1 && (zw & 2));
}

__device__ __forceinline__ void site_xyz(int s, const Geo &g, int &x, int &y, int &z) {
    x = s % g.nx;
    const int t = s / g.nx;
    y = t % g.ny;
    z = t / g.ny;
}

// Load the 19 population deviations of a site and its (gathered) bbar deviation.  The gather
// weights are the full post-stream populations w_i rho_ref + d_i; since they sum to rho, the
// reference part of bbar passes through unchanged and only beta is averaged.
template <int S, bool GATHERED>
__device__ __forceinline__ void load_site(const typename Storage<S>::T *__restrict__ F,
                                          const typename Storage<S>::T *__restrict__ B, size_t n,
                                          const Nbr &nb, int s, const Codec &cd, typename Storage<S>::C rho_ref,
                                          typename Storage<S>::C f[Q], typename Storage<S>::C bbar[NB],
                                          PopMoments<typename Storage<S>::C> &m, int zw = 0) {
    using C = typename Storage<S>::C;
    Unroll<0, Q>::run([&](auto I) { f[I] = Storage<S>::load(F, (size_t)I * n + s, I, cd); });
    m = pop_moments(f, rho_ref);
    if constexpr (GATHERED) {
#pragma unroll
        for (int c = 0; c < NB; c++) bbar[c] = Storage<S>::load(B, (size_t)c * n + s, Q + c, cd);
    } else {
        C acc[NB];
#pragma unroll
        for (int c = 0; c < NB; c++) acc[c] = C(0);
        Unroll<0, Q>::run([&](auto I) {
            const int up = arrives_from_wall<I>(zw) ? s : nb.at(-EX[I], -EY[I], -EZ[I]);
            const C wgt = fma(C(WQ[I]), rho_ref, f[I]);
#pragma unroll
            for (int c = 0; c < NB; c++) acc[c] += wgt * Storage<S>::load(B, (size_t)c * n + up, Q + c, cd);
        });
        const C inv = recip(m.rho);
#pragma unroll
        for (int c = 0; c < NB; c++) bbar[c] = acc[c] * inv;
    }
}

template <typename C>
__device__ __forceinline__ C site_T(const C *Tf, C Tconst, int s) {
    return Tf ? Tf[s] : Tconst;
}

// ---- pass A: predictor sources ---------------------------------------------------------------
// The launch covers sites s0 .. s0 + count - 1 (all of them, or the planes next to the walls
// that the wall planes' collision reads when the interior steps in the fused sweep).
template <int S, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_predict(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
          typename Storage<S>::C *__restrict__ src, const typename Storage<S>::C *__restrict__ Tf,
          typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd, int s0, int count) {
    using C = typename Storage<S>::C;
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= count) return;
    const int s = s0 + t;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    C f[Q], bbar[NB];
    PopMoments<C> m;
    load_site<S, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, f, bbar, m, wall_bits(g, z));
    C o[NSRC];
    predictor_sources(m, bbar, site_T(Tf, Tconst, s), k, o);
#pragma unroll
    for (int c = 0; c < NSRC; c++) src[(size_t)c * g.n + s] = o[c];
}

// Gradient forcing moments at a site from the source planes.  WALLS: the lattice has walls;
// zw: wall bits of the site; nxy: the plane stride (used only next to a wall).
template <bool WALLS, typename C>
__device__ __forceinline__ void gradient_from_src(const C *__restrict__ src, size_t n, const Nbr &nb, C K,
                                                  C F[3], C S[6], int zw = 0, int nxy = 0) {
    GradAcc<C> acc;
    grad_init(acc);
    Unroll<1, Q>::run([&](auto I) {
        if (WALLS && leaves_into_wall<I>(zw)) {
            // the column of the neighbour, inwards from the wall-adjacent plane
            const int base = nb.at(EX[I], EY[I], 0);
            const int step = EZ[I] < 0 ? nxy : -nxy;
            C s0[NSRC], s1[NSRC], s2[NSRC];
#pragma unroll
            for (int c = 0; c < NSRC; c++) {
                s0[c] = src[(size_t)c * n + base];
                s1[c] = src[(size_t)c * n + base + step];
                s2[c] = src[(size_t)c * n + base + 2 * step];
            }
            grad_add_wall<C, I>(acc, s0, s1, s2, K);
            return;
        }
        const int at = nb.at(EX[I], EY[I], EZ[I]);
        C sv[NSRC];
#pragma unroll
        for (int c = 0; c < NSRC; c++) sv[c] = src[(size_t)c * n + at];
        grad_add<C, I>(acc, sv, K);
    });
    grad_finish(acc, F, S);
}

// ---- pass B: gradients, collision, push-stream ------------------------------------------------
// MRT: the non-hydrodynamic moments relax at their own rate (ghost_relax).  WALLS: the lattice
// has walls (the periodic instantiation carries no wall code; on a lattice with walls it serves
// the interior planes, which no wall touches).  The launch covers sites s0 .. s0 + count - 1.
template <int S, bool GATHERED, bool MRT = false, bool WALLS = false>
__global__ void __launch_bounds__(BLOCK)
k_collide(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
          const typename Storage<S>::C *__restrict__ src, typename Storage<S>::T *__restrict__ Fo,
          typename Storage<S>::T *__restrict__ Bo, const typename Storage<S>::C *__restrict__ Tf,
          typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd,
          unsigned *__restrict__ flag, const typename Storage<S>::C *__restrict__ accel, int s0, int count) {
    using C = typename Storage<S>::C;
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= count) return;
    const int s = s0 + t;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    const int zw = WALLS ? wall_bits(g, z) : 0;
    C f[Q], bbar[NB];
    PopMoments<C> m;
    load_site<S, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, f, bbar, m, zw);
    C Fv[3], Sv[6];
    gradient_from_src<WALLS>(src, g.n, nb, k.K, Fv, Sv, zw, g.nx * g.ny);
    if (accel || k.force_u) {  // body force (a branch uniform over the launch)
        C a[3];
        site_accel(k, accel, g.n, s, a);
        add_body_force(m, a, Fv, Sv);
    }
    C g0[MRT ? 9 : 1];
    if constexpr (MRT) ghost_moments(f, g0);
    collide(f, bbar, m, Fv, Sv, site_T(Tf, Tconst, s), k);
    if constexpr (MRT) ghost_relax(g0, f, k.ghost);
    unsigned sat = 0;
    Unroll<0, Q>::run([&](auto I) {
        if (WALLS && leaves_into_wall<I>(zw)) {  // half-way bounce-back, moving-wall momentum
            const C *uw = EZ[I] < 0 ? k.uwb : k.uwt;
            const C mom = C(6.0 * WQ[I]) * m.rho * (C(EX[I]) * uw[0] + C(EY[I]) * uw[1]);
            Storage<S>::store(Fo, (size_t)OPP[I] * g.n + s, OPP[I], f[I] - mom, cd, sat);
        } else {
            Storage<S>::store(Fo, (size_t)I * g.n + nb.at(EX[I], EY[I], EZ[I]), I, f[I], cd, sat);
        }
    });
#pragma unroll
    for (int c = 0; c < NB; c++) Storage<S>::store(Bo, (size_t)c * g.n + s, Q + c, bbar[c], cd, sat);
    if (sat) *flag = 1u;
}

// ---- readout of corrected moments (after k_predict on the same state) -----------------------
template <int S, bool GATHERED, typename OUT>
__global__ void __launch_bounds__(BLOCK)
k_readout(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
          const typename Storage<S>::C *__restrict__ src, const typename Storage<S>::C *__restrict__ Tf,
          typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd, double T_ref,
          OUT *__restrict__ rho, OUT *__restrict__ u, OUT *__restrict__ T,
          const typename Storage<S>::C *__restrict__ accel) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    const int zw = wall_bits(g, z);
    C f[Q], bbar[NB];
    PopMoments<C> m;
    load_site<S, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, f, bbar, m, zw);
    C Fv[3], Sv[6];
    gradient_from_src<true>(src, g.n, nb, k.K, Fv, Sv, zw, g.nx * g.ny);
    if (accel || k.force_u) {
        C a[3];
        site_accel(k, accel, g.n, s, a);
        add_body_force(m, a, Fv, Sv);
    }
    C uc[3], Tc;
    collide(f, bbar, m, Fv, Sv, site_T(Tf, Tconst, s), k, uc, &Tc);
    if (rho) rho[s] = (OUT)((double)k.rho_ref + (double)m.drho);
    if (u) {
        u[s] = (OUT)uc[0];
        u[(size_t)g.n + s] = (OUT)uc[1];
        u[2 * (size_t)g.n + s] = (OUT)uc[2];
    }
    if (T) T[s] = (OUT)(T_ref + (double)Tc);
}

// ---- initialisation from fields: fbar = feq(rho,u), bbar = beq(u,T) (gathered) ---------------
// Deviations are formed in double from the inputs, then stored.  ISO keeps theta = T - T_ref.
template <int S, typename IN>
__global__ void __launch_bounds__(BLOCK)
k_init(const IN *__restrict__ rho, const IN *__restrict__ u, const IN *__restrict__ T, Geo g, Codec cd,
       double rho_ref, double T_ref, typename Storage<S>::T *__restrict__ F, typename Storage<S>::T *__restrict__ B,
       typename Storage<S>::C *__restrict__ Tf, unsigned *__restrict__ flag) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    const size_t n = g.n;
    const double r = (double)rho[s], ux = (double)u[s], uy = (double)u[n + s], uz = (double)u[2 * n + s];
    const double theta = (double)T[s] - T_ref;
    double f[Q], b[NB];
    equilibrium_dev(r - rho_ref, r, ux, uy, uz, f);
    variance_eq_dev(ux, uy, uz, theta, b);
    unsigned sat = 0;
    Unroll<0, Q>::run([&](auto I) { Storage<S>::store(F, (size_t)I * n + s, I, (C)f[I], cd, sat); });
#pragma unroll
    for (int c = 0; c < NB; c++) Storage<S>::store(B, (size_t)c * n + s, Q + c, (C)b[c], cd, sat);
    if (Tf) Tf[s] = (C)theta;
    if (sat) *flag = 1u;
}

// ---- conversion of a caller's field to the compute type ------------------------------------------
template <typename IN, typename C>
__global__ void __launch_bounds__(BLOCK) k_cast(const IN *__restrict__ in, C *__restrict__ out, size_t count) {
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < count) out[i] = (C)in[i];
}

// ---- standard lattice Boltzmann comparator (Sec. I, Eq. 4) ---------------------------------------
// The populations carry no variance: bbar stays at its reference (deviation 0); T is the
// prescribed field (theta = T - T_ref per site, or the constant).
template <int S, typename IN>
__global__ void __launch_bounds__(BLOCK)
k_init_std(const IN *__restrict__ rho, const IN *__restrict__ u, const IN *__restrict__ T, Geo g, Codec cd,
           double rho_ref, double T_ref, typename Storage<S>::T *__restrict__ F, typename Storage<S>::T *__restrict__ B,
           typename Storage<S>::C *__restrict__ Tf, unsigned *__restrict__ flag) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    const size_t n = g.n;
    const double r = (double)rho[s], ux = (double)u[s], uy = (double)u[n + s], uz = (double)u[2 * n + s];
    double f[Q];
    equilibrium_std_dev(r - rho_ref, r, ux, uy, uz, (double)T[s] - 1.0 / 3.0, f);
    unsigned sat = 0;
    Unroll<0, Q>::run([&](auto I) { Storage<S>::store(F, (size_t)I * n + s, I, (C)f[I], cd, sat); });
#pragma unroll
    for (int c = 0; c < NB; c++) Storage<S>::store(B, (size_t)c * n + s, Q + c, C(0), cd, sat);
    if (Tf) Tf[s] = (C)((double)T[s] - T_ref);
    if (sat) *flag = 1u;
}

// One step: BGK with the scheme's relaxation factor, d' = (1 - omega) d + omega d_eq, and the
// push to the 19 neighbours.  With a body force a: u = (j + rho a / 2) / rho and the forcing
// (1 - omega/2) Phi of F = rho a, S = rho (u a + a u); no gradient forcing (no variance).
// Walls as in the bump scheme (the header).
// The launch covers sites s0 .. s0 + count - 1 (walls: the interior planes and the wall planes
// are separate launches, as for k_collide).
template <int S, bool WALLS = false>
__global__ void __launch_bounds__(BLOCK)
k_std(const typename Storage<S>::T *__restrict__ F, typename Storage<S>::T *__restrict__ Fo,
      const typename Storage<S>::C *__restrict__ Tf, typename Storage<S>::C Tconst, Geo g,
      StepConst<typename Storage<S>::C> k, Codec cd, unsigned *__restrict__ flag,
      const typename Storage<S>::C *__restrict__ accel, int s0, int count) {
    using C = typename Storage<S>::C;
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= count) return;
    const int s = s0 + t;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    const int zw = WALLS ? wall_bits(g, z) : 0;
    C d[Q], feq[Q];
    Unroll<0, Q>::run([&](auto I) { d[I] = Storage<S>::load(F, (size_t)I * g.n + s, I, cd); });
    const PopMoments<C> m = pop_moments(d, k.rho_ref);
    const C inv = recip(m.rho);
    const C th = site_T(Tf, Tconst, s) + k.theta_ref;
    if (accel || k.force_u) {  // a branch uniform over the launch
        C a[3];
        site_accel(k, accel, g.n, s, a);
        const C Fv[3] = {m.rho * a[0], m.rho * a[1], m.rho * a[2]};
        const C u[3] = {fma(C(0.5), Fv[0], m.jx) * inv, fma(C(0.5), Fv[1], m.jy) * inv,
                        fma(C(0.5), Fv[2], m.jz) * inv};
        const C Sv[6] = {C(2) * u[0] * Fv[0], C(2) * u[1] * Fv[1], C(2) * u[2] * Fv[2],
                         fma(u[0], Fv[1], u[1] * Fv[0]), fma(u[0], Fv[2], u[2] * Fv[0]),
                         fma(u[1], Fv[2], u[2] * Fv[1])};
        C phi[Q];
        forcing_pops(Fv, Sv, phi);
        equilibrium_std_dev(m.drho, m.rho, u[0], u[1], u[2], th, feq);
#pragma unroll
        for (int i = 0; i < Q; i++) feq[i] = fma(k.fcoef, phi[i], k.omega * feq[i]);
    } else {
        equilibrium_std_dev(m.drho, m.rho, m.jx * inv, m.jy * inv, m.jz * inv, th, feq);
#pragma unroll
        for (int i = 0; i < Q; i++) feq[i] = k.omega * feq[i];
    }
    unsigned sat = 0;
    Unroll<0, Q>::run([&](auto I) {
        const C post = fma(k.om1, d[I], feq[I]);
        if (WALLS && leaves_into_wall<I>(zw)) {
            const C *uw = EZ[I] < 0 ? k.uwb : k.uwt;
            const C mom = C(6.0 * WQ[I]) * m.rho * (C(EX[I]) * uw[0] + C(EY[I]) * uw[1]);
            Storage<S>::store(Fo, (size_t)OPP[I] * g.n + s, OPP[I], post - mom, cd, sat);
        } else {
            Storage<S>::store(Fo, (size_t)I * g.n + nb.at(EX[I], EY[I], EZ[I]), I, post, cd, sat);
        }
    });
    if (sat) *flag = 1u;
}

// Moments of the standard model: rho, u = (j + rho a / 2) / rho (a: the body force, or none),
// and the prescribed T.
template <int S, typename OUT>
__global__ void __launch_bounds__(BLOCK)
k_readout_std(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::C *__restrict__ Tf,
              typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd, double T_ref,
              OUT *__restrict__ rho, OUT *__restrict__ u, OUT *__restrict__ T,
              const typename Storage<S>::C *__restrict__ accel) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    C d[Q];
    Unroll<0, Q>::run([&](auto I) { d[I] = Storage<S>::load(F, (size_t)I * g.n + s, I, cd); });
    const PopMoments<C> m = pop_moments(d, k.rho_ref);
    C j[3] = {m.jx, m.jy, m.jz};
    if (accel || k.force_u) {
        C a[3];
        site_accel(k, accel, g.n, s, a);
#pragma unroll
        for (int c = 0; c < 3; c++) j[c] = fma(C(0.5) * m.rho, a[c], j[c]);
    }
    if (rho) rho[s] = (OUT)((double)k.rho_ref + (double)m.drho);
    if (u) {
        u[s] = (OUT)(j[0] / m.rho);
        u[(size_t)g.n + s] = (OUT)(j[1] / m.rho);
        u[2 * (size_t)g.n + s] = (OUT)(j[2] / m.rho);
    }
    if (T) T[s] = (OUT)(T_ref + (double)site_T(Tf, Tconst, s));
}

// ---- state codec ------------------------------------------------------------------------------
template <int S>
__global__ void __launch_bounds__(BLOCK)
k_encode_state(const double *__restrict__ Fin, const double *__restrict__ Bin, Geo g, Codec cd,
               typename Storage<S>::T *__restrict__ F, typename Storage<S>::T *__restrict__ B,
               unsigned *__restrict__ flag) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    const size_t n = g.n;
    unsigned sat = 0;
#pragma unroll
    for (int i = 0; i < Q; i++) Storage<S>::store(F, (size_t)i * n + s, i, (C)(Fin[(size_t)i * n + s] - cd.ref[i]), cd, sat);
#pragma unroll
    for (int c = 0; c < NB; c++)
        Storage<S>::store(B, (size_t)c * n + s, Q + c, (C)(Bin[(size_t)c * n + s] - cd.ref[Q + c]), cd, sat);
    if (sat) *flag = 1u;
}

template <int S, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_decode_state(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
               Geo g, Codec cd, typename Storage<S>::C rho_ref, double *__restrict__ Fout, double *__restrict__ Bout) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    C f[Q], bbar[NB];
    PopMoments<C> m;
    load_site<S, GATHERED>(F, B, g.n, nb, s, cd, rho_ref, f, bbar, m, wall_bits(g, z));
    if (Fout) {
#pragma unroll
        for (int i = 0; i < Q; i++) Fout[(size_t)i * g.n + s] = cd.ref[i] + (double)f[i];
    }
    if (Bout) {
#pragma unroll
        for (int c = 0; c < NB; c++) Bout[(size_t)c * g.n + s] = cd.ref[Q + c] + (double)bbar[c];
    }
}

// Element-wise decode of the stored representation (no gather).
template <int S>
__global__ void __launch_bounds__(BLOCK)
k_decode_stored(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B, Geo g,
                Codec cd, double *__restrict__ Fout, double *__restrict__ Bout) {
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    const size_t n = g.n;
    if (Fout) {
#pragma unroll
        for (int i = 0; i < Q; i++) Fout[(size_t)i * n + s] = cd.ref[i] + (double)Storage<S>::load(F, (size_t)i * n + s, i, cd);
    }
    if (Bout) {
#pragma unroll
        for (int c = 0; c < NB; c++)
            Bout[(size_t)c * n + s] = cd.ref[Q + c] + (double)Storage<S>::load(B, (size_t)c * n + s, Q + c, cd);
    }
}

// ---- deterministic block reductions in double ------------------------------------------------
// Each block writes K partial results; a one-block second pass folds them in a fixed order.
constexpr int RED_MAX_BLOCKS = 1024;
constexpr int RED_K = 32;

template <int K, bool MAX>
__device__ __forceinline__ void block_reduce_store(double v[K], double *__restrict__ partial) {
    __shared__ double sh[BLOCK / 64][K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; k++) {
        double a = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double b = __shfl_down(a, off, 64);
            a = MAX ? fmax(a, b) : a + b;
        }
        if (lane == 0) sh[wave][k] = a;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double a = sh[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < BLOCK / 64; w++) a = MAX ? fmax(a, sh[w][threadIdx.x]) : a + sh[w][threadIdx.x];
        partial[(size_t)blockIdx.x * RED_K + threadIdx.x] = a;
    }
}

template <bool MAX>
__global__ void __launch_bounds__(BLOCK) k_reduce_final(const double *__restrict__ partial, int nblocks, int K,
                                                        double *__restrict__ out) {
    __shared__ double sh[BLOCK];
    for (int k = 0; k < K; k++) {
        double a = MAX ? -INFINITY : 0.0;
        for (int b = threadIdx.x; b < nblocks; b += BLOCK) {
            const double v = partial[(size_t)b * RED_K + k];
            a = MAX ? fmax(a, v) : a + v;
        }
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] = MAX ? fmax(sh[threadIdx.x], sh[threadIdx.x + w]) : sh[threadIdx.x] + sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = sh[0];
        __syncthreads();
    }
}

// mass, momentum, energy (K = 5)
template <int S, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_invariants(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B, Geo g,
             Codec cd, typename Storage<S>::C rho_ref, double theta_ref, double *__restrict__ partial) {
    using C = typename Storage<S>::C;
    double v[5] = {0, 0, 0, 0, 0};
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < g.n; s += gridDim.x * BLOCK) {
        int x, y, z;
        site_xyz(s, g, x, y, z);
        const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
        C f[Q], bbar[NB];
        PopMoments<C> m;
        load_site<S, GATHERED>(F, B, g.n, nb, s, cd, rho_ref, f, bbar, m, wall_bits(g, z));
        const double rho = (double)rho_ref + (double)m.drho;
        v[0] += rho;
        v[1] += (double)m.jx;
        v[2] += (double)m.jy;
        v[3] += (double)m.jz;
        // sum_i fbar_i |e_i|^2 = rho + P,  tr bbar = tr beta + 3 theta_ref
        v[4] += 0.5 * (rho + (double)m.P +
                       rho * ((double)bbar[0] + (double)bbar[1] + (double)bbar[2] + 3.0 * theta_ref));
    }
    block_reduce_store<5, false>(v, partial);
}

// non-finite sites, rho <= 0 sites, max |u*| (K = 3; counts stored as doubles, max in slot 2)
template <int S, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_health(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B, Geo g,
         Codec cd, typename Storage<S>::C rho_ref, double *__restrict__ partial_sum, double *__restrict__ partial_max) {
    using C = typename Storage<S>::C;
    double cnt[2] = {0, 0};
    double mx[1] = {0};
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < g.n; s += gridDim.x * BLOCK) {
        int x, y, z;
        site_xyz(s, g, x, y, z);
        const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
        C f[Q], bbar[NB];
        PopMoments<C> m;
        load_site<S, GATHERED>(F, B, g.n, nb, s, cd, rho_ref, f, bbar, m, wall_bits(g, z));
        bool finite = true;
#pragma unroll
        for (int i = 0; i < Q; i++) finite = finite && isfinite((double)f[i]);
#pragma unroll
        for (int c = 0; c < NB; c++) finite = finite && isfinite((double)bbar[c]);
        if (!finite) cnt[0] += 1.0;
        if (!(m.rho > C(0))) cnt[1] += 1.0;
        if (finite && m.rho > C(0)) {
            const double ux = (double)m.jx / (double)m.rho, uy = (double)m.jy / (double)m.rho,
                         uz = (double)m.jz / (double)m.rho;
            mx[0] = fmax(mx[0], sqrt(ux * ux + uy * uy + uz * uz));
        }
    }
    block_reduce_store<2, false>(cnt, partial_sum);
    __syncthreads();
    block_reduce_store<1, true>(mx, partial_max);
}

// Largest |value - ref_k| per field k of the initial equilibrium (deviation codec scales), and
// a count of invalid inputs (rho <= 0 or any non-finite input) in slot 25.
template <typename IN>
__global__ void __launch_bounds__(BLOCK)
k_absmax_fields(const IN *__restrict__ rho, const IN *__restrict__ u, const IN *__restrict__ T, Geo g,
                double rho_ref, double T_ref, double *__restrict__ partial) {
    double v[NFIELD + 1];
#pragma unroll
    for (int k = 0; k <= NFIELD; k++) v[k] = 0.0;
    const size_t n = g.n;
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < g.n; s += gridDim.x * BLOCK) {
        const double r = rho[s], ux = u[s], uy = u[n + s], uz = u[2 * n + s], t = T[s];
        const bool ok = r > 0.0 && isfinite(r) && isfinite(ux) && isfinite(uy) && isfinite(uz) && isfinite(t);
        if (!ok) {
            v[NFIELD] = 1.0;
            continue;
        }
        double f[Q], b[NB];
        equilibrium_dev(r - rho_ref, r, ux, uy, uz, f);
        variance_eq_dev(ux, uy, uz, t - T_ref, b);
#pragma unroll
        for (int i = 0; i < Q; i++) v[i] = fmax(v[i], fabs(f[i]));
#pragma unroll
        for (int c = 0; c < NB; c++) v[Q + c] = fmax(v[Q + c], fabs(b[c]));
    }
    block_reduce_store<NFIELD + 1, true>(v, partial);
}

// Same for a given double state (set_state); slot 25 counts non-finite values.  (A template so
// that every translation unit including this header may instantiate it.)
template <int UNUSED = 0>
__global__ void __launch_bounds__(BLOCK)
k_absmax_state(const double *__restrict__ F, const double *__restrict__ B, Geo g, Codec cd, double *__restrict__ partial) {
    double v[NFIELD + 1];
#pragma unroll
    for (int k = 0; k <= NFIELD; k++) v[k] = 0.0;
    const size_t n = g.n;
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < g.n; s += gridDim.x * BLOCK) {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            const double a = F[(size_t)i * n + s];
            if (!isfinite(a)) v[NFIELD] = 1.0;
            else v[i] = fmax(v[i], fabs(a - cd.ref[i]));
        }
#pragma unroll
        for (int c = 0; c < NB; c++) {
            const double a = B[(size_t)c * n + s];
            if (!isfinite(a)) v[NFIELD] = 1.0;
            else v[Q + c] = fmax(v[Q + c], fabs(a - cd.ref[Q + c]));
        }
    }
    block_reduce_store<NFIELD + 1, true>(v, partial);
}

}  // namespace lbm
