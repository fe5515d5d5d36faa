// lbm_proj.hpp -- projected lattices: the D3Q19 step (Sec. II C) for flows that do not vary along
// z (D = 2, a D2Q9 lattice of nx x ny x 1 sites) or along y and z (D = 1, D1Q3, nx x 1 x 1), held
// as sums over the classes of populations that share their in-plane velocity.
//
// Why this is exact.  On such a lattice the populations of one class stream to the same site and
// the step's per-site update is linear in each population, with feq_i, Phi_i and the relaxation
// targets depending only on moments: rho, j, the in-plane variance, the forcing moments and (the
// energy-conserving mode) the trace of the second moment.  So the class sums
//     F_c = sum_{i in c} fbar_i  and, for the temperature closure,  G_c = sum_{i in c} |e_i,t|^2 fbar_i
// (e_t: the transverse part of e_i) evolve on their own, together with the in-plane components of
// bbar and (energy-conserving mode) the trace of its transverse block.  Transverse velocities stay
// zero and the transverse forcing moments vanish, as the lattice has no transverse gradient.
//
// Implementation.  A site's class sums are expanded into a canonical D3Q19 site -- the transverse
// members of class c carry deviations proportional to their weights, alpha_c w_i with
// alpha_c = dG_c / sum_{i in c} w_i |e_i,t|^2, the in-plane member the rest -- on which the D3Q19
// per-site arithmetic (predictor_sources, collide) runs unchanged; the result is summed back into
// classes.  The split cannot change the sums (the update is linear per population and reads
// moments the split preserves).  The gradient is the D3Q19 stencil restricted to the plane (the
// nine in-plane offsets for D = 2, the two x offsets for D = 1), which is what the D3Q19 stencil
// reduces to when the transverse neighbours are the site's own column.
//
// Stored per site (deviations from the references; storage F64, F32, or 16-bit deviation codes:
// BF16 holds the deviation itself, FP16 a power-of-two-scaled deviation per plane):
//   F planes: dF_c for the NC classes, then dG_c for the NG classes with transverse members
//             (energy-conserving mode only)
//   B planes: the in-plane bbar deviations (D = 2: xx yy xy; D = 1: xx), then the transverse trace
//             (energy-conserving mode only; D = 2: zz; D = 1: yy + zz)
//   src     : the in-plane predictor sources (D = 2: R'xx R'yy R'xy u*x u*y; D = 1: R'xx u*x)
// bbar is gathered or scattered exactly as on the D3Q19 lattice.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

template <int D> struct ProjSet;
template <> struct ProjSet<2> {
    static constexpr int NC = 9, NG = 5, NBI = 3, NSP = 5;
    // class of each population: its (e_x, e_y) in the order of populations 0-4 and 7-10
    static constexpr int CLS[Q] = {0, 1, 2, 3, 4, 0, 0, 5, 6, 7, 8, 1, 1, 3, 3, 2, 2, 4, 4};
    static constexpr int CX[NC] = {0, 1, 0, -1, 0, 1, 1, -1, -1};
    static constexpr int CY[NC] = {0, 0, 1, 0, -1, 1, -1, 1, -1};
};
template <> struct ProjSet<1> {
    static constexpr int NC = 3, NG = 3, NBI = 1, NSP = 2;
    static constexpr int CLS[Q] = {0, 1, 0, 2, 0, 0, 0, 1, 1, 2, 2, 1, 1, 2, 2, 0, 0, 0, 0};
    static constexpr int CX[NC] = {0, 1, -1};
    static constexpr int CY[NC] = {0, 0, 0};
};

// Loads and stores of the projected state; f is the plane's codec field (class sum c: c; its G:
// NC + c; variance plane k: Q + k).  BF16 codes hold the deviation itself (their scale is always
// 1), so they read no codec: in the server the codec sits in a descriptor in device memory.
// FP16 codes use the field's power-of-two scale, chosen at lbm_set_fields.
template <int S>
__device__ __forceinline__ typename Storage<S>::C proj_ld(const typename Storage<S>::T *p, size_t i, int f,
                                                          const Codec &cd) {
    if constexpr (S == 3)
        return bf16_bits_to_float(p[i]);
    else if constexpr (S == 2)
        return Storage<2>::load(p, i, f, cd);
    else
        return p[i];
}
template <int S>
__device__ __forceinline__ void proj_st(typename Storage<S>::T *p, size_t i, typename Storage<S>::C v, int f,
                                        const Codec &cd, unsigned &sat) {
    if constexpr (S == 3)
        p[i] = float_to_bf16_bits(v, sat);
    else if constexpr (S == 2)
        Storage<2>::store(p, i, f, v, cd, sat);
    else
        p[i] = v;
}

// A 16-bit code overflowed somewhere in this wavefront: one lane records it.  (A diverging
// lattice overflows at every site and every step until its health check retires it; one store
// per wavefront instead of one atomic per site keeps that from serialising the sweep.)
__device__ __forceinline__ void proj_flag_overflow(unsigned *flag, unsigned sat) {
    const unsigned long long m = __ballot(sat != 0u);
    if (m && __lane_id() == (unsigned)(__ffsll((long long)m) - 1)) *flag = 1u;
}

// |e_i,t|^2, the squared transverse speed of population i
template <int D> constexpr int et2(int i) { return D == 2 ? EZ[i] * EZ[i] : EY[i] * EY[i] + EZ[i] * EZ[i]; }
// sum over class c of w_i, of w_i |e_i,t|^2, and of w_i over its transverse members
template <int D> constexpr double class_w(int c) {
    double s = 0.0;
    for (int i = 0; i < Q; i++)
        if (ProjSet<D>::CLS[i] == c) s += WQ[i];
    return s;
}
template <int D> constexpr double class_gw(int c) {
    double s = 0.0;
    for (int i = 0; i < Q; i++)
        if (ProjSet<D>::CLS[i] == c) s += WQ[i] * et2<D>(i);
    return s;
}
template <int D> constexpr double class_tw(int c) {
    double s = 0.0;
    for (int i = 0; i < Q; i++)
        if (ProjSet<D>::CLS[i] == c && et2<D>(i) > 0) s += WQ[i];
    return s;
}

template <int D, bool TH> struct ProjLayout {
    static constexpr int NF = ProjSet<D>::NC + (TH ? ProjSet<D>::NG : 0);
    static constexpr int NBP = ProjSet<D>::NBI + (TH ? 1 : 0);
};

// Canonical D3Q19 site from class sums (dG = 0 without the energy-conserving mode).
template <int D, bool TH, typename C>
__device__ __forceinline__ void proj_expand(const C dF[ProjSet<D>::NC], const C *dG, const C bred[ProjLayout<D, TH>::NBP],
                                            C d[Q], C beta[NB]) {
    Unroll<0, Q>::run([&](auto I) {
        constexpr int c = ProjSet<D>::CLS[I];
        constexpr double tw = class_tw<D>(c);
        if constexpr (tw == 0.0) {
            d[I] = dF[c];
        } else if constexpr (!TH) {
            d[I] = et2<D>(I) > 0 ? C(0) : dF[c];
        } else {
            constexpr double inv_gw = 1.0 / class_gw<D>(c);
            const C alpha = dG[c] * C(inv_gw);
            if constexpr (et2<D>(I) > 0)
                d[I] = alpha * C(WQ[I]);
            else
                d[I] = dF[c] - alpha * C(tw);
        }
    });
#pragma unroll
    for (int k = 0; k < NB; k++) beta[k] = C(0);
    beta[0] = bred[0];
    if constexpr (D == 2) {
        beta[1] = bred[1];
        beta[3] = bred[2];
        if constexpr (TH) beta[2] = bred[3];
    } else if constexpr (TH) {
        beta[1] = beta[2] = C(0.5) * bred[1];
    }
}

// Class sums of a D3Q19 site.
template <int D, bool TH, typename C>
__device__ __forceinline__ void proj_contract(const C d[Q], const C beta[NB], C dF[ProjSet<D>::NC], C *dG,
                                              C bred[ProjLayout<D, TH>::NBP]) {
#pragma unroll
    for (int c = 0; c < ProjSet<D>::NC; c++) dF[c] = C(0);
    if constexpr (TH) {
#pragma unroll
        for (int c = 0; c < ProjSet<D>::NG; c++) dG[c] = C(0);
    }
    Unroll<0, Q>::run([&](auto I) {
        constexpr int c = ProjSet<D>::CLS[I];
        dF[c] += d[I];
        if constexpr (TH && et2<D>(I) > 0) dG[c] += C(et2<D>(I)) * d[I];
    });
    bred[0] = beta[0];
    if constexpr (D == 2) {
        bred[1] = beta[1];
        bred[2] = beta[3];
        if constexpr (TH) bred[3] = beta[2];
    } else if constexpr (TH) {
        bred[1] = beta[1] + beta[2];
    }
}

// Neighbour of a site at in-plane offset (cx, cy).
__device__ __forceinline__ int proj_at(const Nbr &nb, int cx, int cy) { return nb.at(cx, cy, 0); }

// Load a site's class sums and its gathered bbar (Eq. 66 over classes: every member of class c
// arrives from x - c), expanded.
template <int S, int D, bool TH, bool GATHERED>
__device__ __forceinline__ void proj_load(const typename Storage<S>::T *__restrict__ F,
                                          const typename Storage<S>::T *__restrict__ B, size_t n, const Nbr &nb, int s,
                                          const Codec &cd, typename Storage<S>::C rho_ref, typename Storage<S>::C d[Q],
                                          typename Storage<S>::C beta[NB], PopMoments<typename Storage<S>::C> &m) {
    using C = typename Storage<S>::C;
    using PS = ProjSet<D>;
    using PL = ProjLayout<D, TH>;
    C dF[PS::NC], dG[TH ? PS::NG : 1], bred[PL::NBP];
#pragma unroll
    for (int c = 0; c < PS::NC; c++) dF[c] = proj_ld<S>(F, (size_t)c * n + s, c, cd);
    if constexpr (TH) {
#pragma unroll
        for (int c = 0; c < PS::NG; c++) dG[c] = proj_ld<S>(F, (size_t)(PS::NC + c) * n + s, PS::NC + c, cd);
    }
    if constexpr (GATHERED) {
#pragma unroll
        for (int k = 0; k < PL::NBP; k++) bred[k] = proj_ld<S>(B, (size_t)k * n + s, Q + k, cd);
    } else {
        C acc[PL::NBP], rho = rho_ref;
#pragma unroll
        for (int k = 0; k < PL::NBP; k++) acc[k] = C(0);
        Unroll<0, PS::NC>::run([&](auto c) {
            const int up = proj_at(nb, -PS::CX[c], -PS::CY[c]);
            const C wgt = fma(C(class_w<D>(c)), rho_ref, dF[c]);
            rho += dF[c];
#pragma unroll
            for (int k = 0; k < PL::NBP; k++) acc[k] += wgt * proj_ld<S>(B, (size_t)k * n + up, Q + k, cd);
        });
        const C inv = recip(rho);
#pragma unroll
        for (int k = 0; k < PL::NBP; k++) bred[k] = acc[k] * inv;
    }
    proj_expand<D, TH>(dF, dG, bred, d, beta);
    m = pop_moments(d, rho_ref);
}

// In-plane gradient forcing moments from the reduced source planes.
template <int D, typename C>
__device__ __forceinline__ void proj_gradient(const C *__restrict__ src, size_t n, const Nbr &nb, C K, C F[3], C S[6]) {
    GradAcc<C> acc;
    grad_init(acc);
    auto add = [&](auto I) {
        const int at = proj_at(nb, EX[I], EY[I]);
        C sv[NSRC];
#pragma unroll
        for (int c = 0; c < NSRC; c++) sv[c] = C(0);
        if constexpr (D == 2) {
            sv[0] = src[at];
            sv[1] = src[n + at];
            sv[3] = src[2 * n + at];
            sv[6] = src[3 * n + at];
            sv[7] = src[4 * n + at];
        } else {
            sv[0] = src[at];
            sv[6] = src[n + at];
        }
        grad_add<C, decltype(I)::value>(acc, sv, K);
    };
    add(std::integral_constant<int, 1>{});
    add(std::integral_constant<int, 3>{});
    if constexpr (D == 2) {
        add(std::integral_constant<int, 2>{});
        add(std::integral_constant<int, 4>{});
        add(std::integral_constant<int, 7>{});
        add(std::integral_constant<int, 8>{});
        add(std::integral_constant<int, 9>{});
        add(std::integral_constant<int, 10>{});
        grad_finish_thin(acc, F, S);
    } else {
        // each x face also stands for the four edges reading the same site (1/18 + 4/36 = 1/6);
        // their transverse parts cancel
#pragma unroll
        for (int c = 0; c < 3; c++) F[c] = C(0);
#pragma unroll
        for (int c = 0; c < 6; c++) S[c] = C(0);
        F[0] = -C(0.5) * acc.fF[0];
        S[0] = -acc.fS[0];
    }
}

// ---- pass A: predictor sources -------------------------------------------------------------------
template <int S, int D, bool TH, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_proj_predict(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
               typename Storage<S>::C *__restrict__ src, const typename Storage<S>::C *__restrict__ Tf,
               typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    C d[Q], beta[NB];
    PopMoments<C> m;
    proj_load<S, D, TH, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, d, beta, m);
    C o[NSRC];
    predictor_sources(m, beta, site_T(Tf, Tconst, s), k, o);
    const size_t n = g.n;
    src[s] = o[0];
    if constexpr (D == 2) {
        src[n + s] = o[1];
        src[2 * n + s] = o[3];
        src[3 * n + s] = o[6];
        src[4 * n + s] = o[7];
    } else {
        src[n + s] = o[6];
    }
}

// ---- pass B: gradient, collision, push by class ----------------------------------------------------
template <int S, int D, bool TH, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_proj_collide(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
               const typename Storage<S>::C *__restrict__ src, typename Storage<S>::T *__restrict__ Fo,
               typename Storage<S>::T *__restrict__ Bo, const typename Storage<S>::C *__restrict__ Tf,
               typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd,
               unsigned *__restrict__ flag) {
    using C = typename Storage<S>::C;
    using PS = ProjSet<D>;
    using PL = ProjLayout<D, TH>;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    C d[Q], beta[NB];
    PopMoments<C> m;
    proj_load<S, D, TH, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, d, beta, m);
    C Fv[3], Sv[6];
    proj_gradient<D>(src, g.n, nb, k.K, Fv, Sv);
    collide(d, beta, m, Fv, Sv, site_T(Tf, Tconst, s), k);
    C dF[PS::NC], dG[TH ? PS::NG : 1], bred[PL::NBP];
    proj_contract<D, TH>(d, beta, dF, dG, bred);
    unsigned sat = 0;
    Unroll<0, PS::NC>::run([&](auto c) {
        const int to = proj_at(nb, PS::CX[c], PS::CY[c]);
        proj_st<S>(Fo, (size_t)c * g.n + to, dF[c], c, cd, sat);
        if constexpr (TH && c < PS::NG) proj_st<S>(Fo, (size_t)(PS::NC + c) * g.n + to, dG[c], PS::NC + c, cd, sat);
    });
#pragma unroll
    for (int kk = 0; kk < PL::NBP; kk++) proj_st<S>(Bo, (size_t)kk * g.n + s, bred[kk], Q + kk, cd, sat);
    if constexpr (S >= 2) proj_flag_overflow(flag, sat);
}

// ---- one-launch step: sources of a tile and its one-site halo in LDS -------------------------------
// A work-group owns a TX x TY tile (D = 2: 128 x 8; D = 1: 256 x 1).  Phase 1 computes the in-plane
// predictor sources of the tile and its one-site ring (periodic wrap) into LDS; phase 2 takes each
// owned site's gradient from LDS, collides it and pushes its class sums.  The ring's sources are
// recomputed by the neighbouring tiles (1.27x the source work for D = 2), and the reads they need
// mostly hit in L2; the state goes through HBM once each way.
#ifndef PROJ2_TX
#define PROJ2_TX 128
#endif
#ifndef PROJ2_TY
#define PROJ2_TY 8
#endif
template <int D, int TX_, int TY_> struct ProjTileT {
    static constexpr int TX = TX_, TY = TY_, HY = D == 2 ? 1 : 0;
    static constexpr int NT = TX * TY, LX = TX + 2, LY = TY + 2 * HY, HN = LX * LY;
    static constexpr int NRING = HN - NT;  // D = 2: two rows of LX and two columns of TY
    // staged bbar* of the previous step: the source grid plus one more ring
    static constexpr int BX = LX + 2, BY = LY + 2 * HY, BN = BX * BY;
};
// the one-launch step's tiles; the server's persistent kernel takes the same ones, so that a
// served lattice steps bitwise as it would alone
template <int D> using ProjTile = ProjTileT<D, D == 2 ? PROJ2_TX : 256, D == 2 ? PROJ2_TY : 1>;

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// LDS slot of ring site r: the top and bottom rows, then the left and right columns (D = 2), or
// the two ends of the row (D = 1).
template <int D, typename TL> __device__ __forceinline__ int proj_ring_slot(int r) {
    if constexpr (D == 1) {
        return r == 0 ? 0 : TL::LX - 1;
    } else {
        if (r < TL::LX) return r;
        if (r < 2 * TL::LX) return (TL::LY - 1) * TL::LX + (r - TL::LX);
        r -= 2 * TL::LX;
        const int j = 1 + (r >> 1);
        return j * TL::LX + ((r & 1) ? TL::LX - 1 : 0);
    }
}

// Sources of the site held in LDS slot l of the tile at (x0, y0), periodic (a lattice smaller
// than the tile wraps as often as needed), into lsrc (NSP planes of TL::HN).  STAGED: its gather
// reads the staged bbar* (lb, NBP planes of TL::BN).
template <int S, int D, bool TH, bool GATHERED, bool STAGED, typename TL>
__device__ __forceinline__ void proj_tile_site(const typename Storage<S>::T *__restrict__ F,
                                               const typename Storage<S>::T *__restrict__ B,
                                               const typename Storage<S>::C *__restrict__ Tf,
                                               typename Storage<S>::C Tconst, const Geo &g,
                                               const StepConst<typename Storage<S>::C> &k, const Codec &cd, int x0,
                                               int y0, int l, typename Storage<S>::C *lsrc,
                                               const typename Storage<S>::C *lb, typename Storage<S>::C d[Q],
                                               typename Storage<S>::C beta[NB], PopMoments<typename Storage<S>::C> &m) {
    using C = typename Storage<S>::C;
    using PS = ProjSet<D>;
    using PL = ProjLayout<D, TH>;
    const int i = l % TL::LX, j = l / TL::LX;
    const int x = wrap_mod(x0 - 1 + i, g.nx), y = wrap_mod(y0 - TL::HY + j, g.ny);
    const int s = y * g.nx + x;
    const Nbr nb = make_nbr(x, y, 0, g.nx, g.ny, 1);
    if constexpr (!STAGED) {
        proj_load<S, D, TH, GATHERED>(F, B, (size_t)g.n, nb, s, cd, k.rho_ref, d, beta, m);
    } else {
        // class sums from HBM, the gather (Eq. 66 over classes) from the staged bbar*
        const size_t n = g.n;
        C dF[PS::NC], dG[TH ? PS::NG : 1], bred[PL::NBP], acc[PL::NBP], rho = k.rho_ref;
#pragma unroll
        for (int c = 0; c < PS::NC; c++) dF[c] = proj_ld<S>(F, (size_t)c * n + s, c, cd);
        if constexpr (TH) {
#pragma unroll
            for (int c = 0; c < PS::NG; c++) dG[c] = proj_ld<S>(F, (size_t)(PS::NC + c) * n + s, PS::NC + c, cd);
        }
#pragma unroll
        for (int kk = 0; kk < PL::NBP; kk++) acc[kk] = C(0);
        const int bl = (j + TL::HY) * TL::BX + i + 1;  // this site in the staging grid
        Unroll<0, PS::NC>::run([&](auto c) {
            const int up = bl - PS::CY[c] * TL::BX - PS::CX[c];
            const C wgt = fma(C(class_w<D>(c)), k.rho_ref, dF[c]);
            rho += dF[c];
#pragma unroll
            for (int kk = 0; kk < PL::NBP; kk++) acc[kk] += wgt * lb[kk * TL::BN + up];
        });
        const C inv = recip(rho);
#pragma unroll
        for (int kk = 0; kk < PL::NBP; kk++) bred[kk] = acc[kk] * inv;
        proj_expand<D, TH>(dF, dG, bred, d, beta);
        m = pop_moments(d, k.rho_ref);
    }
    C o[NSRC];
    predictor_sources(m, beta, site_T(Tf, Tconst, s), k, o);
    lsrc[l] = o[0];
    if constexpr (D == 2) {
        lsrc[TL::HN + l] = o[1];
        lsrc[2 * TL::HN + l] = o[3];
        lsrc[3 * TL::HN + l] = o[6];
        lsrc[4 * TL::HN + l] = o[7];
    } else {
        lsrc[TL::HN + l] = o[6];
    }
}

// One step of tile (bx, by) of a projected lattice, by a work-group of TL::NT threads.  Phase 0
// (D2Q9, scattered state) stages the previous step's bbar* of the source grid plus one ring;
// phase 1 evaluates the sources of the owned slot (its state stays in registers) and of the ring
// into LDS; phase 2 takes each owned site's gradient from LDS, collides it and pushes its class
// sums.  lsrc: NSP x TL::HN, lb: NBP x TL::BN values of LDS (lb unused without staging).  Every
// thread returns (none leaves early), so a caller may synchronise after it.
template <int S, int D, bool TH, bool GATHERED, typename TL>
__device__ __forceinline__ void proj_tile_step(const typename Storage<S>::T *__restrict__ F,
                                               const typename Storage<S>::T *__restrict__ B,
                                               typename Storage<S>::T *__restrict__ Fo,
                                               typename Storage<S>::T *__restrict__ Bo,
                                               const typename Storage<S>::C *__restrict__ Tf,
                                               typename Storage<S>::C Tconst, const Geo &g,
                                               const StepConst<typename Storage<S>::C> &k, const Codec &cd, int bx,
                                               int by, typename Storage<S>::C *lsrc, typename Storage<S>::C *lb,
                                               unsigned *__restrict__ flag) {
    using C = typename Storage<S>::C;
    using PS = ProjSet<D>;
    using PL = ProjLayout<D, TH>;
    // D2Q9 stages the previous step's bbar* for the gathers (nine upstream classes); D1Q3, with
    // three, gathers from L2 directly
    constexpr bool STAGED = !GATHERED && D == 2;
    const int x0 = bx * TL::TX, y0 = by * TL::TY;
    const size_t n = g.n;
    const int tx = threadIdx.x % TL::TX, ty = threadIdx.x / TL::TX;
    if constexpr (STAGED) {
        for (int l = threadIdx.x; l < TL::BN; l += TL::NT) {
            const int x = wrap_mod(x0 - 2 + l % TL::BX, g.nx), y = wrap_mod(y0 - 2 * TL::HY + l / TL::BX, g.ny);
            const int s = y * g.nx + x;
#pragma unroll
            for (int kk = 0; kk < PL::NBP; kk++) lb[kk * TL::BN + l] = proj_ld<S>(B, (size_t)kk * n + s, Q + kk, cd);
        }
        __syncthreads();
    }
    C d[Q], beta[NB];
    PopMoments<C> m;
    proj_tile_site<S, D, TH, GATHERED, STAGED, TL>(F, B, Tf, Tconst, g, k, cd, x0, y0, (ty + TL::HY) * TL::LX + tx + 1,
                                                   lsrc, lb, d, beta, m);
    for (int r = threadIdx.x; r < TL::NRING; r += TL::NT) {
        C d2[Q], beta2[NB];
        PopMoments<C> m2;
        proj_tile_site<S, D, TH, GATHERED, STAGED, TL>(F, B, Tf, Tconst, g, k, cd, x0, y0, proj_ring_slot<D, TL>(r),
                                                       lsrc, lb, d2, beta2, m2);
    }
    __syncthreads();
    const int x = x0 + tx, y = y0 + ty;
    if (x < g.nx && y < g.ny) {
        const int s = y * g.nx + x;
        const Nbr nb = make_nbr(x, y, 0, g.nx, g.ny, 1);
        GradAcc<C> acc;
        grad_init(acc);
        auto add = [&](auto I) {
            constexpr int ex = EX[decltype(I)::value], ey = EY[decltype(I)::value];
            const int l = (ty + TL::HY + ey) * TL::LX + (tx + 1 + ex);
            C sv[NSRC];
#pragma unroll
            for (int c = 0; c < NSRC; c++) sv[c] = C(0);
            sv[0] = lsrc[l];
            if constexpr (D == 2) {
                sv[1] = lsrc[TL::HN + l];
                sv[3] = lsrc[2 * TL::HN + l];
                sv[6] = lsrc[3 * TL::HN + l];
                sv[7] = lsrc[4 * TL::HN + l];
            } else {
                sv[6] = lsrc[TL::HN + l];
            }
            grad_add<C, decltype(I)::value>(acc, sv, k.K);
        };
        C Fv[3], Sv[6];
        add(std::integral_constant<int, 1>{});
        add(std::integral_constant<int, 3>{});
        if constexpr (D == 2) {
            add(std::integral_constant<int, 2>{});
            add(std::integral_constant<int, 4>{});
            add(std::integral_constant<int, 7>{});
            add(std::integral_constant<int, 8>{});
            add(std::integral_constant<int, 9>{});
            add(std::integral_constant<int, 10>{});
            grad_finish_thin(acc, Fv, Sv);
        } else {
#pragma unroll
            for (int c = 0; c < 3; c++) Fv[c] = C(0);
#pragma unroll
            for (int c = 0; c < 6; c++) Sv[c] = C(0);
            Fv[0] = -C(0.5) * acc.fF[0];
            Sv[0] = -acc.fS[0];
        }
        collide(d, beta, m, Fv, Sv, site_T(Tf, Tconst, s), k);
        C dF[PS::NC], dG[TH ? PS::NG : 1], bred[PL::NBP];
        proj_contract<D, TH>(d, beta, dF, dG, bred);
        unsigned sat = 0;
        Unroll<0, PS::NC>::run([&](auto c) {
            const int to = proj_at(nb, PS::CX[c], PS::CY[c]);
            proj_st<S>(Fo, (size_t)c * n + to, dF[c], c, cd, sat);
            if constexpr (TH && c < PS::NG) proj_st<S>(Fo, (size_t)(PS::NC + c) * n + to, dG[c], PS::NC + c, cd, sat);
        });
#pragma unroll
        for (int kk = 0; kk < PL::NBP; kk++) proj_st<S>(Bo, (size_t)kk * n + s, bred[kk], Q + kk, cd, sat);
        if constexpr (S >= 2) proj_flag_overflow(flag, sat);
    }
}

template <int S, int D, bool TH, bool GATHERED>
__global__ void __launch_bounds__(ProjTile<D>::NT)
k_proj_fused(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
             typename Storage<S>::T *__restrict__ Fo, typename Storage<S>::T *__restrict__ Bo,
             const typename Storage<S>::C *__restrict__ Tf, typename Storage<S>::C Tconst, Geo g,
             StepConst<typename Storage<S>::C> k, Codec cd, unsigned *__restrict__ flag) {
    using C = typename Storage<S>::C;
    using TL = ProjTile<D>;
    constexpr bool STAGED = !GATHERED && D == 2;
    __shared__ C lsrc[ProjSet<D>::NSP * TL::HN];
    __shared__ C lb[STAGED ? ProjLayout<D, TH>::NBP * TL::BN : 1];
    proj_tile_step<S, D, TH, GATHERED, TL>(F, B, Fo, Bo, Tf, Tconst, g, k, cd, blockIdx.x, blockIdx.y, lsrc, lb, flag);
}

// ---- health of a projected lattice: non-finite sites, rho <= 0 sites, max |u*| -----------------
template <int S, int D, bool TH, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_proj_health(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B, Geo g,
              Codec cd, typename Storage<S>::C rho_ref, double *__restrict__ partial_sum,
              double *__restrict__ partial_max) {
    using C = typename Storage<S>::C;
    double cnt[2] = {0, 0};
    double mx[1] = {0};
    for (int s = blockIdx.x * BLOCK + threadIdx.x; s < g.n; s += gridDim.x * BLOCK) {
        int x, y, z;
        site_xyz(s, g, x, y, z);
        const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
        C d[Q], beta[NB];
        PopMoments<C> m;
        proj_load<S, D, TH, GATHERED>(F, B, (size_t)g.n, nb, s, cd, rho_ref, d, beta, m);
        bool finite = true;
#pragma unroll
        for (int i = 0; i < Q; i++) finite = finite && isfinite((double)d[i]);
#pragma unroll
        for (int c = 0; c < NB; c++) finite = finite && isfinite((double)beta[c]);
        if (!finite) cnt[0] += 1.0;
        if (!(m.rho > C(0))) cnt[1] += 1.0;
        if (finite && m.rho > C(0)) {
            const double ux = (double)m.jx / (double)m.rho, uy = (double)m.jy / (double)m.rho;
            mx[0] = fmax(mx[0], sqrt(ux * ux + uy * uy));
        }
    }
    block_reduce_store<2, false>(cnt, partial_sum);
    __syncthreads();
    block_reduce_store<1, true>(mx, partial_max);
}

// ---- readout of corrected moments (after k_proj_predict on the same state) ----------------------
template <int S, int D, bool TH, bool GATHERED, typename OUT>
__global__ void __launch_bounds__(BLOCK)
k_proj_readout(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
               const typename Storage<S>::C *__restrict__ src, const typename Storage<S>::C *__restrict__ Tf,
               typename Storage<S>::C Tconst, Geo g, StepConst<typename Storage<S>::C> k, Codec cd, double T_ref,
               OUT *__restrict__ rho, OUT *__restrict__ u, OUT *__restrict__ T) {
    using C = typename Storage<S>::C;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    C d[Q], beta[NB];
    PopMoments<C> m;
    proj_load<S, D, TH, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, d, beta, m);
    C Fv[3], Sv[6];
    proj_gradient<D>(src, g.n, nb, k.K, Fv, Sv);
    C uc[3], Tc;
    collide(d, beta, m, Fv, Sv, site_T(Tf, Tconst, s), k, uc, &Tc);
    if (rho) rho[s] = (OUT)((double)k.rho_ref + (double)m.drho);
    if (u) {
        u[s] = (OUT)uc[0];
        u[(size_t)g.n + s] = (OUT)uc[1];
        u[2 * (size_t)g.n + s] = (OUT)uc[2];
    }
    if (T) T[s] = (OUT)(T_ref + (double)Tc);
}

// ---- initialisation: class sums of feq(rho, u) and the reduced beq(u, T) (gathered) -------------
// Transverse velocity components must be zero; a site with one sets bit 2 of *flag (bit 1: a
// 16-bit code overflowed).
template <int S, int D, bool TH, typename IN>
__global__ void __launch_bounds__(BLOCK)
k_proj_init(const IN *__restrict__ rho, const IN *__restrict__ u, const IN *__restrict__ T, Geo g, double rho_ref,
            double T_ref, typename Storage<S>::T *__restrict__ F, typename Storage<S>::T *__restrict__ B,
            typename Storage<S>::C *__restrict__ Tf, unsigned *__restrict__ flag, Codec cd) {
    using C = typename Storage<S>::C;
    using PS = ProjSet<D>;
    using PL = ProjLayout<D, TH>;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    const size_t n = g.n;
    const double r = (double)rho[s], ux = (double)u[s], uy = (double)u[n + s], uz = (double)u[2 * n + s];
    if (uz != 0.0 || (D == 1 && uy != 0.0)) atomicOr(flag, 2u);
    const double theta = (double)T[s] - T_ref;
    double f[Q], b[NB];
    equilibrium_dev(r - rho_ref, r, ux, D == 2 ? uy : 0.0, 0.0, f);
    variance_eq_dev(ux, D == 2 ? uy : 0.0, 0.0, theta, b);
    double dF[PS::NC], dG[TH ? PS::NG : 1], bred[PL::NBP];
    proj_contract<D, TH>(f, b, dF, dG, bred);
    unsigned sat = 0;
#pragma unroll
    for (int c = 0; c < PS::NC; c++) proj_st<S>(F, (size_t)c * n + s, (C)dF[c], c, cd, sat);
    if constexpr (TH) {
#pragma unroll
        for (int c = 0; c < PS::NG; c++) proj_st<S>(F, (size_t)(PS::NC + c) * n + s, (C)dG[c], PS::NC + c, cd, sat);
    }
#pragma unroll
    for (int kk = 0; kk < PL::NBP; kk++) proj_st<S>(B, (size_t)kk * n + s, (C)bred[kk], Q + kk, cd, sat);
    if (Tf) Tf[s] = (C)theta;
    if (sat) atomicOr(flag, 1u);
}

// ---- decoded state in FP64: full class sums and gathered reduced bbar ----------------------------
template <int S, int D, bool TH, bool GATHERED>
__global__ void __launch_bounds__(BLOCK)
k_proj_decode(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B, Geo g,
              Codec cd, typename Storage<S>::C rho_ref, double theta_ref, double *__restrict__ Fout,
              double *__restrict__ Bout) {
    using C = typename Storage<S>::C;
    using PS = ProjSet<D>;
    using PL = ProjLayout<D, TH>;
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= g.n) return;
    int x, y, z;
    site_xyz(s, g, x, y, z);
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    C d[Q], beta[NB];
    PopMoments<C> m;
    proj_load<S, D, TH, GATHERED>(F, B, g.n, nb, s, cd, rho_ref, d, beta, m);
    C dF[PS::NC], dG[TH ? PS::NG : 1], bred[PL::NBP];
    proj_contract<D, TH>(d, beta, dF, dG, bred);
    const size_t n = g.n;
    if (Fout) {
        Unroll<0, PS::NC>::run([&](auto c) {
            Fout[(size_t)c * n + s] = class_w<D>(c) * (double)rho_ref + (double)dF[c];
            if constexpr (TH && c < PS::NG)
                Fout[(size_t)(PS::NC + c) * n + s] = class_gw<D>(c) * (double)rho_ref + (double)dG[c];
        });
    }
    if (Bout) {
        // references: theta_ref on each in-plane diagonal, 0 off the diagonal; the transverse
        // trace holds 3 - D diagonal components
        Bout[s] = theta_ref + (double)bred[0];
        if constexpr (D == 2) {
            Bout[n + s] = theta_ref + (double)bred[1];
            Bout[2 * n + s] = (double)bred[2];
            if constexpr (TH) Bout[3 * n + s] = theta_ref + (double)bred[3];
        } else if constexpr (TH) {
            Bout[n + s] = 2.0 * theta_ref + (double)bred[1];
        }
    }
}

}  // namespace lbm
