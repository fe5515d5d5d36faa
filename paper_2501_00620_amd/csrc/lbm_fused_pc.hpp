// lbm_fused_pc.hpp -- the fused sweep with producer and consumer waves (one launch per step).
//
// The same step as k_fused (Sec. II C: predictor sources, isotropic gradients, collision and the
// stream with the bbar gather of Eq. 66), organised for occupancy.  A work-group of 1024 threads
// owns a 64 x 8 xy tile and marches through a chunk of z planes with two kinds of waves:
//   producers (waves 0-7, one tile site per thread, ring sites on the first threads) stage the
//     post-collision bbar* of plane p+2 in LDS and evaluate the predictor sources (rho b and u*,
//     Eqs. 59-61 with Eq. 68) of plane p over the tile and its one-site ring, gathering bbar with
//     the arriving populations (Eq. 66); they hand each tile site's gathered bbar on through LDS;
//   consumers (waves 8-15, one tile site per thread) take the isotropic gradient of the sources
//     plane by plane: each source plane q adds its 3 x 3 in-plane neighbourhood to the gradient
//     sums of the sites in planes q-1, q and q+1, so only the newest source plane lives in LDS and
//     the sums of plane q-1 are complete once plane q is in.  They then collide plane q-1 and push
//     it out.
// Both kinds run in the same iteration, separated by one barrier per plane: producers of plane p
// next to consumers of plane p-2.  Each kind keeps about half of the single-role sweep's live
// values (108-114 VGPRs per lane, no spills), so every SIMD holds four waves (two of each kind)
// to cover each other's LDS and memory waits.
//
// Walls (half-way bounce-back at z = -1/2 and nz - 1/2, Sec. III A and C): the sweep updates the
// interior planes 1 .. nz-2 only, whose gather, gradient and push cross no wall.  The sources of
// the two wall-adjacent planes, which the gradients of planes 1 and nz-2 take, come from the
// source planes the two-pass predictor wrote for the wall kernel (the same sources, gathered with
// the bounce-back rule), read through descriptors bounded to one plane; the wall kernel steps
// planes 0 and nz-1 itself.
// LDS: four bbar* staging planes (tile plus two rings), two source planes (tile plus one ring),
// and three hand-off planes of gathered bbar: 162,720 B of the 163,840 B a CU has.
// The consumers read the populations of the plane they collide a second time from global memory
// (the producers read them three iterations earlier, mostly an L2 hit).
#pragma once

#include "lbm_fused.hpp"

namespace lbm {

// Gradient sums with the face weight folded in: T = 2 (face terms) + (edge terms), so that
// F = -T_F / 12, S_aa = -T_Saa / 6 (the diagonal collects v_a u_a once) and S_ab = -T_Sab / 12,
// the same moments as grad_finish (weights 1/18 and 1/36 of the isotropic difference).
template <typename C> struct GradT {
    C F[3], S[6];
};

template <typename C> __device__ __forceinline__ void gradt_zero(GradT<C> &a) {
#pragma unroll
    for (int c = 0; c < 3; c++) a.F[c] = C(0);
#pragma unroll
    for (int c = 0; c < 6; c++) a.S[c] = C(0);
}

// Direction I's term for a neighbour with sources s: v = sum_a e_Ia R'_a. and, for the
// second-moment source, w = v + K e_I (the constant rho_ref b_ref when HASK), as grad_add.
template <typename C, int I, bool HASK>
__device__ __forceinline__ void gradt_add(GradT<C> &a, const C s[NSRC], C K) {
    constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
    constexpr bool face = (ex * ex + ey * ey + ez * ez) == 1;
    const C vx = C(ex) * s[0] + C(ey) * s[3] + C(ez) * s[4];
    const C vy = C(ex) * s[3] + C(ey) * s[1] + C(ez) * s[5];
    const C vz = C(ex) * s[4] + C(ey) * s[5] + C(ez) * s[2];
    C wx = vx, wy = vy, wz = vz;
    if constexpr (HASK) {
        wx = vx + C(ex) * K;
        wy = vy + C(ey) * K;
        wz = vz + C(ez) * K;
    }
    if constexpr (face) {  // weight 2 (exact scaling)
        wx = C(2) * wx;
        wy = C(2) * wy;
        wz = C(2) * wz;
        a.F[0] = fma(C(2), vx, a.F[0]);
        a.F[1] = fma(C(2), vy, a.F[1]);
        a.F[2] = fma(C(2), vz, a.F[2]);
    } else {
        a.F[0] += vx;
        a.F[1] += vy;
        a.F[2] += vz;
    }
    const C ux = s[6], uy = s[7], uz = s[8];
    a.S[0] = fma(wx, ux, a.S[0]);
    a.S[1] = fma(wy, uy, a.S[1]);
    a.S[2] = fma(wz, uz, a.S[2]);
    a.S[3] = fma(wx, uy, fma(wy, ux, a.S[3]));
    a.S[4] = fma(wx, uz, fma(wz, ux, a.S[4]));
    a.S[5] = fma(wy, uz, fma(wz, uy, a.S[5]));
}

template <typename C> __device__ __forceinline__ void gradt_finish(const GradT<C> &a, C F[3], C S[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] = -a.F[c] * C(1.0 / 12.0);
#pragma unroll
    for (int c = 0; c < 3; c++) S[c] = -a.S[c] * C(1.0 / 6.0);
#pragma unroll
    for (int c = 3; c < 6; c++) S[c] = -a.S[c] * C(1.0 / 12.0);
}

// The same term as the first one into sums a: it sets them (a sum that starts a plane needs no
// zeroing).
template <typename C, int I, bool HASK>
__device__ __forceinline__ void gradt_set(GradT<C> &a, const C s[NSRC], C K) {
    gradt_zero(a);
    gradt_add<C, I, HASK>(a, s, K);
}

// Index of the D3Q19 velocity (ex, ey, ez), or -1.
constexpr int dir_index(int ex, int ey, int ez) {
    for (int i = 0; i < Q; i++)
        if (EX[i] == ex && EY[i] == ey && EZ[i] == ez) return i;
    return -1;
}

// The first in-plane offset O (dx = O % 3 - 1, dy = O / 3 - 1) whose direction (dx, dy, -1) is a
// D3Q19 velocity: the offset at which the consumers' sums of a new plane take their first term.
constexpr int first_up_offset() {
    for (int o = 0; o < 9; o++)
        if (dir_index(o % 3 - 1, o / 3 - 1, -1) > 0) return o;
    return -1;
}

// Sources of one site whose bbar* neighbourhood is staged in LDS, as source_site_staged, with the
// gather's partial sums pinned in registers after every PC_GATHER_GROUP directions.  Left free, the
// compiler issues all 114 LDS reads of the gather first and sinks the multiply-adds below them
// (they wait on the populations' loads), which needs far more than the 128 registers a lane has
// at four waves per SIMD; the empty asm statements, which only claim to read and write the
// partial sums, keep each group's reads next to their use.
#ifndef PC_GATHER_GROUP
#define PC_GATHER_GROUP 2
#endif
#ifndef PC_GRAD_GROUP
#define PC_GRAD_GROUP 3
#endif
template <typename C> __device__ __forceinline__ void pin(C &v) { asm volatile("" : "+v"(v)); }

template <int S, typename TL, bool KEEP>
__device__ __forceinline__ void source_site_pc(const Buf<S> &bF, const typename Buf<S>::R raw[Q],
                                               const typename Storage<S>::C *__restrict__ Tf,
                                               typename Storage<S>::C Tconst,
                                               const StepConst<typename Storage<S>::C> &k, const Codec &cd,
                                               int s, int bidx, const typename Storage<S>::C *const bs[3],
                                               typename Storage<S>::C *plane, int lidx,
                                               SiteState<typename Storage<S>::C> &keep) {
    using C = typename Storage<S>::C;
    C d[Q], beta[NB];
    Unroll<0, Q>::run([&](auto I) { d[I] = bF.template decode<I, 0>(raw[I], cd); });
    const PopMoments<C> m = pop_moments(d, k.rho_ref);
    C acc[NB];
#pragma unroll
    for (int c = 0; c < NB; c++) acc[c] = C(0);
    Unroll<0, Q>::run([&](auto I) {
        constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
        const C *pl = bs[1 - ez] + bidx;  // upstream site y - e_i lies in plane z - e_iz
        constexpr int off = -ey * TL::BX - ex;
        const C wgt = fma(C(WQ[I]), k.rho_ref, d[I]);
#pragma unroll
        for (int c = 0; c < NB; c++) acc[c] = fma(wgt, pl[c * TL::NB2 + off], acc[c]);
        if constexpr (I % PC_GATHER_GROUP == PC_GATHER_GROUP - 1) {
#pragma unroll
            for (int c = 0; c < NB; c++) pin(acc[c]);
        }
    });
    const C inv = recip(m.rho);
#pragma unroll
    for (int c = 0; c < NB; c++) beta[c] = acc[c] * inv;
    const C th = site_T(Tf, Tconst, s);
    C o[NSRC];
    predictor_sources(m, beta, th, k, o);
#pragma unroll
    for (int c = 0; c < NSRC; c++) plane[c * TL::NS + lidx] = o[c];
    if constexpr (KEEP) {
#pragma unroll
        for (int c = 0; c < NB; c++) keep.beta[c] = beta[c];
        keep.theta = th;
    }
}

using PcTile = Tile<64, 8>;
constexpr int PC_THREADS = 2 * PcTile::NT;

// LDS of one work-group (bytes), checked against the 160 KiB of a CU.
constexpr size_t pc_lds_bytes() {
    return sizeof(float) * (4 * (size_t)NB * PcTile::NB2 + 2 * (size_t)NSRC * PcTile::NS + 3 * (size_t)NB * PcTile::NT);
}
static_assert(pc_lds_bytes() <= 163840, "producer/consumer sweep exceeds the LDS of a CU");

// One plane of a source array (NSRC planes of n values, as the two-pass predictor writes them):
// field c of lattice plane z, as a buffer descriptor whose range is that plane alone, so that no
// offset can read outside it (a load past the range returns 0).
template <typename C>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t src_plane_rsrc(const C *src, int c, int z, int n, int nxy) {
    const unsigned long long a = (unsigned long long)(src + (size_t)c * n + (size_t)z * nxy);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    void *ptr = (void *)(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ptr, (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(nxy * (int)sizeof(C)), 0x00020000);
}

// MRT: the non-hydrodynamic moments relax at their own rate (ghost_relax, which carries the 9
// ghost moments of the pre-collision populations across the collision).  WALLS: the interior
// planes of a lattice with walls, the sources of planes 0 and nz-1 read from wsrc.
template <int S, bool HASK, bool FORCE, bool MRT, bool WALLS>
__global__ void __launch_bounds__(PC_THREADS)
k_fused_pc(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
           typename Storage<S>::T *__restrict__ Fo, typename Storage<S>::T *__restrict__ Bo,
           const typename Storage<S>::C *__restrict__ Tf, typename Storage<S>::C Tconst, Geo g,
           StepConst<typename Storage<S>::C> k, Codec cd, unsigned *__restrict__ flag, FusedGeo fg,
           const typename Storage<S>::C *__restrict__ accel, const typename Storage<S>::C *__restrict__ wsrc) {
    static_assert(S != 0, "double precision keeps the single-role sweep");
    using C = typename Storage<S>::C;
    using T = typename Storage<S>::T;
    using R = typename Buf<S>::R;
    using TL = PcTile;
    constexpr int TX = TL::TX, TY = TL::TY, NT = TL::NT, NS = TL::NS, NB2 = TL::NB2;
    constexpr int NSTAGE = (NB2 + NT - 1) / NT;
    constexpr int NRING = (TL::NH + NT - 1) / NT;
    constexpr int SB = (int)sizeof(T);
    __shared__ C bst[4][NB * NB2];     // staged bbar*, by plane mod 4
    __shared__ C lsrc[2][NSRC * NS];   // sources, by plane mod 2
    __shared__ C hand[3][NB * NT];     // gathered bbar of the tile sites, by plane mod 3

    // XCD-aware work-group numbering, as k_fused
    const int nblk = gridDim.x;
    int L = blockIdx.x;
    if ((nblk & 7) == 0) L = (L & 7) * (nblk >> 3) + (L >> 3);
    const int tx = L % fg.tiles_x;
    L /= fg.tiles_x;
    const int ty = L % fg.tiles_y;
    const int chunk = L / fg.tiles_y;

    Buf<S> bF, bB, bFo, bBo;
    bF.init(F, Q, g.n);
    bB.init(B, NB, g.n);
    bFo.init(Fo, Q, g.n);
    bBo.init(Bo, NB, g.n);

    // the chunk's planes [z0, z1): of 0 .. nz-1, or of the interior planes 1 .. nz-2 with walls
    const int z0 = (WALLS ? 1 : 0) + chunk * fg.zchunk;
    const int z1 = min(z0 + fg.zchunk, WALLS ? g.nz - 1 : g.nz);
    const int nxy = g.nx * g.ny;
    const bool producer = threadIdx.x < NT;
    const int t = threadIdx.x & (NT - 1);

    // the thread's tile site
    const int lx = t % TX, ly = t / TX;
    const int x0 = tx * TX, y0 = ty * TY;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool inside = gx < g.nx && gy < g.ny;
    const int wx = wrapc(gx, g.nx), wy = wrapc(gy, g.ny);
    const int ixy = wy * g.nx + wx;
    const int iidx = (ly + 1) * TL::HX + (lx + 1);
    const int ibidx = (ly + 2) * TL::BX + (lx + 2);

    // slots of plane q (q >= z0 - 2): staging q mod 4, sources q mod 2, hand-off q mod 3
    auto sslot = [&](int q) { return (q - z0 + 8) & 3; };
    auto cslot = [&](int q) { return (q - z0 + 8) & 1; };
    auto hslot = [&](int q) { return (q - z0 + 9) % 3; };
    auto zoff = [&](int q) { return wrapc(q, g.nz) * nxy; };

    RangeMax amax;

    // Issue priority on a SIMD: the producer waves that hold ring sites (the longest load chains
    // of an iteration) first, then the consumers, then the other producers, which finish their
    // plane with time to spare.  Raising the consumers above every producer instead delays the
    // ring loads and costs 11% in 16-bit storage.
    if (producer) {
        if (__builtin_amdgcn_readfirstlane(t >> 6) < (TL::NH + 63) / 64) __builtin_amdgcn_s_setprio(2);
        // ring sites and staging sites of this thread
        int rxy[NRING], rlidx[NRING], rbidx[NRING];
#pragma unroll
        for (int j = 0; j < NRING; j++) {
            const int h = t + j * NT;
            int rlx = 0, rly = 0;
            if (h < TL::HX) {
                rly = -1;
                rlx = h - 1;
            } else if (h < 2 * TL::HX) {
                rly = TY;
                rlx = h - TL::HX - 1;
            } else if (h < 2 * TL::HX + TY) {
                rlx = -1;
                rly = h - 2 * TL::HX;
            } else {
                rlx = TX;
                rly = h - 2 * TL::HX - TY;
            }
            rxy[j] = wrapc(y0 + rly, g.ny) * g.nx + wrapc(x0 + rlx, g.nx);
            rlidx[j] = (rly + 1) * TL::HX + (rlx + 1);
            rbidx[j] = (rly + 2) * TL::BX + (rlx + 2);
        }
        // Staged sites: every thread takes one (site t) and the last NB2 - NT threads a second
        // (site t + NT - SHIFT), so that the waves holding ring sites (the first NH threads) stage
        // one site and the others two.  A wave with any second site loads for all its lanes (a
        // lane without one repeats site NT, a line already fetched); the others skip the round.
        static_assert(NSTAGE == 2 && TL::NH <= (2 * NT - NB2) / 64 * 64, "staging rounds of the producer tile");
        constexpr int SHIFT = 2 * NT - NB2;
        const bool stage2 = __builtin_amdgcn_readfirstlane(t >> 6) >= SHIFT / 64;  // wave-uniform
        int sxy[NSTAGE];  // byte offsets within a plane
#pragma unroll
        for (int j = 0; j < NSTAGE; j++) {
            const int r = j == 0 ? t : max(t + NT - SHIFT, NT);
            const int bx = r % TL::BX - 2, by = r / TL::BX - 2;
            sxy[j] = (wrapc(y0 + by, g.ny) * g.nx + wrapc(x0 + bx, g.nx)) * SB;
        }
        // Past the chunk's end the last plane it needs is read again (an L2 hit) and not used:
        // loads issued on every path need no register copies between the loop's iterations.
        R sraw[NSTAGE][NB];
        R praw[Q];
        auto stage_issue = [&](int q) {
            const int zb = zoff(q) * SB;
            Unroll<0, NB>::run([&](auto c) { sraw[0][c] = bB.template loadraw<c>(sxy[0], zb); });
            if (stage2) Unroll<0, NB>::run([&](auto c) { sraw[1][c] = bB.template loadraw<c>(sxy[1], zb); });
        };
        auto stage_commit = [&](int q) {
            C *dst = bst[sslot(q)];
            Unroll<0, NB>::run([&](auto c) { dst[c * NB2 + t] = bB.template decode<c, Q>(sraw[0][c], cd); });
            if (stage2 && t >= SHIFT) {
                const int r = t + NT - SHIFT;
                Unroll<0, NB>::run([&](auto c) { dst[c * NB2 + r] = bB.template decode<c, Q>(sraw[1][c], cd); });
            }
        };
        auto pops_issue = [&](int p) {
            const int zb = zoff(p) * SB;
            Unroll<0, Q>::run([&](auto I) { praw[I] = bF.template loadraw<I>(ixy * SB, zb); });
        };

        // prologue: staged planes z0-2 .. z0 in LDS, z0+1 and the populations of z0-1 loading
        for (int q = z0 - 2; q <= z0; q++) {
            stage_issue(q);
            stage_commit(q);
        }
        stage_issue(z0 + 1);
        pops_issue(z0 - 1);
        __syncthreads();
        // one plane per iteration; the iteration after the last only meets the consumers'
        // barrier (kept out of the loop, so that no path skips the loop's loads)
        for (int p = z0 - 1; p <= z1; p++) {
            // staged plane p+2 for the next iteration (its slot last served plane p-2)
            stage_commit(p + 2);
            stage_issue(min(p + 3, z1 + 1));
            C *plane = lsrc[cslot(p)];
            if constexpr (WALLS) {
                static_assert(sizeof(C) == 4, "the wall planes' sources are read as 32-bit values");
                if (p == 0 || p == g.nz - 1) {  // a wall-adjacent plane (wave-uniform): no gather here
#pragma unroll
                    for (int c = 0; c < NSRC; c++) {
                        const __amdgpu_buffer_rsrc_t rs = src_plane_rsrc(wsrc, c, p, g.n, nxy);
                        plane[c * NS + iidx] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, ixy * 4, 0, 0));
#pragma unroll
                        for (int j = 0; j < NRING; j++)
                            if (t + j * NT < TL::NH)
                                plane[c * NS + rlidx[j]] =
                                    __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, rxy[j] * 4, 0, 0));
                    }
                    pops_issue(min(p + 1, z1));
                    __syncthreads();
                    continue;
                }
            }
            const C *bs[3] = {bst[sslot(p - 1)], bst[sslot(p)], bst[sslot(p + 1)]};
            const int zo = zoff(p);
            SiteState<C> keep;
            source_site_pc<S, TL, true>(bF, praw, Tf, Tconst, k, cd, zo + ixy, ibidx, bs, plane, iidx, keep);
            C *hd = hand[hslot(p)];
#pragma unroll
            for (int c = 0; c < NB; c++) hd[c * NT + t] = keep.beta[c];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < NRING; j++) {
                if (t + j * NT < TL::NH) {
                    R rraw[Q];
                    const int zb = zo * SB;
                    Unroll<0, Q>::run([&](auto I) { rraw[I] = bF.template loadraw<I>(rxy[j] * SB, zb); });
                    SiteState<C> dummy;
                    source_site_pc<S, TL, false>(bF, rraw, Tf, Tconst, k, cd, zo + rxy[j], rbidx[j], bs, plane,
                                                     rlidx[j], dummy);
                }
            }
            pops_issue(min(p + 1, z1));
            __syncthreads();
        }
        __syncthreads();
    } else {
        __builtin_amdgcn_s_setprio(1);
        // push targets of the tile site: byte offsets of its 3 x 3 in-plane neighbourhood
        // (periodic), fixed for the whole chunk; the target plane's offset is wave-uniform
        int yx[9];
        {
            const int Xo[3] = {wx == 0 ? g.nx - 1 : wx - 1, wx, wx == g.nx - 1 ? 0 : wx + 1};
            const int Yo[3] = {(wy == 0 ? g.ny - 1 : wy - 1) * g.nx, wy * g.nx, (wy == g.ny - 1 ? 0 : wy + 1) * g.nx};
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int a = 0; a < 3; a++) yx[b * 3 + a] = (Yo[b] + Xo[a]) * SB;
        }
        GradT<C> X, Y, Z;  // gradient sums of three consecutive planes, roles rotating
        gradt_zero(X);
        gradt_zero(Y);
        gradt_zero(Z);
        __syncthreads();  // the producers' prologue
        // One iteration with A0, A1, A2 the sums of planes q-1, q, q+1; A0 is then done and
        // serves as the next iteration's plane q+2, whose first term sets it (gradt_set).  Rotating
        // the roles by argument order (the loop unrolled by three) moves no registers.
        // The populations of the plane a consumer collides, read a second time (their last use:
        // non-temporal in single precision), at the top priority, above the ring producers, then
        // back to the consumers' level: in float and BF16 storage the chain the collision waits
        // on starts earlier (+3% / +2%); FP16 storage measured -0.5% and keeps its level.  In
        // single precision they are loaded one iteration ahead, after the previous plane's
        // stores (loop-carried, no extra registers: +2.5%); in 16-bit storage that costs 5%, and
        // they are loaded at the start of their own iteration.
        constexpr int POL = S == 1 ? 2 : 0;
        constexpr bool AHEAD = S == 1;
        constexpr bool LOAD_FIRST = S != 2;
        R craw[Q];
        auto craw_issue = [&](int zl) {  // zl: the plane's offset in sites
            if constexpr (LOAD_FIRST) __builtin_amdgcn_s_setprio(3);
            Unroll<0, Q>::run([&](auto I) { craw[I] = bF.template loadraw<I, POL>(ixy * SB, zl * SB); });
            if constexpr (LOAD_FIRST) __builtin_amdgcn_s_setprio(1);
        };
        if constexpr (AHEAD) craw_issue(zoff(z0));
        auto iter = [&](int p, GradT<C> &A0, GradT<C> &A1, GradT<C> &A2) {
            const int q = p - 1;  // the source plane the producers finished last iteration
            if (q >= z0 - 1) {
                const int zc = zoff(q - 1);
                // plane q-1 is one of the chunk's (wave-uniform); its lanes outside the lattice
                // compute on the wrapped site and store nothing
                const bool live = q - 1 >= z0;
                // 16-bit storage: the populations of plane q-1 now.  The chunk's first
                // iteration, which has no plane to collide, loads the plane the producers read
                // first (an L2 hit) and discards it: a value defined on every path costs no
                // register fill.
                if constexpr (!AHEAD) craw_issue(live ? zc : zoff(z0 - 1));
                // source plane q: its 3 x 3 neighbourhood adds to the sums of planes q-1, q, q+1
                const C *pl = lsrc[cslot(q)] + iidx;
                Unroll<0, 9>::run([&](auto O) {
                    constexpr int dx = (int)O % 3 - 1, dy = (int)O / 3 - 1;
                    C sv[NSRC];
#pragma unroll
                    for (int c = 0; c < NSRC; c++) sv[c] = pl[c * NS + dy * TL::HX + dx];
                    constexpr int dn = dir_index(dx, dy, 1);   // from a site of plane q-1
                    constexpr int d0 = dir_index(dx, dy, 0);   // from a site of plane q
                    constexpr int up = dir_index(dx, dy, -1);  // from a site of plane q+1
                    if constexpr (dn > 0) gradt_add<C, dn, HASK>(A0, sv, k.K);
                    if constexpr (d0 > 0) gradt_add<C, d0, HASK>(A1, sv, k.K);
                    if constexpr (up > 0) {
                        if constexpr (O == first_up_offset())  // the first of plane q+1's terms
                            gradt_set<C, up, HASK>(A2, sv, k.K);
                        else
                            gradt_add<C, up, HASK>(A2, sv, k.K);
                    }
                    if constexpr (O % PC_GRAD_GROUP == PC_GRAD_GROUP - 1) {  // as in the gather
#pragma unroll
                        for (int c = 0; c < 3; c++) {
                            pin(A0.F[c]);
                            pin(A1.F[c]);
                            pin(A2.F[c]);
                        }
#pragma unroll
                        for (int c = 0; c < 6; c++) {
                            pin(A0.S[c]);
                            pin(A1.S[c]);
                            pin(A2.S[c]);
                        }
                    }
                });
                if (live) {
                    C Fv[3], Sv[6];
                    gradt_finish(A0, Fv, Sv);
                    C d[Q];
                    Unroll<0, Q>::run([&](auto I) { d[I] = bF.template decode<I, 0>(craw[I], cd); });
                    SiteState<C> cur;
                    const C *hd = hand[hslot(q - 1)];
#pragma unroll
                    for (int c = 0; c < NB; c++) cur.beta[c] = hd[c * NT + t];
                    const int s = zc + ixy;
                    cur.theta = site_T(Tf, Tconst, s);
                    const PopMoments<C> m = pop_moments(d, k.rho_ref);
                    if constexpr (FORCE) {
                        C a[3];
                        site_accel(k, accel, g.n, s, a);
                        add_body_force(m, a, Fv, Sv);
                    }
                    C g0[MRT ? 9 : 1];
                    if constexpr (MRT) ghost_moments(d, g0);
                    collide(d, cur.beta, m, Fv, Sv, cur.theta, k);
                    if constexpr (MRT) ghost_relax(g0, d, k.ghost);
                    const int wz = wrapc(q - 1, g.nz);
                    int Zo[3];
                    Zo[0] = (wz == 0 ? g.nz - 1 : wz - 1) * nxy;
                    Zo[1] = zc;
                    Zo[2] = (wz == g.nz - 1 ? 0 : wz + 1) * nxy;
                    if (inside) {
                        Unroll<0, Q>::run([&](auto I) {
                            bFo.template storef<I, 0>(yx[(EY[I] + 1) * 3 + EX[I] + 1], d[I], cd, amax,
                                                      Zo[EZ[I] + 1] * SB);
                        });
                        Unroll<0, NB>::run(
                            [&](auto c) { bBo.template storef<c, Q>(ixy * SB, cur.beta[c], cd, amax, zc * SB); });
                    }
                }
                // single precision: the populations of plane q, collided next iteration (past the
                // chunk's end its last plane again, unused)
                if constexpr (AHEAD) craw_issue(zoff(min(max(q, z0), z1 - 1)));
            }
            __syncthreads();
        };
        int p = z0 - 1;
        for (; p + 2 <= z1 + 1; p += 3) {
            iter(p, X, Y, Z);
            iter(p + 1, Y, Z, X);
            iter(p + 2, Z, X, Y);
        }
        if (p <= z1 + 1) iter(p++, X, Y, Z);
        if (p <= z1 + 1) iter(p, Y, Z, X);
    }
    report_range<S>(amax, cd, flag);
}

// Shapes the producer/consumer sweep takes: float and 16-bit storage, more than two z planes
// (it marches; with walls at least one interior plane), buffers within the fused sweep's 32-bit
// offsets.
inline bool fused_pc_supported(const Geo &g, int storage) {
    return storage != 0 && g.nz >= 3 && fused_supported(g, storage);
}

}  // namespace lbm
