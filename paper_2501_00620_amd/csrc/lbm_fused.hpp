// lbm_fused.hpp -- single-pass step: z-marching sweep with LDS planes of predictor sources.
//
// One work-group owns an xy tile of TX x TY sites and marches through a chunk of z planes.
// The forcing moments at a site need the predictor sources (rho b and u*, Eqs. 59-61 with
// Eq. 68) of its 18 neighbours, and each source needs the site's post-stream populations and
// its gathered bbar (Eq. 66): bbar(y) = sum_i fbar_i(y) bbar*(y - e_i) / rho(y), one more hop.
// Per plane z the work-group
//   1. stages the post-collision bbar* of plane z+2 over the tile plus two rings in LDS
//      (coalesced loads; each value is then read by up to 19 gathers from LDS);
//   2. evaluates the sources of plane z+1 on the tile plus a one-site ring (the ring overlaps
//      the neighbouring tiles) into one of three LDS source planes, keeping the tile's gathered
//      bbar in registers and part of its populations in LDS for the next iteration;
//   3. takes the isotropic gradients of plane z from the source planes z-1, z, z+1, collides
//      the registers kept from the previous iteration, and pushes the results out.
// The algorithmic minimum is 2 x 25 values per lattice update: each site's state read once and
// written once.  On top of it come the ring sites (neighbouring tiles on the same XCD bring them
// into L2 at about the same time) and the collision's second read of the tile's populations not
// kept in LDS (an L2 hit unless the stream in between evicted them).  The staging and source
// loads are issued one plane iteration ahead of their use.
//
// Work-groups are numbered so that the ones dispatched to one XCD (block index mod 8) take
// neighbouring tiles of the same z chunk, which share their rings through that XCD's L2.
// Any lattice shape works: tile sites beyond the lattice are computed (wrapped) only as ring
// sources and never stored; nz <= 2 stages and evaluates each plane once.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

#ifndef FUSED_PREFETCH_RING
#define FUSED_PREFETCH_RING 0  // ring populations loaded one plane ahead too (more VGPRs)
#endif
#ifndef GRAD_GROUP
#define GRAD_GROUP 3    // neighbours per scheduling group in the gradient
#endif
#ifndef GATHER_GROUP
#define GATHER_GROUP 5  // directions per scheduling group in the gather
#endif
// Populations of the tile's own sites kept in LDS from the source evaluation to the collision
// one plane later, in 4- and 2-byte storage: the first N of the 19, as many as fit the LDS
// beside the source and staging planes.  The rest are read again at the collision.
#ifndef FUSED_STASH_F32
#define FUSED_STASH_F32 8
#endif
#ifndef FUSED_STASH_16
#define FUSED_STASH_16 16
#endif
#ifndef FUSED_STASH_F64
#define FUSED_STASH_F64 0
#endif

template <int TX_, int TY_> struct Tile {
    static constexpr int TX = TX_, TY = TY_;
    static constexpr int NT = TX * TY;            // threads = tile sites
    static constexpr int HX = TX + 2, HY = TY + 2;
    static constexpr int NS = HX * HY;            // source sites per LDS plane (tile + ring)
    static constexpr int NH = NS - NT;            // ring sites
    static constexpr int BX = TX + 4, BY = TY + 4;
    static constexpr int NB2 = BX * BY;           // bbar* staging sites (tile + two rings)
};

// 4- and 2-byte storage compute in float: 64 x 8 tiles (71 KB of sources + 59 KB of staged
// bbar*).  Double needs twice the bytes per site: 32 x 8 tiles (73 + 62 KB), 256 threads, so
// that the one work-group the LDS admits per CU still gives each SIMD a wave (64 x 2 tiles left
// two SIMDs idle and recomputed a ring larger than the tile: 2.3x slower).
#ifndef FUSED_TX
#define FUSED_TX 64
#endif
#ifndef FUSED_TY
#define FUSED_TY 8
#endif
template <int S> struct TileFor { using type = Tile<FUSED_TX, FUSED_TY>; };
#ifndef FUSED64_TX
#define FUSED64_TX 32
#endif
#ifndef FUSED64_TY
#define FUSED64_TY 8
#endif
template <> struct TileFor<0> { using type = Tile<FUSED64_TX, FUSED64_TY>; };
// populations kept in LDS by the marching single-lattice kernel (none in the one-plane kernel,
// which runs several work-groups per CU)
template <int S> constexpr int fused_stash() {
    return S == 0 ? FUSED_STASH_F64 : (S == 1 ? FUSED_STASH_F32 : FUSED_STASH_16);
}
// Tiles of the one-plane serving kernel.  With one LDS slot of each kind (43 KB) and the in-plane
// arithmetic it fits 128 VGPRs, so two 512-thread work-groups share a CU (four waves per SIMD),
// each covering the other's load waits.
#ifndef SERVE_THIN_TX
#define SERVE_THIN_TX 64
#endif
#ifndef SERVE_THIN_TY
#define SERVE_THIN_TY 8
#endif
template <int S> struct ThinTileFor { using type = Tile<SERVE_THIN_TX, SERVE_THIN_TY>; };

// Largest |value| a thread stored into each array (populations, bbar), unscaled, for the 16-bit
// range check (report_range).
struct RangeMax {
    float f = 0.0f, b = 0.0f;
};

struct FusedGeo {
    int tiles_x, tiles_y, nchunks, zchunk;
};

// Buffer addressing of an array of planes (n values each): one buffer resource (4 SGPRs) per
// group of PPG planes and a 32-bit per-lane byte offset (site offset plus the plane's offset
// inside its group; the scalar-offset operand stays 0, since a uniform offset the compiler
// keeps in a VGPR would otherwise be re-scalarised lane by lane).  No 64-bit per-lane address is ever formed, and a
// group stays below 4 GiB for every lattice the fused kernel accepts.
template <int S> struct Buf {
    using T = typename Storage<S>::T;
    using C = typename Storage<S>::C;
    static constexpr int PPG = S == 0 ? 3 : (S == 1 ? 5 : 9);
    static constexpr int NG = (Q + PPG - 1) / PPG;
    __amdgpu_buffer_rsrc_t r[NG];
    int pb;  // plane bytes

    // Every descriptor is assigned (groups past the last plane get an empty range), from base
    // addresses passed through readfirstlane, so the compiler knows them to be wave-uniform and
    // keeps them in SGPRs instead of looping over lanes.
    __device__ __forceinline__ void init(const T *base, int nplanes, int n) {
        pb = __builtin_amdgcn_readfirstlane(n * (int)sizeof(T));
#pragma unroll
        for (int g = 0; g < NG; g++) {
            const int np = nplanes - g * PPG;
            const unsigned bytes = np > 0 ? (unsigned)(np < PPG ? np : PPG) * (unsigned)pb : 0u;
            const unsigned long long a = (unsigned long long)(base + (size_t)(np > 0 ? g : 0) * PPG * n);
            const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
            const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
            void *p = (void *)(((unsigned long long)hi << 32) | lo);
            r[g] = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)__builtin_amdgcn_readfirstlane((int)bytes),
                                                     0x00020000);
        }
    }
    // Byte offset of plane j (< PPG) inside its group.  It can reach 2^31 and beyond (a 512^3
    // lattice puts plane 4 of a float group at 2^31 bytes), so it is formed in unsigned 32-bit
    // arithmetic, exact below the group's 4 GiB (fused_supported_s), and handed to the buffer
    // instruction's unsigned offset operand as the same 32 bits.
    __device__ __forceinline__ int plane_offset(int j) const {
        return (int)((unsigned)j * (unsigned)pb);
    }
    // A value as loaded (the storage type), decoded only where it is used: a load whose result
    // is kept raw can be issued one plane ahead without the wait for it coming at the load.
    using R = T;
    // plane K of this array: its byte offset in its group goes to the scalar-offset operand
    // through readfirstlane, so it is known to be wave-uniform.  POL: cache-policy bits.
    // zoff: a further byte offset the whole wavefront shares (a plane of the lattice), added to
    // the scalar operand so that the per-lane offset can stay fixed from plane to plane.
    template <int K, int POL = 0> __device__ __forceinline__ R loadraw(int off, int zoff = 0) const {
        constexpr int g = K / PPG, j = K % PPG;
        const __amdgpu_buffer_rsrc_t rs = r[g];
        const int so = __builtin_amdgcn_readfirstlane((int)((unsigned)plane_offset(j) + (unsigned)zoff));
        if constexpr (S == 0) {
            return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, so, POL));
        } else if constexpr (S == 1) {
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, so, POL));
        } else {
            return __builtin_amdgcn_raw_buffer_load_b16(rs, off, so, POL);
        }
    }
    // plane K of this array holds codec field F0 + K.  A D3Q19 lattice's fp16 codec has one
    // scale per array (populations from field 0, bbar from field Q), so field F0 stands for the
    // whole array: two constants stay in scalar registers instead of fifty.
    template <int K, int F0> __device__ __forceinline__ C decode(R v, const Codec &cd) const {
        if constexpr (S == 0 || S == 1) {
            return v;
        } else if constexpr (S == 2) {
            // scale x code as a multiply-add with a zero addend: one mixed-precision FMA that
            // reads the fp16 code directly, instead of a conversion and a multiply (the product
            // is exact in float; only a zero's sign can differ)
            return fmaf(cd.scale[F0], half_bits_to_float(v), 0.0f);
        } else {  // bf16 codes hold the deviation itself (unit scale)
            return bf16_bits_to_float(v);
        }
    }
    template <int K, int F0> __device__ __forceinline__ C loadf(int off, const Codec &cd) const {
        return decode<K, F0>(loadraw<K>(off), cd);
    }
    // Stores a value; for 16-bit codes, rm collects |value| per array so that one comparison after
    // the sweep detects overflow (an overflowing code is stored as +-inf and reported as RANGE, the
    // same rule as the other kernels' encoders).
    template <int K, int F0>
    __device__ __forceinline__ void storef(int off, C v, const Codec &cd, RangeMax &rm, int zoff = 0) const {
        constexpr int g = K / PPG, j = K % PPG;
        const __amdgpu_buffer_rsrc_t rs = r[g];
        const int so = __builtin_amdgcn_readfirstlane((int)((unsigned)plane_offset(j) + (unsigned)zoff));
        if constexpr (S == 0) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0)), v),
                                                  rs, off, so, 0);
        } else if constexpr (S == 1) {
            // non-temporal (cache-policy bit NT): in single precision the stores would otherwise
            // evict from L2 the populations the collision reads a second time
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, off, so, 2);
        } else if constexpr (S == 2) {
            float &m = F0 == 0 ? rm.f : rm.b;
            m = fmaxf(m, fabsf(v));
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (_Float16)(v * cd.inv[F0])), rs, off,
                                                  so, 0);
        } else {
            float &m = F0 == 0 ? rm.f : rm.b;
            m = fmaxf(m, fabsf(v));
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (__bf16)v), rs, off, so, 0);
        }
    }
};

// What a thread carries from the source evaluation of its site to the site's collision one
// plane later: the gathered bbar (which cannot be re-gathered then, its upstream plane is no
// longer staged) and the ISO temperature offset.  The populations travel in LDS as far as it
// has room (NST of them, as loaded); the others are read again at the collision (the same
// work-group read them one plane earlier, so they mostly come from L2).
template <typename C> struct SiteState {
    C beta[NB];
    C theta;
};

__device__ __forceinline__ int wrapc(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <int S>
__device__ __forceinline__ void load_pops(const Buf<S> &bF, int off, const Codec &cd, typename Storage<S>::C d[Q]) {
    Unroll<0, Q>::run([&](auto I) { d[I] = bF.template loadf<I, 0>(off, cd); });
}

// Sources of one site from its stored, gathered bbar (the first step after the state was set).
template <int S, int NS, bool KEEP>
__device__ __forceinline__ void source_site_gathered(const Buf<S> &bF, const Buf<S> &bB,
                                                     const typename Storage<S>::C *__restrict__ Tf,
                                                     typename Storage<S>::C Tconst,
                                                     const StepConst<typename Storage<S>::C> &k, const Codec &cd,
                                                     int s, typename Storage<S>::C *plane, int lidx,
                                                     SiteState<typename Storage<S>::C> &keep) {
    using C = typename Storage<S>::C;
    const int off = s * (int)sizeof(typename Storage<S>::T);
    C d[Q], beta[NB];
    load_pops<S>(bF, off, cd, d);
    const PopMoments<C> m = pop_moments(d, k.rho_ref);
    Unroll<0, NB>::run([&](auto c) { beta[c] = bB.template loadf<c, Q>(off, cd); });
    const C th = site_T(Tf, Tconst, s);
    C o[NSRC];
    predictor_sources(m, beta, th, k, o);
#pragma unroll
    for (int c = 0; c < NSRC; c++) plane[c * NS + lidx] = o[c];
    if constexpr (KEEP) {
#pragma unroll
        for (int c = 0; c < NB; c++) keep.beta[c] = beta[c];
        keep.theta = th;
    }
}

// Sources of one site whose bbar* neighbourhood is staged in LDS: the gather of Eq. 66 reads
// the staged planes bs[0..2] (planes z-1, z, z+1); bidx is the site's staging index.
// The site's populations arrive raw (loaded one plane ahead).  THIN1 (one z plane): the upstream
// sites y - e_i of a direction and of its mirror in z coincide, so the gather runs over the 9
// in-plane offsets with the arriving populations summed per offset first.
template <int S, typename TL, bool KEEP, bool THIN1 = false>
__device__ __forceinline__ void source_site_staged(const Buf<S> &bF, const typename Buf<S>::R raw[Q],
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
    if constexpr (THIN1) {
        // arriving populations summed per in-plane offset (ex, ey), index (ey + 1) * 3 + ex + 1
        C wg[9];
#pragma unroll
        for (int q = 0; q < 9; q++) wg[q] = C(0);
        Unroll<0, Q>::run([&](auto I) {
            constexpr int q = (EY[I] + 1) * 3 + EX[I] + 1;
            wg[q] += fma(C(WQ[I]), k.rho_ref, d[I]);
        });
        const C *pl = bs[0] + bidx;
        Unroll<0, 9>::run([&](auto Q9) {
            constexpr int ex = (int)Q9 % 3 - 1, ey = (int)Q9 / 3 - 1;
            constexpr int off = -ey * TL::BX - ex;
#pragma unroll
            for (int c = 0; c < NB; c++) acc[c] = fma(wg[Q9], pl[c * TL::NB2 + off], acc[c]);
            if constexpr (Q9 % 3 == 2) __builtin_amdgcn_sched_barrier(0);
        });
    } else {
        Unroll<0, Q>::run([&](auto I) {
            constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
            const C *pl = bs[1 - ez] + bidx;  // upstream site y - e_i lies in plane z - e_iz
            constexpr int off = -ey * TL::BX - ex;
            const C wgt = fma(C(WQ[I]), k.rho_ref, d[I]);
#pragma unroll
            for (int c = 0; c < NB; c++) acc[c] = fma(wgt, pl[c * TL::NB2 + off], acc[c]);
            if constexpr (I % GATHER_GROUP == GATHER_GROUP - 1) __builtin_amdgcn_sched_barrier(0);
        });
    }
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

// One work-group sweeps tile (tx, ty) of z chunk `chunk` for one step.  Shared by the
// single-lattice kernel and the multi-lattice serving kernel.  HASK: T_ref != 1/3 (the constant
// part of rho b enters the second-moment source).  THIN1: the lattice has exactly one z plane
// (one LDS slot of each kind, about a third of the LDS, so that several work-groups share a CU).
// amax collects |16-bit codes| stored.  NST_: populations of the tile's own sites carried in
// LDS from the source evaluation to the collision (staged kernels only).  FORCE: a body-force
// acceleration (the field `accel`, 3 planes of n, or the uniform one of k) enters the forcing
// moments before the collision.
template <int S, bool GATHERED, bool HASK, bool THIN1 = false, typename TL = typename TileFor<S>::type, int NST_ = 0,
          bool FORCE = false>
__device__ __forceinline__ void sweep_tile(const typename Storage<S>::T *__restrict__ F,
                                           const typename Storage<S>::T *__restrict__ B,
                                           typename Storage<S>::T *__restrict__ Fo,
                                           typename Storage<S>::T *__restrict__ Bo,
                                           const typename Storage<S>::C *__restrict__ Tf,
                                           typename Storage<S>::C Tconst, const Geo &g,
                                           const StepConst<typename Storage<S>::C> &k, const Codec &cd,
                                           const FusedGeo &fg, int tx, int ty, int chunk, RangeMax &amax,
                                           const typename Storage<S>::C *__restrict__ accel = nullptr) {
    using C = typename Storage<S>::C;
    using T = typename Storage<S>::T;
    constexpr int TX = TL::TX, TY = TL::TY, NS = TL::NS, NB2 = TL::NB2;
    constexpr int NSTAGE = (NB2 + TL::NT - 1) / TL::NT;  // staging sites per thread
    constexpr int SB = (int)sizeof(T);
    constexpr int NSLOT = THIN1 ? 1 : 3;
    __shared__ C lds[NSLOT][NSRC * NS];
    __shared__ C bst[GATHERED ? 1 : NSLOT][GATHERED ? 1 : NB * NB2];
    // two slots by plane parity: the sources of plane z+1 are evaluated before plane z collides
    constexpr int NST = GATHERED ? 0 : NST_;
    __shared__ typename Buf<S>::R pst[NST > 0 ? 2 * NST * TL::NT : 1];
    (void)pst;

    Buf<S> bF, bB, bFo, bBo;
    bF.init(F, Q, g.n);
    bB.init(B, NB, g.n);
    bFo.init(Fo, Q, g.n);
    bBo.init(Bo, NB, g.n);

    const int z0 = chunk * fg.zchunk;
    const int z1 = min(z0 + fg.zchunk, g.nz);
    const int nxy = g.nx * g.ny;

    // --- per-thread offsets, computed once (xy part; the plane offset is added per plane) ---
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x0 = tx * TX, y0 = ty * TY;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool inside = gx < g.nx && gy < g.ny;
    const int wx = wrapc(gx, g.nx), wy = wrapc(gy, g.ny);
    const int ixy = wy * g.nx + wx;
    const int iidx = (ly + 1) * TL::HX + (lx + 1);
    const int ibidx = (ly + 2) * TL::BX + (lx + 2);
    // push targets: x and y offsets of the 3x3 neighbourhood (periodic)
    int Xo[3], Yo[3];
    Xo[0] = wx == 0 ? g.nx - 1 : wx - 1;
    Xo[1] = wx;
    Xo[2] = wx == g.nx - 1 ? 0 : wx + 1;
    Yo[0] = (wy == 0 ? g.ny - 1 : wy - 1) * g.nx;
    Yo[1] = wy * g.nx;
    Yo[2] = (wy == g.ny - 1 ? 0 : wy + 1) * g.nx;
    // ring sites (one per thread when the tile has 8 rows; general stride below)
    constexpr int NRING = (TL::NH + TL::NT - 1) / TL::NT;
    int rxy[NRING], rlidx[NRING], rbidx[NRING];
#pragma unroll
    for (int j = 0; j < NRING; j++) {
        const int h = threadIdx.x + j * TL::NT;
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
    // bbar* staging sites
    int sxy[NSTAGE];
#pragma unroll
    for (int j = 0; j < NSTAGE; j++) {
        const int r = threadIdx.x + j * TL::NT;
        const int bx = r % TL::BX - 2, by = r / TL::BX - 2;
        sxy[j] = wrapc(y0 + by, g.ny) * g.nx + wrapc(x0 + bx, g.nx);
    }

    const bool thin = THIN1 || g.nz <= 2;

    // Raw values loaded one plane ahead: the staged bbar* of the next plane to stage, and the
    // populations of the next plane whose sources are evaluated (tile site and ring sites).
    // Loads one plane ahead (PIPE) in every storage (in double precision +35% at one wave per
    // SIMD); the first step from a gathered bbar and the one-plane kernel load where they use.
    constexpr bool PIPE = !GATHERED && !THIN1;
    using R = typename Buf<S>::R;
    R sraw[NSTAGE][NB];
    R praw[Q];
    R rraw[NRING][Q];
    (void)sraw;
    (void)praw;
    (void)rraw;

    auto stage_issue = [&](int q) {
        if constexpr (!GATHERED) {
            const int zo = wrapc(q, g.nz) * nxy;
#pragma unroll
            for (int j = 0; j < NSTAGE; j++) {
                if (threadIdx.x + j * TL::NT < NB2) {
                    const int off = (zo + sxy[j]) * SB;
                    Unroll<0, NB>::run([&](auto c) { sraw[j][c] = bB.template loadraw<c>(off); });
                }
            }
        }
    };
    auto stage_commit = [&](int slot) {
        if constexpr (!GATHERED) {
#pragma unroll
            for (int j = 0; j < NSTAGE; j++) {
                const int r = threadIdx.x + j * TL::NT;
                if (r < NB2) {
                    Unroll<0, NB>::run([&](auto c) { bst[slot][c * NB2 + r] = bB.template decode<c, Q>(sraw[j][c], cd); });
                }
            }
        }
    };
    auto stage = [&](int q, int slot) {
        if constexpr (PIPE) {
            stage_issue(q);
            stage_commit(slot);
        } else if constexpr (!GATHERED) {
            const int zo = wrapc(q, g.nz) * nxy;
#pragma unroll
            for (int j = 0; j < NSTAGE; j++) {
                const int r = threadIdx.x + j * TL::NT;
                if (r < NB2) {
                    const int off = (zo + sxy[j]) * SB;
                    Unroll<0, NB>::run([&](auto c) { bst[slot][c * NB2 + r] = bB.template loadf<c, Q>(off, cd); });
                }
            }
        }
    };
    // slot of a staged plane q: (q - z0 + 6) % 3 when marching, q itself when nz <= 2
    auto bslot = [&](int q) { return thin ? wrapc(q, g.nz) : (q - z0 + 6) % 3; };

    // populations of plane p (tile site and ring sites), kept raw
    auto fill_issue = [&](int p) {
        if constexpr (!GATHERED) {
            // (with PIPE, this runs one plane ahead of fill_compute)
            const int zo = wrapc(p, g.nz) * nxy;
            const int off = (zo + ixy) * SB;
            Unroll<0, Q>::run([&](auto I) { praw[I] = bF.template loadraw<I>(off); });
#if FUSED_PREFETCH_RING
            if constexpr (PIPE)
#pragma unroll
            for (int j = 0; j < NRING; j++) {
                if (threadIdx.x + j * TL::NT < TL::NH) {
                    const int roff = (zo + rxy[j]) * SB;
                    Unroll<0, Q>::run([&](auto I) { rraw[j][I] = bF.template loadraw<I>(roff); });
                }
            }
#endif
        }
    };
    // sources of plane p into LDS source slot `slot`, keeping the tile state; the staged path
    // takes the populations fill_issue(p) loaded
    // (b0, b1, b2: staging slots of planes p-1, p, p+1)
    auto fill_compute = [&](int p, int slot, SiteState<C> &keep, int b0, int b1, int b2) {
        const int zo = wrapc(p, g.nz) * nxy;
        if constexpr (GATHERED) {
            source_site_gathered<S, NS, true>(bF, bB, Tf, Tconst, k, cd, zo + ixy, lds[slot], iidx, keep);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < NRING; j++) {
                if (threadIdx.x + j * TL::NT < TL::NH) {
                    SiteState<C> dummy;
                    source_site_gathered<S, NS, false>(bF, bB, Tf, Tconst, k, cd, zo + rxy[j], lds[slot], rlidx[j], dummy);
                }
            }
        } else {
            const C *bs[3] = {bst[b0], bst[b1], bst[b2]};
            // ring populations not loaded one plane ahead are loaded just before their use
            // (issued before the tile's own sources, they cost more registers than they save)
            constexpr bool ahead = PIPE && FUSED_PREFETCH_RING;
            if constexpr (NST > 0) {
                typename Buf<S>::R *ps = pst + ((p - z0) & 1) * NST * TL::NT + threadIdx.x;
                Unroll<0, NST>::run([&](auto I) { ps[I * TL::NT] = praw[I]; });
            }
            source_site_staged<S, TL, true, THIN1>(bF, praw, Tf, Tconst, k, cd, zo + ixy, ibidx, bs, lds[slot], iidx, keep);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < NRING; j++) {
                if (threadIdx.x + j * TL::NT < TL::NH) {
                    if constexpr (!ahead) {
                        const int roff = (zo + rxy[j]) * SB;
                        Unroll<0, Q>::run([&](auto I) { rraw[j][I] = bF.template loadraw<I>(roff); });
                    }
                    SiteState<C> dummy;
                    source_site_staged<S, TL, false, THIN1>(bF, rraw[j], Tf, Tconst, k, cd, zo + rxy[j], rbidx[j], bs,
                                                     lds[slot], rlidx[j], dummy);
                }
            }
        }
    };
    auto fill = [&](int p, int slot, SiteState<C> &keep) {
        fill_issue(p);
        fill_compute(p, slot, keep, bslot(p - 1), bslot(p), bslot(p + 1));
    };

    // gradient, collision and push of plane z from the source slots (sm, s0, sp)
    auto final_plane = [&](int z, int sm, int s0, int sp, SiteState<C> &cur) {
        __builtin_amdgcn_sched_barrier(0);
        if (!inside) return;
        const int wz = wrapc(z, g.nz);
        const int zc = wz * nxy;
        C d[Q];
        if constexpr (NST > 0) {
            // the first NST as the source evaluation of this plane left them in LDS, the rest
            // read again (issued early, consumed after the gradient).  It is the last use of
            // those lines, so in single precision they are read non-temporally, leaving L2 to
            // the ring and staging reads, which are shared (+1.7%; no measurable effect in 2-byte
            // storage, which keeps the default policy)
            constexpr int POL = S == 1 ? 2 : 0;
            const typename Buf<S>::R *ps = pst + ((z - z0) & 1) * NST * TL::NT + threadIdx.x;
            const int off = (zc + ixy) * SB;
            Unroll<0, Q>::run([&](auto I) {
                if constexpr (I < NST) d[I] = bF.template decode<I, 0>(ps[I * TL::NT], cd);
                else d[I] = bF.template decode<I, 0>(bF.template loadraw<I, POL>(off), cd);
            });
        } else {
            load_pops<S>(bF, (zc + ixy) * SB, cd, d);  // issued early, consumed after the gradient
        }
        GradAcc<C> acc;
        grad_init(acc);
        C Fv[3], Sv[6];
        if constexpr (THIN1) {
            // One z plane: the +-z pair at the site itself cancels, and the two z edges at an
            // in-plane axis offset read the site the face there reads (their z parts cancel,
            // the in-plane parts double); 8 in-plane neighbours, directions 1-4 and 7-10.
            const C *p0 = lds[s0] + iidx;
            Unroll<1, 11>::run([&](auto I) {
                if constexpr (I != 5 && I != 6) {
                    constexpr int off = EY[I] * TL::HX + EX[I];
                    C sv[NSRC];
#pragma unroll
                    for (int c = 0; c < NSRC; c++) sv[c] = p0[c * NS + off];
                    grad_add<C, I, HASK>(acc, sv, k.K);
                    if constexpr (I % GRAD_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
                }
            });
            grad_finish_thin(acc, Fv, Sv);
        } else {
            const C *pm = lds[sm] + iidx, *p0 = lds[s0] + iidx, *pp = lds[sp] + iidx;
            Unroll<1, Q>::run([&](auto I) {
                constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
                const C *pl = ez < 0 ? pm : (ez > 0 ? pp : p0);
                constexpr int off = ey * TL::HX + ex;
                C sv[NSRC];
#pragma unroll
                for (int c = 0; c < NSRC; c++) sv[c] = pl[c * NS + off];
                grad_add<C, I, HASK>(acc, sv, k.K);
                if constexpr (I % GRAD_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
            });
            grad_finish(acc, Fv, Sv);
        }
        const PopMoments<C> m = pop_moments(d, k.rho_ref);
        if constexpr (FORCE) {
            const int s = zc + ixy;
            C a[3];
            site_accel(k, accel, g.n, s, a);
            add_body_force(m, a, Fv, Sv);
        }
        collide(d, cur.beta, m, Fv, Sv, cur.theta, k);
        int Zo[3];
        Zo[0] = (wz == 0 ? g.nz - 1 : wz - 1) * nxy;
        Zo[1] = zc;
        Zo[2] = (wz == g.nz - 1 ? 0 : wz + 1) * nxy;
        Unroll<0, Q>::run([&](auto I) {
            const int t = Zo[EZ[I] + 1] + Yo[EY[I] + 1] + Xo[EX[I] + 1];
            bFo.template storef<I, 0>(t * SB, d[I], cd, amax);
        });
        const int so = (zc + ixy) * SB;
        Unroll<0, NB>::run([&](auto c) { bBo.template storef<c, Q>(so, cur.beta[c], cd, amax); });
    };

    SiteState<C> sa, sb;
    if constexpr (THIN1) {
        stage(0, 0);
        __syncthreads();
        fill(0, 0, sa);
        __syncthreads();
        final_plane(0, 0, 0, 0, sa);
    } else if (thin) {
        for (int q = 0; q < g.nz; q++) stage(q, q);
        __syncthreads();
        fill(0, 0, sa);
        if (g.nz == 2) fill(1, 1, sb);
        __syncthreads();
        final_plane(0, g.nz == 1 ? 0 : 1, 0, g.nz == 1 ? 0 : 1, sa);
        if (g.nz == 2) final_plane(1, 0, 1, 0, sb);
    } else {
        stage(z0 - 2, bslot(z0 - 2));
        stage(z0 - 1, bslot(z0 - 1));
        stage(z0, bslot(z0));
        __syncthreads();
        fill(z0 - 1, 2, sb);  // source slot of plane p is (p - z0 + 3) % 3; sb is scratch here
        __syncthreads();
        stage(z0 + 1, bslot(z0 + 1));  // overwrites the slot of z0 - 2
        __syncthreads();
        fill(z0, 0, sa);
        if constexpr (PIPE) {  // the loads the first iteration consumes
            stage_issue(z0 + 2);
            fill_issue(z0 + 1);
        }
        __syncthreads();
        // one plane: stage z+2, sources of z+1 into `nxt`, then the final of z from `cur`; the
        // global loads of the staging and the sources are issued one iteration ahead.  Plane q's
        // staging slot and source slot are both (q - z0) mod 3.
        auto iter = [&](int z, SiteState<C> &cur, SiteState<C> &nxt) {
            const int m = (z - z0) % 3, m1 = (m + 1) % 3, m2 = (m + 2) % 3;
            const bool more = z + 1 < z1;
            // the staged slot is that of plane z-1, whose last gather was for plane z
            if constexpr (PIPE) {
                stage_commit(m2);
                if (more) stage_issue(z + 3);
            } else {
                stage(z + 2, m2);
            }
            __syncthreads();
            if constexpr (PIPE) {
                fill_compute(z + 1, m1, nxt, m, m1, m2);
                if (more) fill_issue(z + 2);
            } else {
                fill_issue(z + 1);
                fill_compute(z + 1, m1, nxt, m, m1, m2);
            }
            __syncthreads();
            final_plane(z, m2, m, m1, cur);
            // No barrier here: the next staging overwrites the bbar* slot of plane z, last read
            // by this iteration's fill (before the barrier above), and the next fill overwrites
            // the source slot of plane z-1, last read by this final, which the next iteration's
            // first barrier separates from it.
        };
        for (int z = z0; z < z1; z++) {
            iter(z, sa, sb);
            sa = sb;
        }
    }
    // the LDS may be reused at once by the next tile of a persistent work-group
    __syncthreads();
}

// Overflow check of the 16-bit codes a thread stored: rm holds the largest |value| stored into
// each array, and a code overflowed (was stored as +-inf) exactly when its scaled value reached the
// rounding midpoint above the largest finite code.  Scaling the maximum once gives the maximum of
// the scaled values, since rounding a product is monotone in the factor; a NaN does not enter it.
template <int S>
__device__ __forceinline__ void report_range(const RangeMax &rm, const Codec &cd, unsigned *flag) {
    if constexpr (S == 2) {
        if (rm.f * cd.inv[0] >= HALF_OVERFLOW || rm.b * cd.inv[Q] >= HALF_OVERFLOW) *flag = 1u;
    } else if constexpr (S == 3) {
        if (fmaxf(rm.f, rm.b) >= bf16_overflow()) *flag = 1u;
    }
}

#ifndef FUSED_WAVES_PER_EU
#define FUSED_WAVES_PER_EU 2
#endif

// Occupancy: the LDS (159 KB of 160 KB with the kept populations) admits one 512-thread
// work-group per CU, i.e. two waves per SIMD.  FORCE: with a body force (the field accel, or
// the uniform acceleration of the step constants).
template <int S, bool GATHERED, bool HASK, bool THIN1, bool FORCE>
__global__ void __launch_bounds__(TileFor<S>::type::NT) __attribute__((amdgpu_waves_per_eu(FUSED_WAVES_PER_EU)))
k_fused(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
        typename Storage<S>::T *__restrict__ Fo, typename Storage<S>::T *__restrict__ Bo,
        const typename Storage<S>::C *__restrict__ Tf, typename Storage<S>::C Tconst, Geo g,
        StepConst<typename Storage<S>::C> k, Codec cd, unsigned *__restrict__ flag, FusedGeo fg,
        const typename Storage<S>::C *__restrict__ accel) {
    // XCD-aware work-group numbering: the work-groups of one XCD (block index mod 8) take
    // neighbouring tiles of the same z chunk
    const int nblk = gridDim.x;
    int L = blockIdx.x;
    if ((nblk & 7) == 0) L = (L & 7) * (nblk >> 3) + (L >> 3);
    const int tx = L % fg.tiles_x;
    L /= fg.tiles_x;
    const int ty = L % fg.tiles_y;
    const int chunk = L / fg.tiles_y;
    RangeMax amax;
    sweep_tile<S, GATHERED, HASK, THIN1, typename TileFor<S>::type, THIN1 ? 0 : fused_stash<S>(), FORCE>(
        F, B, Fo, Bo, Tf, Tconst, g, k, cd, fg, tx, ty, chunk, amax, accel);
    report_range<S>(amax, cd, flag);
}

// Tiles of the xy plane times z chunks.  `slots` is the number of work-groups resident at once
// (one per CU: each takes more than half of a CU's LDS).  A chunk costs its planes plus about
// two of warm-up, and the work-groups run in ceil(blocks / slots) rounds, so the chunk count
// minimises rounds x (chunk + 2): one round with all CUs marching in step through their chunk
// is best (neighbouring tiles then share their halo rings in L2 at the same time).  Chunks keep
// at least 16 planes.
template <typename TL> inline FusedGeo fused_geometry_t(const Geo &g, int slots) {
    FusedGeo fg;
    fg.tiles_x = (g.nx + TL::TX - 1) / TL::TX;
    fg.tiles_y = (g.ny + TL::TY - 1) / TL::TY;
    const int nz = g.nz;
    const long long tiles = (long long)fg.tiles_x * fg.tiles_y;
    if (nz <= 2) {
        fg.nchunks = 1;
        fg.zchunk = nz;
        return fg;
    }
    if (slots < 1) slots = 1;
    const int maxc = nz / 16 > 0 ? nz / 16 : 1;
    int best = 1;
    long long best_cost = -1;
    for (int nch = 1; nch <= maxc; nch++) {
        const long long zc = (nz + nch - 1) / nch;
        const long long rounds = (tiles * nch + slots - 1) / slots;
        const long long cost = rounds * (zc + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = nch;
        }
    }
    fg.zchunk = (nz + best - 1) / best;
    fg.nchunks = (nz + fg.zchunk - 1) / fg.zchunk;
    return fg;
}

template <int S> inline FusedGeo fused_geometry(const Geo &g, int slots) {
    return fused_geometry_t<typename TileFor<S>::type>(g, slots);
}

// Every buffer-resource group (PPG planes) must stay below 4 GiB.
template <int S> inline bool fused_supported_s(const Geo &g) {
    return (unsigned long long)Buf<S>::PPG * (unsigned long long)g.n * sizeof(typename Storage<S>::T) < (1ull << 32);
}
inline bool fused_supported(const Geo &g, int storage) {
    switch (storage) {
    case 0: return fused_supported_s<0>(g);
    case 1: return fused_supported_s<1>(g);
    case 2: return fused_supported_s<2>(g);
    default: return fused_supported_s<3>(g);
    }
}

}  // namespace lbm
