// lbm_fused.hpp -- single-pass step: z-marching sweep with LDS planes of predictor sources.
//
// One work-group owns an xy tile of FTX x FTY sites and marches through a chunk of z planes.
// The forcing moments at a site need the predictor sources (rho b and u*, Eqs. 59-61 with
// Eq. 68) of its 18 neighbours, and each source needs the site's post-stream populations and
// its gathered bbar (Eq. 66), i.e. one more hop.  Per plane z the work-group
//   A. evaluates the sources of plane z+1 on the tile plus a one-site ring (the ring overlaps
//      the neighbouring tiles) into one of three LDS planes, keeping the tile's own
//      populations, bbar and moments in registers for the next iteration;
//   B. takes the isotropic gradients of plane z from the LDS planes z-1, z, z+1, collides the
//      registers kept from the previous iteration, and pushes the results out.
// Each site's state is read from HBM once per step for its own update (plus the ring, which
// neighbouring tiles on the same XCD usually bring into L2 at about the same time) and written
// once: 2 x 25 values per lattice update, the algorithmic minimum.
//
// Work-groups are numbered so that the ones dispatched to one XCD (block index mod 8) take
// neighbouring tiles of the same z chunk, which share their rings through that XCD's L2.
// Any lattice shape works: tile sites beyond the lattice are computed (wrapped) only as ring
// sources and never stored; nz <= 2 evaluates each plane's sources once and reuses them.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

constexpr int FTX = 64, FTY = 4;
constexpr int FNT = FTX * FTY;      // threads = tile sites
constexpr int FHX = FTX + 2;        // LDS row length with the ring
constexpr int FHY = FTY + 2;
constexpr int FNS = FHX * FHY;      // source sites per LDS plane
constexpr int FNH = FNS - FNT;      // ring sites

#ifndef FUSED_WAVES_PER_EU
#define FUSED_WAVES_PER_EU 2
#endif

struct FusedGeo {
    int tiles_x, tiles_y, nchunks, zchunk;
};

template <typename C> struct SiteState {
    C d[Q];
    C beta[NB];
    PopMoments<C> m;
    C theta;  // prescribed temperature offset (ISO)
};

__device__ __forceinline__ int wrapc(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Sources of one site (global coordinates already wrapped) into an LDS plane; optionally keep
// its state.
template <int S, bool GATHERED, bool KEEP>
__device__ __forceinline__ void source_site(const typename Storage<S>::T *__restrict__ F,
                                            const typename Storage<S>::T *__restrict__ B,
                                            const typename Storage<S>::C *__restrict__ Tf,
                                            typename Storage<S>::C Tconst, const Geo &g,
                                            const StepConst<typename Storage<S>::C> &k, const Codec &cd, int x,
                                            int y, int z, typename Storage<S>::C *plane, int lidx,
                                            SiteState<typename Storage<S>::C> &keep) {
    using C = typename Storage<S>::C;
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    const int s = nb.at(0, 0, 0);
    C d[Q], beta[NB];
    PopMoments<C> m;
    load_site<S, GATHERED>(F, B, g.n, nb, s, cd, k.rho_ref, d, beta, m);
    const C th = site_T(Tf, Tconst, s);
    C o[NSRC];
    predictor_sources(m, beta, th, k, o);
#pragma unroll
    for (int c = 0; c < NSRC; c++) plane[c * FNS + lidx] = o[c];
    if constexpr (KEEP) {
#pragma unroll
        for (int i = 0; i < Q; i++) keep.d[i] = d[i];
#pragma unroll
        for (int c = 0; c < NB; c++) keep.beta[c] = beta[c];
        keep.m = m;
        keep.theta = th;
    }
}

// Occupancy: two waves per SIMD (two 256-thread work-groups per CU) leave 256 VGPRs per lane for
// the two planes of site state and the gradient sums; three would cap it at 168 and spill.
template <int S, bool GATHERED>
__global__ void __launch_bounds__(FNT) __attribute__((amdgpu_waves_per_eu(FUSED_WAVES_PER_EU)))
k_fused(const typename Storage<S>::T *__restrict__ F, const typename Storage<S>::T *__restrict__ B,
        typename Storage<S>::T *__restrict__ Fo, typename Storage<S>::T *__restrict__ Bo,
        const typename Storage<S>::C *__restrict__ Tf, typename Storage<S>::C Tconst, Geo g,
        StepConst<typename Storage<S>::C> k, Codec cd, unsigned *__restrict__ flag, FusedGeo fg) {
    using C = typename Storage<S>::C;
    __shared__ C lds[3][NSRC * FNS];

    // XCD-aware work-group numbering
    const int nblk = gridDim.x;
    int L = blockIdx.x;
    if ((nblk & 7) == 0) L = (L & 7) * (nblk >> 3) + (L >> 3);
    const int tx = L % fg.tiles_x;
    L /= fg.tiles_x;
    const int ty = L % fg.tiles_y;
    const int chunk = L / fg.tiles_y;
    const int z0 = chunk * fg.zchunk;
    const int z1 = min(z0 + fg.zchunk, g.nz);

    const int lx = threadIdx.x % FTX, ly = threadIdx.x / FTX;
    const int x0 = tx * FTX, y0 = ty * FTY;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool inside = gx < g.nx && gy < g.ny;
    const int wx = wrapc(gx, g.nx), wy = wrapc(gy, g.ny);

    // ring site of this thread (second round), if any
    const bool has_ring = threadIdx.x < FNH;
    int rlx = 0, rly = 0;
    {
        const int h = threadIdx.x;
        if (h < FHX) {
            rly = -1;
            rlx = h - 1;
        } else if (h < 2 * FHX) {
            rly = FTY;
            rlx = h - FHX - 1;
        } else if (h < 2 * FHX + FTY) {
            rlx = -1;
            rly = h - 2 * FHX;
        } else {
            rlx = FTX;
            rly = h - 2 * FHX - FTY;
        }
    }
    const int rwx = wrapc(x0 + rlx, g.nx), rwy = wrapc(y0 + rly, g.ny);
    const int ridx = (rly + 1) * FHX + (rlx + 1);
    const int iidx = (ly + 1) * FHX + (lx + 1);

    SiteState<C> cur, nxt;
    const bool thin = g.nz <= 2;

    // sources of plane p (march index, wrapped) into LDS slot `slot`, keeping the tile state
    auto fill = [&](int p, int slot, SiteState<C> &keep) {
        const int wz = wrapc(p, g.nz);
        source_site<S, GATHERED, true>(F, B, Tf, Tconst, g, k, cd, wx, wy, wz, lds[slot], iidx, keep);
        // keep the two source evaluations apart: interleaving them doubles the loads in flight
        // and the registers they hold
        __builtin_amdgcn_sched_barrier(0);
        if (has_ring) {
            SiteState<C> dummy;
            source_site<S, GATHERED, false>(F, B, Tf, Tconst, g, k, cd, rwx, rwy, wz, lds[slot], ridx, dummy);
        }
    };

    if (thin) {
        fill(0, 0, cur);
        if (g.nz == 2) fill(1, 1, nxt);
    } else {
        SiteState<C> dummy;
        fill(z0 - 1, 2, dummy);  // slot of plane p is (p - z0 + 3) % 3
        fill(z0, 0, cur);
    }
    __syncthreads();

    unsigned sat = 0;
    for (int z = z0; z < z1; z++) {
        int sm, s0, sp;  // slots of planes z-1, z, z+1
        if (thin) {
            s0 = z;
            sm = sp = g.nz == 1 ? 0 : 1 - z;
        } else {
            fill(z + 1, (z + 1 - z0 + 3) % 3, nxt);
            __syncthreads();
            sm = (z - 1 - z0 + 3) % 3;
            s0 = (z - z0) % 3;
            sp = (z + 1 - z0) % 3;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (inside) {
            // isotropic gradients of the sources over the 18 neighbours (LDS)
            GradAcc<C> acc;
            grad_init(acc);
            Unroll<1, Q>::run([&](auto I) {
                constexpr int ex = EX[I], ey = EY[I], ez = EZ[I];
                const C *pl = lds[ez < 0 ? sm : (ez > 0 ? sp : s0)];
                const int li = iidx + ey * FHX + ex;
                C sv[NSRC];
#pragma unroll
                for (int c = 0; c < NSRC; c++) sv[c] = pl[c * FNS + li];
                grad_add<C, I>(acc, sv, k.K);
            });
            C Fv[3], Sv[6];
            grad_finish(acc, Fv, Sv);
            collide(cur.d, cur.beta, cur.m, Fv, Sv, cur.theta, k);
            const Nbr nb = make_nbr(wx, wy, wrapc(z, g.nz), g.nx, g.ny, g.nz);
            Unroll<0, Q>::run([&](auto I) {
                Storage<S>::store(Fo, (size_t)I * g.n + nb.at(EX[I], EY[I], EZ[I]), I, cur.d[I], cd, sat);
            });
            const int s = nb.at(0, 0, 0);
#pragma unroll
            for (int c = 0; c < NB; c++) Storage<S>::store(Bo, (size_t)c * g.n + s, Q + c, cur.beta[c], cd, sat);
        }
        cur = nxt;
        __syncthreads();
    }
    if (sat) *flag = 1u;
}

inline FusedGeo fused_geometry(const Geo &g) {
    FusedGeo fg;
    fg.tiles_x = (g.nx + FTX - 1) / FTX;
    fg.tiles_y = (g.ny + FTY - 1) / FTY;
    const int tiles = fg.tiles_x * fg.tiles_y;
    if (g.nz <= 2) {
        fg.nchunks = 1;
        fg.zchunk = g.nz;
        return fg;
    }
    // enough work-groups to fill 256 CUs several times over, chunks of at least 8 planes
    int want = (2048 + tiles - 1) / tiles;
    int maxc = g.nz / 8 > 0 ? g.nz / 8 : 1;
    int nch = want < maxc ? want : maxc;
    if (nch < 1) nch = 1;
    fg.zchunk = (g.nz + nch - 1) / nch;
    fg.nchunks = (g.nz + fg.zchunk - 1) / fg.zchunk;
    return fg;
}

inline bool fused_supported(const Geo &) { return true; }

template <int S>
int launch_fused(const typename Storage<S>::T *F, const typename Storage<S>::T *B, typename Storage<S>::T *Fo,
                 typename Storage<S>::T *Bo, const typename Storage<S>::C *Tf, typename Storage<S>::C Tconst,
                 const Geo &g, const StepConst<typename Storage<S>::C> &k, const Codec &cd, unsigned *flag,
                 bool gathered, hipStream_t stream) {
    const FusedGeo fg = fused_geometry(g);
    const long long blocks = (long long)fg.tiles_x * fg.tiles_y * fg.nchunks;
    if (blocks > 2147483647LL) return -1;
    if (gathered)
        hipLaunchKernelGGL((k_fused<S, true>), dim3((unsigned)blocks), dim3(FNT), 0, stream, F, B, Fo, Bo, Tf, Tconst,
                           g, k, cd, flag, fg);
    else
        hipLaunchKernelGGL((k_fused<S, false>), dim3((unsigned)blocks), dim3(FNT), 0, stream, F, B, Fo, Bo, Tf, Tconst,
                           g, k, cd, flag, fg);
    return 0;
}

}  // namespace lbm
