// lbm_server.hip -- continuous batching of many independent lattices on one GPU.
//
// Device side: k_serve, a persistent kernel (one work-group per CU) that walks a packed index
// of (lattice, tile) entries and sweeps each tile for one step with the same per-tile code as
// the single-lattice fused kernel.  Per-lattice descriptors (buffers, shape, step constants,
// codec, which buffer holds the state, steps still to take) live in device memory, so the graph
// that captures K launches of k_serve (step 0..K-1 of a bundle) stays valid while lattices come
// and go: only the tables change between replays.
//
// Host side: a worker thread admits queued requests first-fit in arrival order while they fit
// the device-memory budget (a request's first step, from its gathered initial state, runs with
// lbm_step at admission), replays the bundle graph over all resident lattices, retires those
// whose steps are done (health check, moments to host, memory freed), and timestamps each
// request.  Requests submitted while a bundle runs wait at most one bundle for admission.
//
// A one-plane request without transverse velocity is served as a projected D2Q9 lattice (lbm_set_projection): the same step on 18 (THERMAL) or 12 (ISO) values
// per site instead of 25, swept by k_serve_proj.  Its result is what the same lattice stepped
// alone with that projection gives, to the bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_fused.hpp"
#include "lbm_internal.hpp"
#include "lbm_proj.hpp"

using namespace lbm;

namespace {

struct ServeDesc {
    const void *F[2];
    const void *B[2];
    const float *Tf;
    float Tconst;
    int cur0;        // buffer holding the state at the start of the bundle
    int steps_left;  // steps this lattice takes in the bundle at most
    Geo g;
    FusedGeo fg;
    StepConst<float> k;
    unsigned *flag;  // the lattice's own range flag
    Codec cd;
    int proj;        // 1: a projected D2Q9 lattice (k_serve_proj)
};

struct TileRef {
    int lat;   // descriptor index
    int tile;  // (chunk * tiles_y + ty) * tiles_x + tx
};

#ifndef SERVE_THIN_WAVES_PER_EU
#define SERVE_THIN_WAVES_PER_EU 4
#endif
template <int S, bool THIN1>
using ServeTile = typename std::conditional<THIN1, typename ThinTileFor<S>::type, typename TileFor<S>::type>::type;

template <int S, bool THIN1>
__global__ void __launch_bounds__((ServeTile<S, THIN1>::NT))
    __attribute__((amdgpu_waves_per_eu(THIN1 ? SERVE_THIN_WAVES_PER_EU : FUSED_WAVES_PER_EU)))
k_serve(const ServeDesc *__restrict__ descs, const TileRef *__restrict__ tiles, const int *__restrict__ ntiles,
        int step) {
    using T = typename Storage<S>::T;
    // the table lists the tiles of one-plane lattices first: [0, ntiles[0]) for THIN1, then
    // [ntiles[0], ntiles[1]) for the rest
    const int lo = THIN1 ? 0 : ntiles[0];
    const int hi = THIN1 ? ntiles[0] : ntiles[1];
    for (int t = lo + (int)blockIdx.x; t < hi; t += (int)gridDim.x) {
        const TileRef e = tiles[t];
        const ServeDesc &d = descs[e.lat];
        if (step >= d.steps_left) continue;  // this lattice is done for the bundle
        const int cur = (d.cur0 + step) & 1;
        int L = e.tile;
        const int tx = L % d.fg.tiles_x;
        L /= d.fg.tiles_x;
        const int ty = L % d.fg.tiles_y;
        const int chunk = L / d.fg.tiles_y;
        RangeMax amax;
        sweep_tile<S, false, true, THIN1, ServeTile<S, THIN1>>((const T *)d.F[cur], (const T *)d.B[cur], (T *)d.F[1 - cur], (T *)d.B[1 - cur],
                                   d.Tf, d.Tconst, d.g, d.k, d.cd, d.fg, tx, ty, chunk, amax);
        report_range<S>(amax, d.cd, d.flag);
    }
}

// Projected D2Q9 lattices: tiles [ntiles[1], ntiles[2]) of the table.  The per-tile step
// and the tiles are those of the one-launch kernel of a lattice stepped alone, so the results
// agree to the bit: which sites of a tile are ring sites decides how the compiler may fuse their
// source arithmetic, so another tile shape would change the last bit.
using ProjServeTile = ProjTile<2>;
template <int S>
__global__ void __launch_bounds__(ProjServeTile::NT)
k_serve_proj(const ServeDesc *__restrict__ descs, const TileRef *__restrict__ tiles, const int *__restrict__ ntiles,
             int step) {
    using TL = ProjServeTile;
    using T = typename Storage<S>::T;
    __shared__ float lsrc[ProjSet<2>::NSP * TL::HN];
    __shared__ float lb[ProjLayout<2, true>::NBP * TL::BN];
    for (int t = ntiles[1] + (int)blockIdx.x; t < ntiles[2]; t += (int)gridDim.x) {
        const TileRef e = tiles[t];
        const ServeDesc &d = descs[e.lat];
        if (step >= d.steps_left) continue;  // this lattice is done for the bundle (uniform)
        const int cur = (d.cur0 + step) & 1;
        const int bx = e.tile % d.fg.tiles_x, by = e.tile / d.fg.tiles_x;
        const T *F = (const T *)d.F[cur], *B = (const T *)d.B[cur];
        T *Fo = (T *)d.F[1 - cur], *Bo = (T *)d.B[1 - cur];
        if (d.k.iso)
            proj_tile_step<S, 2, false, false, TL>(F, B, Fo, Bo, d.Tf, d.Tconst, d.g, d.k, d.cd, bx, by, lsrc, lb,
                                                   d.flag);
        else
            proj_tile_step<S, 2, true, false, TL>(F, B, Fo, Bo, d.Tf, d.Tconst, d.g, d.k, d.cd, bx, by, lsrc, lb,
                                                  d.flag);
        __syncthreads();  // the next tile reuses the LDS
    }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    long id = 0;
    lbm_params p{};
    long n_steps = 0;
    long steps_left = 0;
    std::vector<double> rho, u, T;  // inputs (host, double), then outputs
    int status = LBM_REQ_QUEUED;
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t bytes = 0;
    lbm_handle lat = nullptr;
    std::string error;
};

}  // namespace

struct lbm_server {
    lbm_server_params prm{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int grid = 0;       // persistent work-groups of the general kernel
    int grid_thin = 0;  // persistent work-groups of the one-plane kernel
    int grid_proj = 0;  // persistent work-groups of the projected kernel

    std::mutex mu;
    std::condition_variable cv;       // worker wake-up
    std::condition_variable done_cv;  // request completion
    std::deque<long> queue;
    std::map<long, Request> reqs;  // node-based: a Request's address is stable
    std::vector<Request *> active;
    long next_id = 1;
    size_t resident = 0;
    bool stop = false;
    std::thread worker;

    // device tables
    ServeDesc *d_desc = nullptr;
    TileRef *d_tiles = nullptr;
    int *d_ntiles = nullptr;
    int tile_cap = 0;
    std::vector<ServeDesc> h_desc;
    std::vector<TileRef> h_tiles;
    bool tables_dirty = true;
    int n_thin = 0, n_all = 0, n_proj_end = 0;   // tile counts of the current table
    bool graph_thin = false, graph_gen = false, graph_proj = false;  // kernels the bundle launches
    hipGraphExec_t graph = nullptr;

    // counters
    double bundles = 0, updates = 0, busy_s = 0;
    long n_done = 0, n_failed = 0;
};

namespace {

template <typename Fn> int dispatch_serve(int storage, Fn &&fn) {
    switch (storage) {
    case LBM_F32: return fn(std::integral_constant<int, 1>{});
    case LBM_F16DEV: return fn(std::integral_constant<int, 2>{});
    case LBM_BF16DEV: return fn(std::integral_constant<int, 3>{});
    }
    return LBM_ERR_ARG;
}

void fail_request(lbm_server *s, Request &r, const std::string &msg) {
    r.status = LBM_REQ_FAILED;
    r.error = msg;
    r.t_done = now_s();
    r.rho.clear();
    r.u.clear();
    r.T.clear();
    s->n_failed++;
}

// A request is served as a projected D2Q9 lattice when the lattice is one plane with no
// transverse velocity.
bool serve_projected(const lbm_server *s, const Request &r) {
    (void)s;
    if (r.p.nz != 1 || r.p.mode == LBM_STANDARD) return false;
    const size_t n = (size_t)r.p.nx * r.p.ny;
    for (size_t i = 0; i < n; i++)
        if (r.u[2 * n + i] != 0.0) return false;
    return true;
}

// Admit queued requests that fit (first fit, arrival order).  Called by the worker, unlocked
// while HIP work runs.
void admit(lbm_server *s) {
    std::vector<long> cand;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        size_t room = s->prm.hbm_budget_bytes > s->resident ? s->prm.hbm_budget_bytes - s->resident : 0;
        int slots = s->prm.max_lattices - (int)s->active.size();
        for (auto it = s->queue.begin(); it != s->queue.end() && slots > 0;) {
            Request &r = s->reqs[*it];
            if (r.bytes <= room) {
                room -= r.bytes;
                slots--;
                cand.push_back(*it);
                it = s->queue.erase(it);
            } else {
                ++it;
            }
        }
        for (long id : cand) s->resident += s->reqs[id].bytes;
    }
    for (long id : cand) {
        Request *r;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r = &s->reqs[id];
        }
        lbm_params p = r->p;
        p.storage = s->prm.storage;
        lbm_handle h = nullptr;
        const bool proj = serve_projected(s, *r);
        int rc = lbm_create(&p, s->stream, &h);
        if (!rc && proj) rc = lbm_set_projection(h, 2);
        if (!rc) rc = lbm_set_fields(h, r->rho.data(), r->u.data(), r->T.data(), LBM_DTYPE_F64, 0);
        if (!rc && !proj) rc = lbm_set_kernel(h, 2);
        if (!rc) rc = lbm_step(h, 1);  // from the gathered initial state
        std::string err = rc ? lbm_last_error() : "";
        std::lock_guard<std::mutex> lk(s->mu);
        if (rc) {
            if (h) lbm_destroy(h);
            s->resident -= r->bytes;
            fail_request(s, *r, "admission: " + err);
            s->done_cv.notify_all();
            continue;
        }
        r->lat = h;
        r->steps_left = r->n_steps - 1;
        r->t_admit = now_s();
        r->status = LBM_REQ_RUNNING;
        r->rho.clear();
        r->u.clear();
        r->T.clear();
        s->active.push_back(r);
        s->tables_dirty = true;
    }
}

int upload_tables(lbm_server *s) {
    // descriptors are refreshed every bundle (buffer parity and steps left change)
    s->h_desc.clear();
    if (s->tables_dirty) s->h_tiles.clear();
    for (size_t a = 0; a < s->active.size(); a++) {
        Request &r = *s->active[a];
        lbm_lattice *h = r.lat;
        ServeDesc d{};
        d.F[0] = h->F[0];
        d.F[1] = h->F[1];
        d.B[0] = h->B[0];
        d.B[1] = h->B[1];
        d.Tf = (const float *)h->Tf;
        d.Tconst = (float)h->Tconst;
        d.cur0 = h->cur;
        d.steps_left = (int)std::min<long>(r.steps_left, s->prm.bundle_steps);
        d.g = Geo{h->p.nx, h->p.ny, h->p.nz, h->n};
        d.proj = h->proj < 3 ? 1 : 0;
        if (d.proj) {
            d.fg = FusedGeo{(h->p.nx + ProjServeTile::TX - 1) / ProjServeTile::TX,
                            (h->p.ny + ProjServeTile::TY - 1) / ProjServeTile::TY, 1, 1};
        } else {
            dispatch_serve(s->prm.storage, [&](auto SI) -> int {
                constexpr int S = decltype(SI)::value;
                d.fg = d.g.nz == 1 ? fused_geometry_t<ServeTile<S, true>>(d.g, s->grid_thin)
                                   : fused_geometry_t<ServeTile<S, false>>(d.g, s->grid);
                return 0;
            });
        }
        d.k = step_const<float>(h);  // the constants lbm_step uses
        d.flag = h->flag;
        d.cd = h->codec;
        s->h_desc.push_back(d);
    }
    if (s->tables_dirty) {
        // tiles of one-plane lattices first (the one-plane kernel), then the other D3Q19 ones,
        // then the projected ones
        for (int pass = 0; pass < 3; pass++) {
            for (size_t a = 0; a < s->h_desc.size(); a++) {
                const ServeDesc &d = s->h_desc[a];
                const int kind = d.proj ? 2 : (d.g.nz == 1 ? 0 : 1);
                if (kind != pass) continue;
                const int nt = d.fg.tiles_x * d.fg.tiles_y * d.fg.nchunks;
                for (int t = 0; t < nt; t++) s->h_tiles.push_back(TileRef{(int)a, t});
            }
            if (pass == 0) s->n_thin = (int)s->h_tiles.size();
            if (pass == 1) s->n_all = (int)s->h_tiles.size();
        }
        s->n_proj_end = (int)s->h_tiles.size();
        const int nt = s->n_proj_end;
        if (nt > s->tile_cap) {
            if (s->graph) {
                (void)hipGraphExecDestroy(s->graph);
                s->graph = nullptr;  // the tile table moves: capture again
            }
            if (s->d_tiles) (void)hipFree(s->d_tiles);
            s->tile_cap = std::max(nt, 2 * s->tile_cap);
            if (hipMalloc(&s->d_tiles, sizeof(TileRef) * s->tile_cap) != hipSuccess) return LBM_ERR_OOM;
        }
        if (nt && hipMemcpyAsync(s->d_tiles, s->h_tiles.data(), sizeof(TileRef) * nt, hipMemcpyHostToDevice, s->stream) != hipSuccess)
            return LBM_ERR_HIP;
        const int counts[3] = {s->n_thin, s->n_all, s->n_proj_end};
        if (hipMemcpyAsync(s->d_ntiles, counts, sizeof(counts), hipMemcpyHostToDevice, s->stream) != hipSuccess)
            return LBM_ERR_HIP;
        // the copy reads a stack array: make it complete before it goes out of scope
        if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_ERR_HIP;
        // a bundle launches only the kernels with tiles to sweep
        const bool want_thin = s->n_thin > 0, want_gen = s->n_all > s->n_thin, want_proj = s->n_proj_end > s->n_all;
        if (s->graph && (want_thin != s->graph_thin || want_gen != s->graph_gen || want_proj != s->graph_proj)) {
            (void)hipGraphExecDestroy(s->graph);
            s->graph = nullptr;
        }
        s->tables_dirty = false;
    }
    if (!s->h_desc.empty() &&
        hipMemcpyAsync(s->d_desc, s->h_desc.data(), sizeof(ServeDesc) * s->h_desc.size(), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
        return LBM_ERR_HIP;
    return LBM_OK;
}

int capture_graph(lbm_server *s) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LBM_ERR_HIP;
    const bool thin = s->n_thin > 0, gen = s->n_all > s->n_thin, proj = s->n_proj_end > s->n_all;
    int rc = dispatch_serve(s->prm.storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        for (int st = 0; st < s->prm.bundle_steps; st++) {
            if (thin)
                hipLaunchKernelGGL((k_serve<S, true>), dim3(s->grid_thin), dim3(ServeTile<S, true>::NT), 0, s->stream, s->d_desc,
                                   s->d_tiles, s->d_ntiles, st);
            if (gen)
                hipLaunchKernelGGL((k_serve<S, false>), dim3(s->grid), dim3(ServeTile<S, false>::NT), 0, s->stream, s->d_desc,
                                   s->d_tiles, s->d_ntiles, st);
            if (proj)
                hipLaunchKernelGGL((k_serve_proj<S>), dim3(s->grid_proj), dim3(ProjServeTile::NT), 0, s->stream,
                                   s->d_desc, s->d_tiles, s->d_ntiles, st);
        }
        return LBM_OK;
    });
    s->graph_thin = thin;
    s->graph_gen = gen;
    s->graph_proj = proj;
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return LBM_ERR_HIP;
    }
    e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

// Health check (non-finite values, rho <= 0, 16-bit overflow) of a running lattice; at
// completion also the readout.  A failing lattice is removed and its request marked FAILED.
void retire(lbm_server *s, Request &r, bool check_only) {
    long counts[2] = {0, 0};
    double umax = 0;
    // lbm_health reads and clears the 16-bit overflow flag: LBM_ERR_RANGE, before DIVERGED
    const int hc = lbm_health(r.lat, counts, &umax);
    const bool range = hc == LBM_ERR_RANGE;
    if (hc != LBM_OK) {
        // A binary16 code past its largest finite value means a deviation grew 1024-fold beyond
        // the largest initial one, which in practice is a diverging run; a bfloat16 code is
        // flagged only when the value itself is no longer finite.
        const std::string sites = std::to_string(counts[0]) + " non-finite sites, " +
                                  std::to_string(counts[1]) + " sites with rho <= 0";
        std::string msg = range && s->prm.storage == LBM_F16DEV ? "16-bit encode saturated (diverging or out of range): " + sites
                          : range || hc == LBM_ERR_DIVERGED     ? "diverged: " + sites
                                                                : std::string("health check: ") + lbm_last_error();
        lbm_destroy(r.lat);
        r.lat = nullptr;
        std::lock_guard<std::mutex> lk(s->mu);
        s->resident -= r.bytes;
        fail_request(s, r, msg);
        s->active.erase(std::find(s->active.begin(), s->active.end(), &r));
        s->tables_dirty = true;
        s->done_cv.notify_all();
        return;
    }
    if (check_only) return;
    const size_t n = (size_t)r.p.nx * r.p.ny * r.p.nz;
    std::vector<double> rho(n), u(3 * n), T(n);
    int rc = lbm_get_moments(r.lat, rho.data(), u.data(), T.data(), LBM_DTYPE_F64, 0);
    std::string err = rc ? lbm_last_error() : "";
    lbm_destroy(r.lat);
    r.lat = nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    s->resident -= r.bytes;
    s->active.erase(std::find(s->active.begin(), s->active.end(), &r));
    s->tables_dirty = true;
    if (rc) {
        fail_request(s, r, "readout: " + err);
    } else {
        r.rho.swap(rho);
        r.u.swap(u);
        r.T.swap(T);
        r.status = LBM_REQ_DONE;
        r.t_done = now_s();
        s->n_done++;
    }
    s->done_cv.notify_all();
}

void worker_loop(lbm_server *s) {
    (void)hipSetDevice(s->device);
    while (true) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->active.empty(); });
            if (s->stop) break;
        }
        admit(s);
        if (s->active.empty()) {
            // nothing admissible right now (queue waits for memory held by no one cannot happen:
            // oversize requests are refused at submit), wait for the next submission
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        int rc = upload_tables(s);
        if (!rc && !s->graph) rc = capture_graph(s);
        const double t0 = now_s();
        if (!rc && hipGraphLaunch(s->graph, s->stream) != hipSuccess) rc = LBM_ERR_HIP;
        if (!rc && hipStreamSynchronize(s->stream) != hipSuccess) rc = LBM_ERR_HIP;
        const double t1 = now_s();
        if (rc) {
            // a device or runtime error: fail every running request and stop serving them
            std::string msg = std::string("bundle failed: ") + hipGetErrorString(hipGetLastError());
            std::vector<Request *> act;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                act = s->active;
            }
            for (Request *rp : act) {
                Request &r = *rp;
                if (r.lat) lbm_destroy(r.lat);
                r.lat = nullptr;
                std::lock_guard<std::mutex> lk(s->mu);
                s->resident -= r.bytes;
                fail_request(s, r, msg);
            }
            std::lock_guard<std::mutex> lk(s->mu);
            s->active.clear();
            s->tables_dirty = true;
            s->done_cv.notify_all();
            continue;
        }
        s->bundles += 1;
        s->busy_s += t1 - t0;
        // account the steps each lattice took and retire the finished ones
        std::vector<Request *> act;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            act = s->active;
        }
        for (Request *rp : act) {
            Request &r = *rp;
            const long taken = std::min<long>(r.steps_left, s->prm.bundle_steps);
            lbm_lattice *h = r.lat;
            h->cur = (int)((h->cur + taken) & 1);
            h->steps += taken;
            h->gathered = false;
            r.steps_left -= taken;
            s->updates += (double)taken * h->n;
            if (r.steps_left == 0) {
                retire(s, r, false);
            } else if (s->prm.health_every > 0 && ((long)s->bundles % s->prm.health_every) == 0) {
                retire(s, r, true);
            }
        }
    }
}

}  // namespace

extern "C" {

int lbm_server_create(const lbm_server_params *p, void *hip_stream, lbm_server_handle *out) {
    if (!p || !out) return set_error(LBM_ERR_ARG, "null argument");
    *out = nullptr;
    if (p->bundle_steps < 1 || p->max_lattices < 1 || p->hbm_budget_bytes == 0)
        return set_error(LBM_ERR_ARG, "bundle_steps, max_lattices and the budget must be positive");
    if (p->storage != LBM_F32 && p->storage != LBM_F16DEV && p->storage != LBM_BF16DEV)
        return set_error(LBM_ERR_ARG, "the server serves F32, F16DEV or BF16DEV storage");
    lbm_server *s = new (std::nothrow) lbm_server();
    if (!s) return set_error(LBM_ERR_OOM, "host allocation");
    s->prm = *p;
    (void)hipGetDevice(&s->device);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    if (cus <= 0) cus = 256;
    s->grid = cus;  // the general kernel's LDS admits one 512-thread work-group per CU
    // the one-plane kernel: as many work-groups per CU as its registers and LDS admit
    int per_cu = 0;
    (void)dispatch_serve(p->storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_serve<S, true>, ServeTile<S, true>::NT, 0) !=
            hipSuccess)
            per_cu = 1;
        return 0;
    });
    s->grid_thin = cus * (per_cu > 0 ? per_cu : 1);
    int per_cu_proj = 0;
    (void)dispatch_serve(p->storage, [&](auto SI) -> int {
        constexpr int S = decltype(SI)::value;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_proj, k_serve_proj<S>, ProjServeTile::NT, 0) !=
            hipSuccess)
            per_cu_proj = 1;
        return 0;
    });
    s->grid_proj = cus * (per_cu_proj > 0 ? per_cu_proj : 1);
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return set_error(LBM_ERR_HIP, "stream creation");
        }
        s->own_stream = true;
    }
    hipError_t e = hipMalloc(&s->d_desc, sizeof(ServeDesc) * p->max_lattices);
    if (e == hipSuccess) e = hipMalloc(&s->d_ntiles, 3 * sizeof(int));
    if (e == hipSuccess) e = hipMemset(s->d_ntiles, 0, 3 * sizeof(int));
    if (e != hipSuccess) {
        lbm_server_destroy(s);
        return set_error(LBM_ERR_OOM, "server tables");
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return LBM_OK;
}

int lbm_server_submit(lbm_server_handle s, const lbm_params *p, const void *rho, const void *u, const void *T,
                      int dtype, long n_steps, long *req_id) {
    if (!s || !p || !rho || !u || !T || !req_id) return set_error(LBM_ERR_ARG, "null argument");
    if (n_steps < 1) return set_error(LBM_ERR_ARG, "n_steps must be >= 1");
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return set_error(LBM_ERR_ARG, "unknown dtype");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->tau > 0) || !(p->rho_ref > 0) ||
        (p->mode != LBM_THERMAL && p->mode != LBM_ISO))
        return set_error(LBM_ERR_ARG, "bad lattice parameters");
    lbm_params q = *p;
    q.storage = s->prm.storage;
    const size_t bytes = lbm_lattice_bytes(&q);
    if (bytes == 0 || bytes > s->prm.hbm_budget_bytes)
        return set_error(LBM_ERR_ARG, "the lattice alone exceeds the server's memory budget");
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    Request r;
    r.p = q;
    r.n_steps = n_steps;
    r.bytes = bytes;
    r.rho.resize(n);
    r.u.resize(3 * n);
    r.T.resize(n);
    auto copy_in = [&](std::vector<double> &dst, const void *src, size_t m) {
        if (dtype == LBM_DTYPE_F64) {
            std::memcpy(dst.data(), src, sizeof(double) * m);
        } else {
            const float *f = (const float *)src;
            for (size_t i = 0; i < m; i++) dst[i] = f[i];
        }
    };
    copy_in(r.rho, rho, n);
    copy_in(r.u, u, 3 * n);
    copy_in(r.T, T, n);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r.id = s->next_id++;
        r.t_submit = now_s();
        *req_id = r.id;
        s->queue.push_back(r.id);
        s->reqs.emplace(r.id, std::move(r));
    }
    s->cv.notify_all();
    return LBM_OK;
}

int lbm_server_poll(lbm_server_handle s, long req_id, int *status, double times[3]) {
    if (!s) return set_error(LBM_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return set_error(LBM_ERR_ARG, "unknown request");
    if (status) *status = it->second.status;
    if (times) {
        times[0] = it->second.t_submit;
        times[1] = it->second.t_admit;
        times[2] = it->second.t_done;
    }
    return LBM_OK;
}

int lbm_server_wait(lbm_server_handle s, long req_id, double timeout_s) {
    if (!s) return set_error(LBM_ERR_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto pred = [&] {
        auto it = s->reqs.find(req_id);
        return it == s->reqs.end() || it->second.status == LBM_REQ_DONE || it->second.status == LBM_REQ_FAILED;
    };
    if (!s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
        return set_error(LBM_ERR_BUSY, "request not finished within the timeout");
    if (s->reqs.find(req_id) == s->reqs.end()) return set_error(LBM_ERR_ARG, "unknown request");
    return LBM_OK;
}

int lbm_server_fetch(lbm_server_handle s, long req_id, void *rho, void *u, void *T, int dtype) {
    if (!s) return set_error(LBM_ERR_ARG, "null server");
    if (dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_F32) return set_error(LBM_ERR_ARG, "unknown dtype");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return set_error(LBM_ERR_ARG, "unknown request");
    Request &r = it->second;
    if (r.status != LBM_REQ_DONE) return set_error(LBM_ERR_STATE, "request not done");
    auto copy_out = [&](void *dst, const std::vector<double> &src) {
        if (!dst) return;
        if (dtype == LBM_DTYPE_F64) {
            std::memcpy(dst, src.data(), sizeof(double) * src.size());
        } else {
            float *f = (float *)dst;
            for (size_t i = 0; i < src.size(); i++) f[i] = (float)src[i];
        }
    };
    copy_out(rho, r.rho);
    copy_out(u, r.u);
    copy_out(T, r.T);
    return LBM_OK;
}

int lbm_server_release(lbm_server_handle s, long req_id) {
    if (!s) return set_error(LBM_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return set_error(LBM_ERR_ARG, "unknown request");
    if (it->second.status != LBM_REQ_DONE && it->second.status != LBM_REQ_FAILED)
        return set_error(LBM_ERR_STATE, "request still queued or running");
    s->reqs.erase(it);
    return LBM_OK;
}

const char *lbm_server_error(lbm_server_handle s, long req_id) {
    if (!s) return "";
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    return it == s->reqs.end() ? "" : it->second.error.c_str();
}

int lbm_server_stats(lbm_server_handle s, double out[8]) {
    if (!s || !out) return set_error(LBM_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = (double)s->resident;
    out[1] = (double)s->active.size();
    out[2] = (double)s->queue.size();
    out[3] = (double)s->n_done;
    out[4] = (double)s->n_failed;
    out[5] = s->bundles;
    out[6] = s->updates;
    out[7] = s->busy_s;
    return LBM_OK;
}

void lbm_server_destroy(lbm_server_handle s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->reqs)
        if (kv.second.lat) lbm_destroy(kv.second.lat);
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_tiles) (void)hipFree(s->d_tiles);
    if (s->d_ntiles) (void)hipFree(s->d_ntiles);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
