/*
 * lbm.h -- C ABI of liblbm, the MI355X (gfx950) implementation of the bump-function D3Q19
 * lattice Boltzmann step of Afrasiabian & Denniston, "A Novel Velocity Discretization for
 * Lattice Boltzmann Method: Application to Compressible Flow" (arXiv:2501.00620).
 *
 * The operation behind every entry point is one time step of Sec. II C of the paper: the
 * populations fbar_i and the variance bbar of the bump functions (Eqs. 49-50, 62-66) are
 * relaxed by the single-relaxation-time update (Eq. 55) towards the equilibria of Appendix A,
 * with the forcing of Eqs. 58-61 built from isotropic finite differences of rho*b and
 * rho*u*b, and then streamed along the D3Q19 velocities with bbar carried by the arriving
 * populations (Eq. 66).  Lattice units throughout: dx = dt = c = 1, periodic in x, y and z.
 *
 * Conventions shared by all calls
 *  - Fields are structure of arrays, x fastest: a scalar field is nz*ny*nx values, C order
 *    (z, y, x); a vector field is 3 such planes (x, y, z components); the population state is
 *    19 planes in the paper's velocity order (rows 2-4 of Table I); bbar is 6 planes in the
 *    order xx, yy, zz, xy, xz, yz.
 *  - Pointers are plain addresses.  `on_device` = 1: device pointers on the lattice's GPU
 *    (e.g. torch CUDA tensors' data_ptr()); 0: host pointers.
 *  - Ownership: the library owns all lattice memory.  The caller owns every buffer it passes and
 *    may reuse it once the call returns; calls that read or write caller buffers finish that
 *    access (on the lattice's stream, synchronised) before returning.
 *  - Streams: each lattice runs on the HIP stream given at creation (NULL = the null stream).
 *    lbm_step is asynchronous on that stream; the other calls synchronise it before returning.
 *  - Errors: every int-returning call returns LBM_OK (0) or a negative code below; a readable
 *    message for the calling thread is available from lbm_last_error().  No C++ exception
 *    crosses this interface.  Handles are not thread-safe; the server is internally locked.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_ERR_ARG (-1)      /* bad size, tau <= 0, rho <= 0, unknown enum, NULL pointer   */
#define LBM_ERR_OOM (-2)      /* device allocation failed                                    */
#define LBM_ERR_HIP (-3)      /* HIP runtime error; message carries the runtime's string     */
#define LBM_ERR_DIVERGED (-4) /* non-finite value or rho <= 0 found by a health check        */
#define LBM_ERR_RANGE (-5)    /* a 16-bit deviation code overflowed (stored as +-inf)       */
#define LBM_ERR_BUSY (-6)     /* server: request queued, not admitted yet (not a failure)   */
#define LBM_ERR_STATE (-7)    /* call out of order (e.g. step before set_fields)            */

/* Storage precision of the populations and bbar in device memory.  F64 computes in double;
 * the others compute in float.  F16DEV / BF16DEV store 16-bit deviations
 * h = (value - ref) / scale from a reference equilibrium (ref_i = w_i rho_ref for the
 * populations, (T_ref - 1/3) delta for bbar), with one power-of-two scale per stored array
 * (the populations; bbar), fixed when the fields or the state are set.  Every kernel encodes
 * with round-to-nearest-even; a value whose code would exceed the largest finite one is stored
 * as +-inf (never clamped) and sets the lattice's range flag, which lbm_set_fields,
 * lbm_set_state and lbm_health report as LBM_ERR_RANGE (and clear). */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16DEV = 2, LBM_BF16DEV = 3 } lbm_storage;

/* Temperature closure.  THERMAL: T from the total second-moment trace of the bump expansion
 * (Eq. 26), so mass, momentum and energy are conserved.  ISO: T is the prescribed per-site field
 * given to lbm_set_fields (the paper's setting in all its experiments); mass and momentum are
 * conserved.  STANDARD: the standard lattice Boltzmann comparator the paper contrasts with its
 * scheme (Sec. I, Eq. 4; Sec. III C): populations without a variance, the second-order Hermite
 * equilibrium feq_i = rho w_i [1 + 3 e.u + 9/2 (u u + (T - 1/3) I):(e e - I/3)] at the prescribed
 * T, BGK with the same omega = 1/(tau + 1/2); bbar stays at its reference.  Not served. */
typedef enum { LBM_THERMAL = 0, LBM_ISO = 1, LBM_STANDARD = 2 } lbm_mode;

/* Field dtypes accepted by set_fields / get_moments. */
typedef enum { LBM_DTYPE_F64 = 0, LBM_DTYPE_F32 = 1 } lbm_dtype;

typedef struct {
    int nx, ny, nz;     /* lattice size, each >= 1; nx*ny*nz <= 2^31 - 1                   */
    double tau;         /* relaxation time of Eq. 55 in units of dt; omega = 1/(tau + 1/2) */
    double T_ref;       /* reference temperature of the deviation codec (usually 1/3)      */
    double rho_ref;     /* reference density of the deviation codec (usually 1)            */
    int storage;        /* lbm_storage                                                      */
    int mode;           /* lbm_mode                                                         */
} lbm_params;

typedef struct lbm_lattice *lbm_handle;

/* Allocate a lattice on the current HIP device.  `hip_stream` is a hipStream_t (may be NULL).
 * Device memory: 2 x (19 + 6) values of the storage type per site (lbm_lattice_bytes gives the
 * total).  Errors: ARG, OOM, HIP. */
int lbm_create(const lbm_params *p, void *hip_stream, lbm_handle *out);

/* Initialise from macroscopic fields (Sec. II B, Appendix A): fbar_i = feq_i(rho, u),
 * bbar = beq(u, T) at every site (STANDARD: the Hermite equilibrium of Eq. 4 at T, bbar at its
 * reference).  rho: n values, u: 3n, T: n, all of `dtype`.  In ISO and STANDARD mode T is also
 * kept as the prescribed temperature field.  For 16-bit storage the codec scales are
 * chosen here from the initial deviations.  Errors: ARG (rho <= 0 or non-finite anywhere),
 * RANGE (an initial value overflowed its code), HIP. */
int lbm_set_fields(lbm_handle h, const void *rho, const void *u, const void *T, int dtype,
                   int on_device);

/* Advance n_steps time steps (Sec. II C) on the lattice's stream; asynchronous.
 * Errors: ARG (n_steps < 0), STATE (no fields set), HIP. */
int lbm_step(lbm_handle h, long n_steps);

/* Read the macroscopic moments of the current state: rho = sum fbar (Eq. 56), the corrected
 * velocity of Eq. 57, and T (the corrected THERMAL temperature, or the prescribed ISO field).
 * STANDARD: rho, u = sum f e / rho and the prescribed T.
 * rho: n, u: 3n, T: n values of `dtype`.  Any pointer may be NULL to skip that field. */
int lbm_get_moments(lbm_handle h, void *rho, void *u, void *T, int dtype, int on_device);

/* Checkpoint / parity: the post-stream state (fbar: 19n doubles, bbar: 6n doubles; on a projected
 * lattice the nf and nb planes of lbm_get_projection, get only), decoded to double.
 * lbm_set_state loads such a state (re-encoding it; codec scales are re-chosen for 16-bit
 * storage).  get then set then step continues the run: the checkpoint holds bbar gathered, which
 * the uninterrupted run gathers inside its next step in another order of summation, so the two
 * agree to the rounding of that sum (about 1e-16 relative in F64, 1e-7 in F32), not bit for bit.
 * Two runs from the same state are bit-identical. */
int lbm_get_state(lbm_handle h, void *F, void *b, int on_device);
int lbm_set_state(lbm_handle h, const void *F, const void *b, int on_device);

/* Deviation codec (16-bit storage only): the 25 power-of-two scales and the 25 references
 * (19 populations, then bbar xx yy zz xy xz yz) as doubles.  Decoding is ref + scale * h.
 * A D3Q19 lattice has one scale for the 19 populations and one for the 6 bbar components
 * (unit scales for BF16DEV); the entries repeat them per field.
 * Errors: ARG for F64/F32 storage or NULL pointers. */
int lbm_get_codec(lbm_handle h, double *scales25, double *refs25);

/* Raw stored 16-bit codes (16-bit storage only), right after lbm_set_state or lbm_set_fields
 * (before any step): 19n codes of the populations and 6n codes of bbar, as uint16.
 * Errors: ARG for F64/F32 storage, STATE after a step (bbar is then held in its pre-gather
 * form). */
int lbm_get_raw(lbm_handle h, void *F_codes, void *b_codes, int on_device);

/* The stored representation, decoded to double: F = the post-stream populations (19n, as
 * lbm_get_state) and b = bbar in the form it is held in (6n): gathered bbar(x) right after
 * set_fields / set_state, otherwise the post-collision bbar*(x) of the last step, before it is
 * carried along with the populations (Eq. 66).  *b_is_gathered reports which.  Exact for every
 * storage (no re-association), so it is what a 16-bit path is checked on element by element. */
int lbm_get_stored(lbm_handle h, void *F, void *b, int *b_is_gathered, int on_device);

/* Global invariants in double precision (wavefront, block, then a fixed-order second pass, so
 * the result is deterministic): out[0] mass, out[1..3] momentum sum fbar e, out[4] energy
 * 1/2 sum (sum_i fbar_i |e_i|^2 + rho tr bbar). */
int lbm_invariants(lbm_handle h, double out[5]);

/* For callers that cannot allocate device memory or wait (code under HIP graph capture, serving
 * loops, hosts that forbid hipMalloc): the 5 values of lbm_invariants, bit for bit, computed
 * without any device allocation.
 *  - on_device = 1: out is a device pointer to 5 doubles on the lattice's GPU; the call only
 *    enqueues the reduction on the lattice's stream and returns (no synchronisation).
 *  - on_device = 0: out is host memory; the call waits for the result.
 * The partial sums live in one static scratch array per GPU (256 KiB, held until the process
 * ends) whose size does not depend on the lattice: at most 1024 work-groups stride over it.
 * Every call on a GPU shares that array, so calls that overlap on one GPU (from other streams
 * or threads) race.  Errors: ARG (null pointer, projected lattice), STATE, HIP. */
int lbm_invariants_noalloc(lbm_handle h, double *out, int on_device);

/* Health check: counts of sites with a non-finite stored value and with rho <= 0, and the
 * largest |u*| (uncorrected velocity).  counts and max_u are filled in whatever the result.
 * Returns LBM_ERR_RANGE if a 16-bit code overflowed since the state was set or last checked
 * (the flag is then cleared), else LBM_ERR_DIVERGED if either count is nonzero. */
int lbm_health(lbm_handle h, long counts[2], double *max_u);

/* Per-step launch configuration. kernel: 0 = auto, 1 = two-pass (predictor sources to a
 * buffer, then gradient + collision), 2 = fused z-marching sweep with LDS planes of sources
 * (every wave does every part of the step), 3 = the same sweep split between producer waves
 * (predictor sources) and consumer waves (gradient, collision, stream) of one work-group, for
 * float and 16-bit storage on lattices with nz >= 3.  All give the same step up to the order of
 * the gradient sums.  Auto takes the split sweep where it applies (from the second step after
 * the state was set; the first gathers bbar in the single-role sweep, or two-pass with walls), a
 * ghost rate, a body force and walls included; else the single-role fused sweep, for a periodic
 * single-rate lattice (with or without a body force) whose buffers fit their 32-bit offsets; else
 * the two-pass step.  With walls the split sweep steps the interior planes 1 .. nz-2, and the two
 * wall planes step with the two-pass wall kernel in the same lbm_step.
 * Errors: ARG (bad choice; a fused sweep on a projected lattice or beyond its offsets; the
 * single-role sweep with walls or a ghost rate; the split sweep in double precision or below 3
 * planes). */
int lbm_set_kernel(lbm_handle h, int kernel);

/* Relaxation time of the nine non-hydrodynamic moments, rows 11-19 of Table I (Appendix B):
 * with a collision matrix diagonal in that basis (the general form of the update the paper
 * reduces to Eq. 55), these moments relax with omega_g = 1/(tau_ghost + 1/2) while rows 1-10
 * keep omega = 1/(tau + 1/2).  tau_ghost = tau restores the single-rate scheme.  A lattice with
 * its own ghost rate steps with the split fused sweep (float and 16-bit storage, nz >= 3) or the
 * two-pass kernel.  Errors: ARG (tau_ghost <= 0 or non-finite, STANDARD mode, or the single-role
 * fused kernel forced by lbm_set_kernel(h, 2)). */
int lbm_set_ghost_relaxation(lbm_handle h, double tau_ghost);

/* Body-force acceleration field: 3n values of `dtype` (x, y, z planes, x fastest), or NULL to
 * remove it.  It enters the forcing moments of Eqs. 58-61 as F += rho a and S += rho (u a + a u)
 * with the corrected velocity of Eq. 57, which then carries half of rho a (a Guo-type forcing;
 * the paper drives its Poiseuille and Couette flows with a body force, Sec. III A and C).  In
 * the STANDARD mode the same F and S build the forcing, with u = (j + rho a / 2) / rho.  The
 * field is copied (3 planes of the compute type on the device).  Both kernels take it: the
 * fused sweep adds it to the forcing moments of each site before the collision, as the two-pass
 * collision does.  Errors: ARG (dtype, projected lattice), OOM, HIP. */
int lbm_set_body_force(lbm_handle h, const void *accel, int dtype, int on_device);

/* A uniform body-force acceleration: accel is a host array of 3 values (x, y, z), or NULL to remove
 * the body force; it replaces a field set by lbm_set_body_force (and that call replaces it).  The
 * same forcing as a field holding the vector at every site, bit for bit, without the field's
 * device memory or its 3 reads per site (the paper's channels are driven by a uniform force).
 * Errors: ARG (non-finite value, projected lattice). */
int lbm_set_body_force_uniform(lbm_handle h, const double *accel);

/* Walls normal to z (the channels of Sec. III A and C): on = 1 places one wall half-way below
 * plane 0 and one half-way above plane nz - 1 (z = -1/2 and nz - 1/2); x and y stay periodic.
 * u_bottom, u_top: host arrays of 3 wall velocities (NULL: at rest); the z components must be 0.
 * A population that would stream through a wall returns reversed to its site (half-way
 * bounce-back) carrying the moving-wall momentum of Ladd, 6 w_i rho e_i.u_w, and the site's own
 * variance.  Beyond a wall the gradient sources of Eqs. 59 and 61 take the wall-adjacent
 * plane's rho b (mirrored) and the second-order extrapolation of rho b u*.  on = 0 restores the
 * periodic z direction.  Applies to every mode.  A float or 16-bit lattice with walls steps its
 * interior planes with the split fused sweep and its two wall planes with the two-pass wall
 * kernel (lbm_set_kernel); double precision steps two-pass.  Errors: ARG (nz < 3, a normal or
 * non-finite wall velocity, the single-role fused kernel forced by lbm_set_kernel(h, 2)). */
int lbm_set_walls(lbm_handle h, int on, const double *u_bottom, const double *u_top);

/* Projected lattice (the lower-dimensional bump lattices that Sec. II B illustrates with D1Q3):
 * the same step for flows that do not vary along z (dims = 2: nz = 1, a D2Q9 lattice) or along
 * y and z (dims = 1: ny = nz = 1, D1Q3), held as class sums.  dims = 3 restores the D3Q19 layout.
 * - Class sums: F_c = sum of the populations that share the in-plane velocity c.  In THERMAL
 *   mode also G_c = the same sum weighted by |e_t|^2, the squared transverse speed.
 * - Variance: the in-plane components of bbar; in THERMAL mode also the trace of its transverse
 *   block.
 * The step is exact: it reproduces the D3Q19 step of such a flow to rounding, since every
 * update is linear per population and reads only moments the class sums carry.
 * Per site the state is 12 values (D2Q9, ISO), 18 (D2Q9, THERMAL), 4 (D1Q3, ISO) or 8
 * (D1Q3, THERMAL), in place of 25.  The call frees the state (set_fields again) and
 * reallocates the buffers.
 * Supports: modes THERMAL and ISO; every storage (F16DEV takes one scale per plane, chosen at
 * lbm_set_fields from the class-summed bound of the initial deviations); lbm_set_fields (the
 * transverse velocity must be 0), lbm_step, lbm_get_moments (transverse u = 0),
 * lbm_get_state (see lbm_get_projection for its layout) and lbm_health.  lbm_set_state,
 * lbm_get_stored, lbm_invariants, walls, body force, a ghost rate and the fused kernel return
 * ARG.
 * Errors: ARG (dims, lattice shape, mode, one of those settings), OOM, HIP. */
int lbm_set_projection(lbm_handle h, int dims);

/* The projection of a lattice and its lbm_get_state layout.
 * - *dims: 3 (D3Q19), 2 or 1.
 * - *nf: planes written to F; *nb: planes written to b.
 * - Projected F holds the class sums F_c, then (THERMAL) the G_c of the classes with transverse
 *   members.  D2Q9 classes: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (1,-1) (-1,1) (-1,-1); the
 *   first five have G.  D1Q3 classes: 0, +1, -1, all with G.
 * - Projected b holds xx yy xy [zz] (D2Q9) or xx [yy+zz] (D1Q3).
 * Any pointer may be NULL.  Errors: ARG (null handle). */
int lbm_get_projection(lbm_handle h, int *dims, int *nf, int *nb);

/* Block until all work queued on the lattice's stream is done. */
int lbm_sync(lbm_handle h);
void lbm_destroy(lbm_handle h);

/* Message of the last failing call on this thread ("" if none). */
const char *lbm_last_error(void);

/* Steps taken since the last set_fields / set_state. */
long lbm_steps_done(lbm_handle h);

/* Device bytes a lattice with these parameters occupies (what lbm_create allocates).  A lattice
 * that steps two-pass (lbm_set_kernel(h, 1), or a ghost rate in double precision or below 3
 * planes) or has walls allocates 9 more planes of the compute type at its first such step. */
size_t lbm_lattice_bytes(const lbm_params *p);

/* ---------------------------------------------------------------------------------------------
 * Serving: continuous batching of many independent lattices on one GPU.
 *
 * A one-plane request (nz = 1) without transverse velocity is held as a projected D2Q9 lattice
 * (lbm_set_projection).  Its result is what that lattice gives stepped
 * alone with the projection, to the bit; every other request is what the D3Q19 lattice gives
 * stepped alone with the fused kernel.
 *
 * Requests (each an initial state and a step count) are queued by lbm_server_submit and
 * admitted, first fit in arrival order, whenever their lattice fits the device-memory budget
 * next to the lattices already resident.  All resident lattices advance together: a persistent
 * kernel walks a packed index of (lattice, tile) pairs and applies the same step as lbm_step to
 * each tile (the first step of a request runs at admission), and bundles of K such steps are
 * replayed from one captured HIP graph.  A lattice whose steps are done leaves the bundle at
 * its own step count, is health-checked, its moments (as lbm_get_moments) are copied to host
 * memory, and its device memory is released for the queue.  Requests that arrive while others
 * run are admitted between bundles.  A request's result does not depend on what else is being
 * served (the per-site arithmetic is the same as stepping it alone).
 *
 * The server runs a worker thread; its calls are thread-safe.  Every served lattice uses the
 * server's storage; F32, F16DEV and BF16DEV are supported.
 * ------------------------------------------------------------------------------------------- */
typedef struct lbm_server *lbm_server_handle;

#define LBM_REQ_QUEUED 0  /* waiting for device memory                          */
#define LBM_REQ_RUNNING 1 /* resident, being stepped                             */
#define LBM_REQ_DONE 2    /* finished; results can be fetched                    */
#define LBM_REQ_FAILED 3  /* rejected or diverged; see lbm_server_error           */

typedef struct {
    size_t hbm_budget_bytes; /* device memory the resident lattices may occupy together   */
    int bundle_steps;        /* K, steps per captured graph replay (>= 1)                  */
    int storage;             /* lbm_storage of the served lattices: F32, F16DEV, BF16DEV    */
    int max_lattices;        /* most lattices resident at once (descriptor table size)     */
    int health_every;        /* bundles between health checks of running lattices (0: only
                                at completion)                                            */
} lbm_server_params;

/* Create a server on the current device and the given HIP stream (NULL: a stream of its own).
 * Errors: ARG, OOM, HIP. */
int lbm_server_create(const lbm_server_params *p, void *hip_stream, lbm_server_handle *out);

/* Queue a request.  p->storage is ignored (the server's storage is used).  rho (n), u (3n) and
 * T (n) are host arrays of `dtype`; they are copied before the call returns.  n_steps >= 1.
 * *req_id receives the request's id.  Errors: ARG (bad parameters, or a lattice larger than
 * the whole budget). */
int lbm_server_submit(lbm_server_handle s, const lbm_params *p, const void *rho, const void *u, const void *T,
                      int dtype, long n_steps, long *req_id);

/* Status of a request and its times in seconds on a monotonic clock: times[0] submitted,
 * times[1] admitted (0 if not yet), times[2] finished (0 if not yet). */
int lbm_server_poll(lbm_server_handle s, long req_id, int *status, double times[3]);

/* Block until the request is DONE or FAILED, or timeout_s elapses (returns LBM_ERR_BUSY). */
int lbm_server_wait(lbm_server_handle s, long req_id, double timeout_s);

/* Copy a finished request's moments (rho n, u 3n, T n of `dtype`, host memory; any may be
 * NULL).  Errors: STATE if not DONE. */
int lbm_server_fetch(lbm_server_handle s, long req_id, void *rho, void *u, void *T, int dtype);

/* Forget a finished request (frees its host copy of the results). */
int lbm_server_release(lbm_server_handle s, long req_id);

/* Message of a FAILED request. */
const char *lbm_server_error(lbm_server_handle s, long req_id);

/* Counters: out[0] resident bytes, [1] running, [2] queued, [3] done, [4] failed, [5] bundles
 * run, [6] lattice updates done by bundles, [7] seconds spent in bundles (device + sync). */
int lbm_server_stats(lbm_server_handle s, double out[8]);

/* Stop the worker (running requests are abandoned) and free everything. */
void lbm_server_destroy(lbm_server_handle s);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
