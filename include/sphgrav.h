/*
 * sphgrav.h -- C ABI of libsphgrav.so: the per-timestep force evaluation of
 * self-gravitating SPH with direct (Particle-Particle) gravity, after
 * Khrapov & Khoperskov, "Smoothed-Particle Hydrodynamics Models:
 * Implementation Features on GPUs" (CCIS 793, 2017), on one AMD Instinct
 * MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Particles: N = N_g + N_h (Sec. 2.1).  Gas (SPH) particles occupy indices
 *   [0, N_g), collisionless halo particles [N_g, N).
 * - Memory: every buffer handed to the library is DEVICE memory owned by the
 *   caller, laid out as structure-of-arrays of FP64.  The library never
 *   allocates or frees device memory: its scratch lives in one caller-owned
 *   workspace blob sized by sg_workspace_bytes().  Host-side it allocates
 *   only the small opaque context.
 * - Streams: the caller owns them.  All work is enqueued on the HIP
 *   stream given to sg_create(); entry points return as soon as the work
 *   is enqueued.  Only sg_status_sync(), sg_export(), sg_profile_read(),
 *   sg_run(), sg_ensemble_create(), sg_ensemble_run() and the destroy calls
 *   wait for streams.  Inside a step the neighbour/SPH chain runs on the
 *   caller's second (auxiliary) stream when one was given, beside the
 *   gravity on the main stream: forked from the main stream and joined back
 *   into it before the step's last kernels, so every step stays ordered on
 *   the main stream (and can be captured from it).  The library creates only the events of those forks and joins,
 *   and, for an ensemble given no chain stream, one CU-masked stream
 *   (sg_ensemble_create).
 * - Errors: every call returns an sg_status; nothing aborts and no C++
 *   exception crosses the ABI.  Argument errors are detected on the host
 *   before any HIP call.  Conditions only the device can see (capacity
 *   overflow, bad smoothing lengths, non-finite positions) are latched in
 *   a device error word: the affected kernels then do nothing, and the
 *   next sg_status_sync() reports the condition and the capacity
 *   required.
 * - Threading: one context per stream; a context is not thread-safe.
 * - Indices are int32 (N < 2^31); CSR offsets are int64.
 */
#ifndef SPHGRAV_H
#define SPHGRAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SG_OK = 0,
    SG_EINVAL = 1,      /* bad argument (null pointer, size, parameter)        */
    SG_ECAPACITY = 2,   /* a device capacity (cells, neighbour pairs) was too small */
    SG_EDEVICE = 3,     /* a HIP runtime call failed                           */
    SG_ESTATE = 4,      /* call out of order (e.g. density before neighbours)  */
    SG_ENONFINITE = 5,  /* non-finite position or non-positive/non-finite h    */
    SG_ERANGE = 6       /* smoothing lengths span more than SG_MAX_LEVELS levels */
} sg_status;

typedef enum {
    SG_FP64 = 0,        /* all pair arithmetic and sums in FP64                 */
    SG_FP32C = 1        /* FP32 pair arithmetic on anchor-relative coordinates,
                           Kahan-compensated FP32 partial sums; FP64 state,
                           update (drift/kick) and reductions                  */
} sg_precision;

/* Flags of sg_compute_accel() / sg_step(). */
#define SG_SPH  1u      /* hydrodynamic acceleration and de/dt (Eqs. dv_dt-SPH, de_dt-SPH) */
#define SG_GRAV 2u      /* direct gravity (Eq. self-gravity)                      */
#define SG_POT  4u      /* also the gravitational potential (needs SG_GRAV)       */

/* Phases of sg_kick_drift(). */
#define SG_PREDICT 0
#define SG_CORRECT 1

#define SG_MAX_LEVELS 16

/* Physical and tuning parameters.
 * G, eps: gravitational constant and Plummer softening length; the
 *   paper's softened pair force (Eq. self-gravity, whose printed
 *   denominator is read as (|r_ij|^2 + eps^2)^{3/2}); eps must be > 0, and
 *   >= 1e-12 in the SG_FP32C form (so that (r^2 + eps^2)^{-3/2} is finite
 *   in FP32).
 * gamma: adiabatic index of the ideal-gas law (Eq. e_p_rho), > 1.
 * alpha, beta, eta: artificial-viscosity constants (Sec. 2.2), >= 0, eta > 0.
 * precision: an sg_precision value.
 * grav_ipl: target particles per GPU lane in the gravity kernel (1, 2 or 4;
 *   0 = automatic); a workgroup of 256 lanes owns 256 * grav_ipl targets.
 *   grav_split: number of source-range splits (>= 1; 0 = automatic).
 *   grav_tile: sources per LDS tile of the gravity kernels (128, 256 or
 *   512; 0 = automatic: 256 for SG_FP32C, 512 for SG_FP64).  None of the
 *   three changes results beyond summation order.
 * grav_variant: 0 = automatic.  FP64 form: 1 = pair differences, reciprocal
 *   square root seeded in FP32 and refined in FP64 (needs eps^2 >=
 *   1.2e-38), 2 = pair differences, seeded in FP64 (both refined to FP64
 *   rounding level); 3 (FP32 seed, needs eps^2 >= 1.2e-38) and 4 (FP64
 *   seed) = Morton-ordered particles with the far field expanded about a
 *   per-workgroup anchor, as the FP32C kernel does, in FP64 (4 is the
 *   automatic choice).  FP32C form: 1 (the only kernel).
 * cell_scale_log2: side of the neighbour-search cells relative to the
 *   default rule, as a power of two (-1, 0 or +1; 0 = default).  Each gas
 *   particle keeps its level (the first l with L0 * 2^l >= (2 + 2^-9) h_i,
 *   L0 the smallest power of two >= (2 + 2^-9) min h); level-l cells get the
 *   side L0 * 2^(l + cell_scale_log2).  It changes cell keys, counts,
 *   offsets and the slot order (so the exported grid arrays and the order
 *   of SPH sums), never which particles are neighbours.
 * step_serial: 0 = in a step, the neighbours -> density -> SPH(corrector)
 *   chain runs on the context's auxiliary stream beside the gravity
 *   (default);
 *   1 = the two one after the other on the context's stream (for kernel
 *   traces whose per-kernel durations should not include waiting beside
 *   the gravity kernel).  Results are the same either way, bit for bit.
 * grav_reorder: gravity preparations per recomputation of the Morton order
 *   that the SG_FP32C and expanded-FP64 kernels visit particles in (0 or
 *   1 = every preparation, at most 1024).  In between, the order is
 *   reused: the sorted copies and the 64-particle boxes are still rebuilt
 *   from the current positions, so the near/far choice and its error bound
 *   hold for any order; a stale order only makes the boxes less compact
 *   (more near-field pairs).  Results depend on the period at rounding
 *   level (other groupings); runs with one period are reproducible bit
 *   for bit, eager or graph-captured (sg_run, sg_ensemble_run). */
typedef struct {
    double G, eps, gamma, alpha, beta, eta;
    int32_t precision;
    int32_t grav_ipl;
    int32_t grav_split;
    int32_t grav_variant;
    int32_t grav_tile;
    int32_t cell_scale_log2;
    int32_t step_serial;
    int32_t grav_reorder;
} sg_params;

/* Capacities the workspace is sized for.
 * n_gas_cap, n_halo_cap: maximum N_g and N_h of any bound state.
 * cell_cap: maximum number of grid cells M (sum over levels).
 * nnz_cap: maximum number of (ordered) neighbour pairs. */
typedef struct {
    int64_t n_gas_cap, n_halo_cap, cell_cap, nnz_cap;
} sg_caps;

/* Device pointers of the particle state (caller-owned, FP64, SoA).
 * Inputs/updated state: x,y,z,vx,vy,vz,m [N]; h,e [N_g].
 * Outputs: ax,ay,az [N] total acceleration (SPH + gravity for gas, gravity
 * for halo), dedt [N_g], rho [N_g]; pot [N] may be NULL unless SG_POT is
 * requested. */
typedef struct {
    double *x, *y, *z, *vx, *vy, *vz, *m;
    double *h, *e;
    double *ax, *ay, *az;
    double *dedt, *rho;
    double *pot;
} sg_state;

typedef struct sg_ctx sg_ctx;   /* opaque */

/* Bytes of device workspace needed for these parameters and capacities.
 * Returns 0 if the arguments are invalid. */
size_t sg_workspace_bytes(const sg_params *prm, const sg_caps *caps);

/* Create a context over a caller-owned workspace of ws_bytes bytes
 * (>= sg_workspace_bytes, 256-byte aligned) on HIP stream `stream`
 * (a hipStream_t; NULL = the default stream).  aux_stream: a second
 * caller-owned stream (hipStream_t) on which each step runs the
 * neighbour/SPH chain beside the gravity; NULL or equal to `stream`: the
 * two run one after the other on `stream` (as with step_serial).  Both streams and
 * the workspace must outlive the context (sg_destroy waits for both
 * streams).  Enqueues a clear of the device status.  On failure *out is
 * NULL and sg_last_error(NULL) says why. */
sg_status sg_create(const sg_params *prm, const sg_caps *caps, void *d_workspace,
                    size_t ws_bytes, void *stream, void *aux_stream, sg_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): sg_create with
 * the library's own workspace instead of a caller-owned one.  The
 * workspace is a device array of SG_STATIC_WS_BYTES bytes inside the
 * library, one per GPU (the current device at the call), held until the
 * process ends; this call allocates nothing (no hipMalloc, no host heap,
 * no stream or event).  At most one such context may exist per GPU at a
 * time (SG_ESTATE otherwise; sg_destroy frees the slot), since all of them
 * would share that array, which keeps the last context's contents: the
 * status word and grid record are cleared here, and everything else is
 * written before it is read.  Calls on it that overlap (from several host
 * threads) race.
 * SG_ECAPACITY, with a message, when sg_workspace_bytes(prm, caps) exceeds
 * SG_STATIC_WS_BYTES (64 MiB: with the Python binding's default
 * capacities, up to 11939 gas + 11939 halo particles); SG_EINVAL as
 * sg_create for bad parameters.  Steps run the gravity and the
 * neighbour/SPH chain one after the other on `stream` (no auxiliary
 * stream).  Every other entry point works on the context as on one from
 * sg_create. */
#define SG_STATIC_WS_BYTES (64ull << 20)
sg_status sg_create_static(const sg_params *prm, const sg_caps *caps, void *stream,
                           sg_ctx **out);

/* Bind a particle state (the "upload" step: the state already sits in
 * device memory owned by the caller).  n_gas <= n_gas_cap, n_halo <=
 * n_halo_cap, n_gas + n_halo >= 1.  Invalidates cached neighbours, density
 * and forces. */
sg_status sg_bind_state(sg_ctx *ctx, int64_t n_gas, int64_t n_halo, const sg_state *st);

/* Grid sort and neighbour lists of the gas at the current positions
 * (Sec. 3, kernels SP): smoothing-length levels and grid parameters, cell
 * keys, per-cell counts and maximum h, prefix sums for cell offsets,
 * stable particle reorder (ascending particle id inside a cell), and a CSR
 * list, by sorted slot, of every other gas particle j with xi_ij < 2, i.e.
 * |r_ij| < h_i + h_j.  The test is done in FP32 so that lists are exact and
 * reproducible: d = (float)(r_i - r_j) per component (FP64 difference
 * rounded once), r2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx)),
 * c = (float)h_i + (float)h_j, neighbour iff r2 < c*c.
 * Grid: levels l = 0,1,.. of cubic cells of side L_l = L_0 2^(l + s)
 * (s = cell_scale_log2, 0 by default), L_0 the smallest power of two >=
 * (2 + 2^-9) min h; particle i sits on the first level with L_0 2^l >=
 * (2 + 2^-9) h_i; each level covers the bounding box of its own particles
 * from origin floor(min/L_l) L_l; keys run level by level, then z, y, x
 * (x fastest).  Device-side conditions (cells or neighbour pairs beyond
 * the capacities, non-finite positions, h <= 0, more than SG_MAX_LEVELS
 * levels) are latched and reported by the next sg_status_sync. */
sg_status sg_build_neighbors(sg_ctx *ctx);

/* SPH density of every gas particle (Eq. SPH-mass-density, self term
 * included, h_ij = (h_i + h_j)/2) into st->rho.  Needs sg_build_neighbors. */
sg_status sg_compute_density(sg_ctx *ctx);

/* Accelerations at the current positions (Eq. dv_dt-SPH): with SG_SPH the
 * pressure + artificial-viscosity sums and de/dt (Eq. de_dt-SPH) over the
 * neighbour lists (needs density); with SG_GRAV the softened direct
 * gravity over all N particles (and with SG_POT the potential).  Writes
 * st->ax/ay/az = latest SPH part + latest gravity, and st->dedt.  After
 * SG_PREDICT the SPH part uses the predicted velocities and energies. */
sg_status sg_compute_accel(sg_ctx *ctx, uint32_t flags);

/* Predictor-corrector update (Sec. 2.2, Eqs. v-predictor .. e-corrector).
 * SG_PREDICT: vt = v + dt a, et = e + dt de/dt (kept in the workspace),
 *   r += dt/2 (vt + v).  SG_CORRECT: v = (v + vt)/2 + dt/2 a,
 *   e = (e + et)/2 + dt/2 de/dt, with a, de/dt evaluated after SG_PREDICT. */
sg_status sg_kick_drift(sg_ctx *ctx, double dt, int32_t phase);

/* One whole step, enqueue-only: [first call: neighbours, density,
 * gravity] -> SPH(predictor) -> SG_PREDICT -> neighbours -> density ->
 * gravity (once per step, reused by the next predictor) -> SPH(corrector)
 * -> SG_CORRECT.  After SG_PREDICT the neighbours -> density ->
 * SPH(corrector) chain runs on the context's auxiliary stream beside the
 * gravity (the two are independent); results equal the sequential order
 * bit for bit.  flags may add SG_POT. */
sg_status sg_step(sg_ctx *ctx, double dt, uint32_t flags);

/* nsteps whole steps (as sg_step) with the conserved quantities of each
 * step written to d_hist[10*k .. 10*k+9] (device, may be NULL).  With
 * use_graph != 0, the first step runs eagerly, then P steady-state steps
 * (step + diagnostics; P = grav_reorder when it is above 1 and the kernel
 * uses the Morton order, else 1: one period of that order's schedule) are
 * captured once into a HIP graph and replayed while P steps remain; the
 * rest run eagerly (dt is fixed inside the graph; stage timing must be
 * off; the context's stream must not be the null stream, which cannot be
 * captured: SG_EINVAL before any work).  Results are identical to nsteps
 * calls of sg_step.  Waits for the stream before returning. */
sg_status sg_run(sg_ctx *ctx, double dt, int64_t nsteps, uint32_t flags, int32_t use_graph,
                 double *d_hist);

/* Time step of Eq. (dt-stability) at the current state into *d_dt (device
 * double): C min_i s_i / (cmax_i (1 + 1.2 alpha) + 1.2 beta mumax_i
 * + sqrt(s_i (|Q_i| + |E_i|))) over gas particles with neighbours, with
 * s_i = min_j |r_ij|, cmax_i = max_j (c_i + c_j)/2, mumax_i = max_j |mu_ij|
 * (mu_ij <= 0 by its definition, so its magnitude is taken), Q_i the total
 * acceleration and E_i = de_i/dt (the square-root term as printed).  +inf
 * if no particle has a neighbour.  Needs neighbours, density and
 * accelerations at the current state (sg_compute_accel with SG_SPH|SG_GRAV,
 * outside a predict/correct pair).  Always FP64. */
sg_status sg_cfl_dt(sg_ctx *ctx, double C, double *d_dt);

/* Smoothing-length update h_i = sigma (m_i / rho_i)^{1/3} (Sec. 2.2) into
 * st->h from the last density.  Invalidates neighbour lists, density and
 * forces. */
sg_status sg_update_h(sg_ctx *ctx, double sigma);

/* Conserved quantities into d_out10 (device, 10 doubles): E_kin, E_int,
 * E_pot (needs SG_POT computed), E_total, momentum (3), angular momentum
 * (3); FP64 sums in a fixed order. */
sg_status sg_diagnostics(sg_ctx *ctx, double *d_out10);

/* What sg_export() copies (device -> device, after a stream sync). */
typedef enum {
    SG_X_KEYS = 0,      /* int32 [N_g] cell key of gas particle i           */
    SG_X_COUNTS = 1,    /* int32 [M]   particles per cell                   */
    SG_X_OFFSETS = 2,   /* int64 [M+1] exclusive prefix sums of COUNTS       */
    SG_X_HMAX = 3,      /* double [M]  largest h in each cell (0 if empty)   */
    SG_X_PERM = 4,      /* int32 [N_g] gas particle stored at sorted slot s  */
    SG_X_NBR_OFF = 5,   /* int64 [N_g+1] CSR row offsets, rows by slot       */
    SG_X_NBR_IDX = 6,   /* int32 [nnz] neighbour slots, ascending per row    */
    SG_X_GRID = 7,      /* sg_grid_info, 1 element                           */
    SG_X_GORDER = 8,    /* int32 [N] gravity target order (SG_FP32C, FP64 grav_variant 3/4) */
    SG_X_ACC_SPH = 9,   /* double [3 N_g] latest SPH part of the acceleration (Eq.
                           dv_dt-SPH): all x, then all y, then all z, by gas
                           particle index; SG_ESTATE before any SG_SPH      */
    SG_X_ACC_GRAV = 10  /* double [3 N] latest gravity part (Eq. self-gravity, G
                           applied), same layout over all particles;
                           SG_ESTATE before any SG_GRAV                     */
} sg_export_what;

/* Host-readable grid description (SG_X_GRID): L0 is the base of the level
 * rule (see cell_scale_log2), L[l] the cell side of level l. */
typedef struct {
    double L0;
    int32_t nlev, pad;
    double L[SG_MAX_LEVELS];
    double org[SG_MAX_LEVELS][3];
    int64_t dim[SG_MAX_LEVELS][3];
    int64_t base[SG_MAX_LEVELS];
    int64_t ncell[SG_MAX_LEVELS];
    int64_t npart[SG_MAX_LEVELS];
    double hmax[SG_MAX_LEVELS];
    int64_t M;
} sg_grid_info;

/* Copy an internal array into caller memory: d_dst (device for arrays,
 * host for SG_X_GRID) of cap_bytes bytes.  *n_out receives the element
 * count.  SG_ECAPACITY if cap_bytes is too small (nothing copied). */
sg_status sg_export(sg_ctx *ctx, int32_t what, void *d_dst, int64_t cap_bytes,
                    int64_t *n_out);

/* Wait for the stream, then report the device error word (and clear it).
 * On SG_ECAPACITY, need[0] = cells required, need[1] = neighbour pairs
 * required (need may be NULL).  SG_ENONFINITE and SG_ERANGE name the other
 * latched conditions; after any of them the cached lists and forces are
 * invalid and the next step rebuilds them. */
sg_status sg_status_sync(sg_ctx *ctx, int64_t need[2]);

/* Ensembles of independent systems (one bound context each, all SG_FP32C,
 * the same G, eps, grav_reorder and stream; SG_EINVAL otherwise).
 * Gravity of all systems runs as ONE persistent launch: workgroups take
 * (system, block of 256 * grav_ipl targets) tasks, largest systems first,
 * from a device counter until none is left; grav_ipl and grav_tile are
 * those of the first context, 0 selecting 2 targets per lane and 512
 * sources per tile for this launch.  Every other per-particle stage of a
 * step (the predictor's SPH pass, the combination of the SPH and gravity
 * parts, predictor and corrector, the Morton order and sorted copies of the
 * gravity inputs, and the corrector's grid, sort, neighbour lists, density
 * and SPH pass) also runs as one launch for all systems, over a device
 * table of the systems' pointers; a stage that only some systems need (a
 * context whose lists are still valid) runs system by system instead.
 * Device-side conditions (capacity overflow, non-finite values) are latched
 * in each context's own status word, as for single contexts: the ensemble
 * calls report only enqueue and host errors, and the caller reads each
 * context's conditions with sg_status_sync(ctx) (after sg_ensemble_run,
 * which has waited already, that call returns at once).
 * The ensemble keeps pointers into the contexts: do not rebind or destroy
 * them while it exists.  d_ws: caller-owned device memory of
 * sg_ensemble_bytes(nsys, total particles), 256-byte aligned; the task and
 * system tables are uploaded once, synchronously, by sg_ensemble_create.
 * chain_stream: the caller's stream (not the contexts' stream) on which the
 * systems' corrector chains run beside the batched gravity, or NULL: then
 * the ensemble creates (and destroys) one stream with every CU in its mask,
 * because a stream of that kind gets a hardware queue of its own, where an
 * ordinary stream may share a queue with the contexts' stream and hold the
 * chains behind the long gravity kernel.  The stream must outlive the
 * ensemble. */
typedef struct sg_ens sg_ens;   /* opaque */
size_t sg_ensemble_bytes(int32_t nsys, int64_t total_particles);
sg_status sg_ensemble_create(sg_ctx *const *ctxs, int32_t nsys, void *d_ws, size_t ws_bytes,
                             void *chain_stream, sg_ens **out);
/* Batched gravity (flags SG_GRAV [| SG_POT]) for every system, then each
 * context's acceleration output is refreshed as in sg_compute_accel. */
sg_status sg_ensemble_gravity(sg_ens *e, uint32_t flags);
/* One predictor-corrector step of every system (as sg_step), gravity
 * batched, on the contexts' stream; after SG_PREDICT the batched gravity
 * runs there while the systems' neighbours -> density -> SPH(corrector)
 * chains run beside it on the chain stream, forked from the contexts'
 * stream before the gravity launch and joined back after the chains.  With
 * step_serial (of the first context) the chains follow the gravity on the
 * contexts' stream.  Results equal those of sg_step on each context alone
 * (same launch shape) bit for bit. */
sg_status sg_ensemble_step(sg_ens *e, double dt, uint32_t flags);
/* nsteps ensemble steps; with use_graph one period of steady-state steps
 * is captured once and replayed (as sg_run).  Waits for the stream. */
sg_status sg_ensemble_run(sg_ens *e, double dt, int64_t nsteps, uint32_t flags, int32_t use_graph);
const char *sg_ensemble_last_error(const sg_ens *e);
void sg_ensemble_destroy(sg_ens *e);

/* Stage timing.  When enabled, every kernel group below is bracketed by a
 * pair of HIP events on the context's stream; sg_profile_read() waits for
 * the stream and returns, per stage, the summed milliseconds and the number
 * of launches since the last enable.  Off by default; do not enable while
 * capturing the stream into a graph. */
typedef enum {
    SG_ST_SORT = 0,       /* levels, keys, counts, offsets, reorder, gather */
    SG_ST_NBR = 1,        /* neighbour count, offsets, fill                  */
    SG_ST_DENSITY = 2,
    SG_ST_SPH = 3,        /* EOS gather + pressure/viscosity sums            */
    SG_ST_GRAV_PREP = 4,  /* FP32C: Morton order, sorted copies, boxes       */
    SG_ST_GRAV = 5,       /* the pair kernel (+ split reduction)             */
    SG_ST_UPDATE = 6,     /* predictor / corrector / combine                 */
    SG_ST_DIAG = 7,
    SG_NSTAGE = 8
} sg_stage;
sg_status sg_profile_enable(sg_ctx *ctx, int32_t on);
sg_status sg_profile_read(sg_ctx *ctx, double ms[SG_NSTAGE], int64_t count[SG_NSTAGE]);

/* Last error message of this context; with ctx == NULL, the reason the
 * calling thread's last sg_create() failed.  Never NULL. */
const char *sg_last_error(const sg_ctx *ctx);

/* Destroy the context (does not free the workspace or the state). */
void sg_destroy(sg_ctx *ctx);

/* Library version and the target architecture it was built for. */
const char *sg_version(void);

#ifdef __cplusplus
}
#endif
#endif
