/*
 * ep.h - C ABI of the MI355X elasto-plastic increment solver (libep.so).
 *
 * The library solves, one load increment at a time, the quasi-static momentum
 * balance of a compressible (visco-)hypoelastic, perfectly plastic
 * Drucker-Prager medium on a conservative staggered grid, by the accelerated
 * pseudo-transient (PT) iteration (paper: "Summary of the governing
 * equations", "Accelerated pseudo-transient method", "Return mapping
 * algorithm for plasticity", "Convergence study").  Every PT iteration is a
 * stencil sweep on the GPU: pressure and deviatoric stress from the velocity
 * gradients, radial return onto the yield surface sqrt(J2) = A p + B c, and a
 * velocity update from the stress divergence.
 *
 * Conventions shared by every call
 *  - Return value: EP_OK (0) or a negative EP_E* code; no exception crosses
 *    the ABI.  ep_last_error() describes the last failure of a handle.
 *  - Host arrays are FP64, x fastest, at the field's own staggered shape
 *    (ep_field_shape).  The caller owns them; the library copies.
 *  - Device memory: the caller allocates ONE workspace of
 *    ep_workspace_size() bytes (any allocator; 256-byte alignment) and keeps
 *    it alive, unmodified, until ep_destroy.  The library allocates no device
 *    memory of its own.
 *  - Streams: all device work of a handle is queued on the stream given to
 *    ep_init (a hipStream_t passed as void*; NULL = default stream).  Calls
 *    that return host data synchronise that stream.  A handle is not
 *    thread-safe; use one handle per stream.
 *  - Units are those of the caller; the workloads use the paper's
 *    nondimensionalisation (L_x = 1, G_0 = 1, background strain rate a = 1).
 */
#ifndef EP_H
#define EP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EP_ABI_VERSION 3

/* return codes */
#define EP_OK          0
#define EP_EINVAL     -1   /* bad argument or parameter set */
#define EP_ENOMEM     -2   /* workspace too small */
#define EP_EDEVICE    -3   /* a HIP call failed (message in ep_last_error) */
#define EP_ENOTCONV   -4   /* max_iter reached: state rolled back to the increment start */
#define EP_EDIVERGED  -5   /* NaN/Inf or residual > 1e8 * reference: rolled back */

/* precision of the PT iteration fields */
#define EP_FP64        0   /* everything FP64 (the paper's precision) */
#define EP_FP32_FIELDS 1   /* v, p, tau iterate in FP32; accumulated stress,
                              displacement, strain and all norms FP64; the
                              increment finishes in FP64 sweeps when FP32
                              stalls above the tolerance */

/* sweep implementation */
#define EP_SWEEP_AUTO     0
#define EP_SWEEP_FUSED    1   /* one kernel per PT iteration (LDS halo tiles) */
#define EP_SWEEP_UNFUSED  2   /* three kernels per iteration (centres, shear, velocity) */

typedef struct ep_params {
    int    ndim;             /* 2 or 3 */
    int    nx, ny, nz;       /* cells per direction, each >= 3 (nz ignored in 2D) */
    double lx, ly, lz;       /* domain extents; the domain is centred at the origin */
    double bulk;             /* K > 0; +inf: incompressible (pseudo-transient pressure equation
                                A2ssP2, 1/(K dt) = 0): the pressure term of the residual then
                                takes the visco-elastic viscosity in place of K dt, and a
                                physical evaluation keeps the pressure's pseudo-time term */
    double shear;            /* G > 0 (uniform) */
    double visc;             /* mu_s > 0; +INFINITY gives the elasto-plastic limit */
    double phi_deg;          /* friction angle */
    double psi_deg;          /* dilation angle, 0 <= psi <= phi: plastic potential
                                Q = sqrt(J2) - C p with C from psi as A from phi (Plasticity
                                section); psi > 0 adds the plastic volume rate lambda_dot C
                                to the pressure equation (dilatant return) */
    double dt;               /* physical time increment per load step */
    double erate[3];         /* background strain rate (diagonal); pure shear = (1,-1,0) */
    double tol;              /* normalised residual tolerance (> 0) */
    int    max_iter;         /* PT iteration cap per increment (> 0) */
    int    n_check;          /* residual checked every n_check iterations (0: 10 in 3D, 100 in 2D) */
    double re;               /* PT numerical Reynolds number (0: 3 sqrt(10) pi / 2) */
    double r;                /* PT ratio K~/G~ (0: 1/2) */
    double cfl;              /* PT Courant number V~ dtau / h (0: 0.9/sqrt(ndim); must be < 1/sqrt(ndim)) */
    int    precision;        /* EP_FP64 or EP_FP32_FIELDS */
    int    sweep;            /* EP_SWEEP_* */
    double fp32_switch;      /* FP32 mode: leave FP32 when the normalised residual is
                                below this (0: 2 * tol), or within 3x (3D) or 10x (2D) of the FP32
                                rounding floor 8 u32 max|sigma| / h, ... */
    int    fp32_stall;       /* ... or, within 20x of that floor, has not halved for
                                this many checks (or for 4x as many anywhere)
                                (0: 16 max(nx,ny,nz) / n_check; < 0: never) */
    int    freeze_iter;      /* frozen plasticity (accelerated PT section): 0 off; else an
                                increment not converged at the first check at or after this
                                iteration continues with the plastic multiplier Lambda of
                                the next sweep held fixed at every cell (a linear problem) */
    double guess_accept;     /* a supplied starting guess (ep_net_predict) is used when the
                                residual of its physical stresses is below guess_accept times
                                that of the plain guess (0: 1, i.e. only when lower).  The PT
                                iteration removes rough errors of a guess within few sweeps,
                                so a larger value can pay off; an increment that fails from
                                the guess is redone from the plain guess */
    int    objective;        /* 1: objective stress update at the start of every increment
                                (Jaumann rate of stress, equations j1-j14 and the appendix
                                on the objective stress terms): the carried stresses become
                                tau + dt (tau^R - v.grad tau) and p - dt v.grad p with the
                                previous increment's velocities, vorticity
                                w_ij = (dv_i/dx_j - dv_j/dx_i)/2 at the shear points,
                                first-order upwind advection, explicit over dt; 0: off */
    double eta_vp;           /* consistency regularisation of the return (the visco-plastic
                                strain rate of the constitutive section): a yielding point
                                returns to tauII = A p + B c + eta_vp lambda_dot, with
                                lambda_dot = 2 eps_dot_p,II from the consistency condition
                                (0: perfect plasticity, the paper's runs; >= 0, finite) */
    double pt_blend;         /* return mapping of the iteration (return-mapping section,
                                Lambda form): the centre plastic multiplier is the radial
                                return of the physical trial S = tau^/(G dt) + 2 e' (shear
                                parts averaged from the four shear points), blended with
                                weight pt_blend in [0, 1] with the return of the pseudo-time
                                trial.  Both agree at the fixed point, which is therefore the
                                solution of the increment's equations with the pseudo-time
                                terms removed for any weight; the blend only shapes the path */
    double pt_blend_late;    /* the weight from the first check at or after 16 max(nx, ny, nz)
                                iterations of an increment on (the workloads use 0.25, then
                                0.75: the only schedule among those measured under which every
                                test increment converged) */
} ep_params;

typedef struct ep_step_stats {
    int    status;           /* EP_OK, EP_ENOTCONV or EP_EDIVERGED */
    int    iters;            /* PT iterations of the increment (all precisions) */
    int    iters_fp32;       /* of which FP32 sweeps */
    double r_ref;            /* momentum residual of the physical stresses of the plain guess */
    double ref;              /* max(r_ref, 2 G max|erate| dt / L): residual normaliser */
    double resid;            /* final residual (absolute; normalised = resid / ref) */
    double eps_rel;          /* dtau/rho~ * resid / max|v| (relative velocity change per iteration) */
    double sxx_centre;       /* integral of sigma_xx = tau_xx - p over the centre column (plane in 3D) */
    double sxx_left;         /* ... over the first column */
    double sxx_right;        /* ... over the last column */
    long long n_yield;       /* cells on the yield surface in the accepted state */
    double max_violation;    /* max over cells of tauII(stored stresses) - (A p + B c) */
    double seconds;          /* wall time of the call */
    double fp32_exit;        /* normalised residual when FP32 handed over (0 in FP64 mode) */
    int    frozen_at;        /* iteration whose check froze Lambda (0: not frozen) */
    int    guess_used;       /* 1: the increment started from a supplied guess (ep_net_predict);
                                -1: it failed from the guess and was redone from the plain guess
                                (iters counts both attempts) */
    double r_guess;          /* momentum residual of the physical stresses of that guess (0: none) */
    double cert;             /* certificate of the accepted state: the FP64 momentum residual of
                                the physical stresses of its velocities (pseudo-time terms
                                removed), <= tol * ref; those stresses are the accepted ones */
} ep_step_stats;

typedef struct ep_residual_info {
    double resid;            /* combined residual of one PT evaluation of the current state */
    double momentum;         /* L-inf momentum residual of one PT update of the current state
                                (the absolute error of the convergence section) */
    double physical;         /* momentum residual of the physical stresses of the current v
                                (the certificate of ep_step_stats) */
    double vmax;             /* max |v| after that update */
    double continuity;       /* L-inf of (p - p^)/(K dt) + div v of the current state (the
                                pressure equation without its pseudo-time term; max|div v| for
                                K = +inf) */
    double eps_rel;          /* relative error of the convergence section: max|v^{k+1} - v^k| /
                                max|v^{k+1}| of that PT update */
} ep_residual_info;

/* field ids for ep_fields / ep_field_shape */
enum {
    EP_F_VX = 0, EP_F_VY, EP_F_VZ,
    EP_F_P, EP_F_TXX, EP_F_TYY, EP_F_TZZ, EP_F_TXY, EP_F_TXZ, EP_F_TYZ,
    EP_F_P_OLD, EP_F_TXX_OLD, EP_F_TYY_OLD, EP_F_TZZ_OLD, EP_F_TXY_OLD, EP_F_TXZ_OLD, EP_F_TYZ_OLD,
    EP_F_UX, EP_F_UY, EP_F_UZ,
    EP_F_EXX, EP_F_EYY, EP_F_EZZ, EP_F_EXY, EP_F_EXZ, EP_F_EYZ,
    EP_F_EPS_P, EP_F_COHESION, EP_F_LAMBDA_DOT, EP_F_TAU_II, EP_F_YIELD,
    EP_F_LAMBDA_FROZEN,      /* 2D: centre Lambda held fixed by the last frozen increment */
    EP_F_COUNT
};
#define EP_GET 0
#define EP_SET 1

typedef struct ep_handle ep_handle;

/* Library version (EP_ABI_VERSION of the build). */
int ep_abi_version(void);

/* Bytes of device workspace needed for *p.  Pure function; EP_EINVAL for an
 * invalid parameter set. */
int ep_workspace_size(const ep_params* p, size_t* bytes);

/* Create a solver in a caller-owned workspace.
 *  cohesion: n_cells FP64 values (x fastest) or NULL for 0; copied.
 *  shear: n_cells FP64 shear moduli (x fastest), each in (0, p->shear], or NULL
 *    for the uniform p->shear; copied; the same as ep_set_shear_modulus right
 *    after creation (the heterogeneous setups of the initial-conditions
 *    section).
 *  d_workspace/ws_bytes: device memory from the caller, >= ep_workspace_size.
 *  stream: hipStream_t (as void*) used for all work of the handle.
 * Initial state (model configuration section): p = tau = 0 and velocities
 * equal to the background pure-shear field v = erate * x (domain centred).
 * Errors: EP_EINVAL (psi outside [0, phi], cfl >= 1/sqrt(ndim), a size < 3, K, G, dt,
 * tol or visc not > 0, NULL out, a shear modulus out of range), EP_ENOMEM (workspace too
 * small), EP_EDEVICE. */
int ep_init(const ep_params* p, const double* cohesion, const double* shear, void* d_workspace, size_t ws_bytes,
            void* stream, ep_handle** out);

/* Solve one load increment: save the increment's starting stresses (p^,
 * tau^); evaluate the physical stresses of the previous velocities (the plain
 * guess) -- their momentum residual is R_ref and they are the pseudo-time
 * starting point of p and tau (accepted at once when R_ref already meets the
 * tolerance); iterate PT sweeps until the residual (momentum L-inf combined
 * with the pressure and deviator pseudo-rates, see the paper's convergence
 * section) is at most tol * ref and, at that check, the FP64 momentum
 * residual of the physical stresses of the current velocities is too (the
 * certificate; those stresses become the accepted state); then add v dt to
 * the displacement and the strain-rate increments to the accumulated
 * strains.  On EP_ENOTCONV / EP_EDIVERGED the state is rolled back to the
 * increment start and st is still filled.  st may be NULL. */
int ep_load_step(ep_handle* h, ep_step_stats* st);

/* Starting guess of the next ep_load_step: face velocities (host FP64 arrays
 * at the shapes of EP_F_VX, EP_F_VY, EP_F_VZ; vz NULL in 2D), copied.  The
 * increment starts from them when the residual of their physical stresses is
 * below guess_accept times that of the plain guess (the previous
 * velocities), else from the plain guess; wall normal velocities are reset
 * to their prescribed values either way; the stopping rule is unchanged
 * (its normaliser is that of the plain guess).  Used once.  EP_EINVAL on a
 * NULL array. */
int ep_set_guess(ep_handle* h, const double* vx, const double* vy, const double* vz);

#define EP_GUESS_VELOCITY 0   /* the arrays are the guessed face velocities */
#define EP_GUESS_CHANGE   1   /* the arrays are velocity changes, added to the current
                                 velocities (those of the last accepted increment) */
#define EP_GUESS_ZERO     2   /* zero velocities inside the domain; no arrays */
#define EP_GUESS_F64      0
#define EP_GUESS_F32      1

/* Starting guess of the next ep_load_step from device memory (e.g. a
 * predictor's output tensor), with the same acceptance rule as ep_set_guess
 * (paper, accelerated pseudo-transient method: the iteration starts from the
 * previous increment's velocities; a better starting point shortens it).
 *  kind: EP_GUESS_VELOCITY, EP_GUESS_CHANGE or EP_GUESS_ZERO (above).
 *  dtype: EP_GUESS_F64 (double) or EP_GUESS_F32 (float) elements.
 *  vx, vy, vz: device pointers to compact arrays at the shapes of EP_F_VX,
 *    EP_F_VY, EP_F_VZ (x fastest; vz NULL in 2D; all NULL for EP_GUESS_ZERO),
 *    on the handle's device; the caller keeps ownership.
 * The arrays are read by a kernel enqueued on the handle's stream by this
 * call, so they must stay valid and unchanged until that stream has passed
 * it (for instance until the next ep_load_step returns).  Wall normal
 * velocities are reset to their prescribed values whatever the arrays hold.
 * Used once.  EP_EINVAL for a bad kind or dtype, a NULL array where one is
 * needed, or a pointer that HIP does not report as device memory;
 * EP_EDEVICE for a launch failure. */
int ep_set_guess_device(ep_handle* h, int kind, int dtype, const void* vx, const void* vy, const void* vz);

/* Residual history of the last ep_load_step: for each check, the normalised
 * residual (resid / ref) and the precision of the sweeps that produced it
 * (EP_FP64 or EP_FP32_FIELDS).  Copies at most cap entries; returns the
 * number of checks recorded (may exceed cap), or EP_EINVAL. */
int ep_step_history(const ep_handle* h, double* resid, int* precision, int cap);

/* Run n PT sweeps on the current state without the increment prologue or
 * epilogue (the previous-increment stresses are whatever ep_fields set or
 * the last increment left).  *resid (may be NULL) gets the combined residual
 * of the last sweep.  For single-sweep parity checks. */
int ep_sweep(ep_handle* h, int n, double* resid);

/* FP64 norms of the current state (no state change).  Synchronous. */
int ep_residual(ep_handle* h, ep_residual_info* r);

/* Allocation-free variant of ep_residual, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same norms as ep_residual, computed by the same
 * kernels; the reduction counters, the two sweep-argument tables and (2D
 * models) the tile list are staged in a static device array of the library
 * (64 KiB per GPU, held until the process ends) instead of the handle's
 * workspace.  Calls no hipMalloc, hipFree or allocating routine; like
 * ep_residual it writes the handle's second iteration buffer (the state is
 * unchanged).  EP_EINVAL (message in ep_last_error) for a 2D model whose tile
 * list exceeds the array (more than 8,000 tiles of 64 x 16 cells).  The
 * array is shared by every call on the same GPU: calls that overlap on one
 * GPU (other streams or threads) race and must be serialised by the caller.
 * Synchronous. */
int ep_residual_noalloc(ep_handle* h, ep_residual_info* r);

/* Objective stress update of the current state with its current velocities,
 * in place (paper: Jaumann rate of stress, equations j1-j14, and the
 * appendix on the objective stress terms; the discretisation of the
 * `objective` parameter): tau <- tau + dt (tau^R - v.grad tau),
 * p <- p - dt v.grad p.  ep_load_step applies the same update first when
 * the handle's `objective` parameter is set; here it runs whatever that
 * parameter.  The increment-start fields (EP_F_*_OLD) then hold the updated
 * stresses, as after an increment prologue.  Asynchronous on the handle's
 * stream. */
int ep_objective_update(ep_handle* h);

/* Background strain rate (the pure-shear loading of the walls) of the next
 * increments, e.g. a loading schedule of velocity increments (the viscous-
 * limit runs of the paper's incompressible limits section raise the
 * prescribed velocity from increment to increment).  Walls take the new rate
 * at the next ep_load_step; the stopping rule's floor 2 G max|erate| dt / L
 * follows it.  Single models only (EP_EINVAL for a batch model, a NULL or a
 * non-finite rate). */
int ep_set_strain_rate(ep_handle* h, const double erate[3]);

/* Shear modulus per cell (the heterogeneous setups of the section on initial
 * conditions and heterogeneities, e.g. a Gaussian G rising from the centre
 * towards the walls).  shear: host array of one value per cell (nx*ny, or
 * nx*ny*nz in 3D), x fastest, each in (0, ep_params.shear]; copied, the
 * caller keeps ownership.  A cell's physical compliance 1/(G dt) replaces the
 * uniform one in its stress update; a vertex (2D) or edge (3D) takes the mean
 * compliance of its four cells; the pseudo-time steps and the residual scales
 * stay those of ep_params.shear (which therefore bounds every G).  The fused
 * 3D sweep reads the compliance of every cell once per sweep (one more field
 * access per cell).  Applies from the next sweep on; may be called again.
 * EP_EINVAL for a batch model, a NULL array or a value out of range (nothing
 * is changed then). */
int ep_set_shear_modulus(ep_handle* h, const double* shear);

/* Copy one field between the device state and a host FP64 array of exactly
 * ep_field_shape() elements.  dir = EP_GET or EP_SET.  EP_SET of TZZ(_OLD) is
 * rejected in 3D (the deviator is stored trace-free: tzz = -(txx + tyy));
 * accumulators, cohesion and the old stresses may be set (checkpoint
 * restore).  LAMBDA_DOT, TAU_II and YIELD describe the last accepted
 * increment and are read-only, as is LAMBDA_FROZEN (meaningful after an
 * increment whose stats report frozen_at > 0).  EP_EINVAL on a bad id or count. */
int ep_fields(ep_handle* h, int field, int dir, double* host, size_t count);

/* Shape (x, y, z extents; z = 1 in 2D) of a field; 0 extents if the field
 * does not exist for this ndim.  Returns the element count or EP_EINVAL. */
long ep_field_shape(const ep_handle* h, int field, int shape[3]);

/* Release the handle (not the workspace). */
void ep_destroy(ep_handle* h);

/* Last error message of a handle (static string for a NULL handle). */
const char* ep_last_error(const ep_handle* h);

/* Timing of the PT sweeps (the dominant kernels).  When enabled, every batch
 * of back-to-back sweeps between two residual checks is bracketed by HIP
 * events on the handle's stream; ep_sweep_timing returns, for the given
 * precision (EP_FP64 / EP_FP32_FIELDS), the accumulated event time divided
 * by the number of sweeps since timing was (re-)enabled, i.e. the average
 * duration of one PT iteration (all of its kernels).  Enabling resets. */
int ep_enable_timing(ep_handle* h, int on);
int ep_sweep_timing(const ep_handle* h, int precision, double* avg_ms, long* sweeps);

/* ---- batches of 2D models ----------------------------------------------------
 * A parameter sweep: n independent 2D models (each its own ep_params: size,
 * material, cohesion field, tolerance) solved one load increment at a time
 * together.  The PT sweeps of all models run as persistent launches that
 * walk one tile list per precision and tile shape, n_check sweeps per
 * replay of a captured HIP graph; after every replay each model is checked
 * with the single-model convergence rule (ep_load_step) and retired from
 * the lists when it has converged or failed, or moved to FP64 sweeps at its
 * FP32 hand-over.  Per model, the iterates, iteration counts and statistics
 * are those of ep_load_step on that model alone.
 * Requirements: every model 2D, all with the same precision and the same
 * (resolved) n_check, which must be even; at most 32767 tiles per direction.
 * Memory: one caller-owned workspace of ep_batch_workspace_size() bytes
 * (256-byte aligned), as for ep_init.  Stream: as for ep_init; graph
 * replays are launched on it (a private stream is used only to record the
 * graph). */
typedef struct ep_batch ep_batch;

/* Bytes of device workspace for n models with parameters p[0..n-1]. */
int ep_batch_workspace_size(int n, const ep_params* p, size_t* bytes);

/* Create a batch.  cohesion: NULL or n pointers, each NULL or n_cells FP64
 * values of model i (copied).  Initial state of every model as in ep_init.
 * Errors: EP_EINVAL (a model's parameters invalid, not 2D, mixed precision or
 * n_check, odd n_check), EP_ENOMEM, EP_EDEVICE. */
int ep_batch_init(int n, const ep_params* p, const double* const* cohesion, void* d_workspace, size_t ws_bytes,
                  void* stream, ep_batch** out);

/* Autotuner: picks the tile shape of each model size (models with equal
 * nx, ny share one) by timing `reps` batched sweeps of all models per
 * candidate, coordinate descent over the size classes; FP32-field batches
 * get a second shape per size for their FP64 finishing sweeps, tuned the
 * same way.  The timed sweeps leave the state unchanged.  Optional; the
 * default shape is 64 x 8. */
int ep_batch_tune(ep_batch* b, int reps);

/* Tile shape used for model i. */
int ep_batch_tile_shape(const ep_batch* b, int i, int* tx, int* ty);

/* One load increment of every model; st: n entries (required), filled as by
 * ep_load_step.  Returns EP_OK when all models converged, else the status
 * of the first model that did not (that model's state rolled back, the
 * others advanced). */
int ep_batch_load_step(ep_batch* b, ep_step_stats* st);

/* The handle of model i, for ep_fields, ep_field_shape, ep_residual,
 * ep_step_history and ep_sweep (owned by the batch: ep_destroy ignores it). */
ep_handle* ep_batch_model(ep_batch* b, int i);

/* Timing of the graph replays: when enabled, each replay is bracketed by
 * HIP events; ep_batch_timing returns the accumulated milliseconds, the
 * cell-sweeps done in FP32 and in FP64 (sum over models of cells x sweeps)
 * and the number of replays since timing was (re-)enabled. */
int ep_batch_enable_timing(ep_batch* b, int on);
int ep_batch_timing(const ep_batch* b, double* ms, double* cell_sweeps32, double* cell_sweeps64, long* replays);

void ep_batch_destroy(ep_batch* b);
const char* ep_batch_last_error(const ep_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* EP_H */
