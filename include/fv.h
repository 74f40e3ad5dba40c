/*
 * fv.h -- C ABI of the MI355X finite-volume library (libfv.so).
 *
 * The library advances cell-average conserved states of the 2D shallow-water
 * equations (state h, hu, hv; thesis eq 2.3) or of the 2D Euler equations
 * (state rho, rho u, rho v, E; eq 2.4 and section 4.2) on a uniform
 * structured grid by explicit finite-volume steps (section 2.3):
 *   - MINMOD slope-limited face states (eq 2.18) or first-order states;
 *   - a numerical flux per face in the face-normal frame (eq 2.24):
 *     HLLE (eq 2.16, default), Rusanov (eq 2.12) or Roe (eq 2.14);
 *   - the conservative update summed over the cell faces (eq 2.9, eq 2.23),
 *     with the bed-slope source of eq 2.3 through a hydrostatic
 *     reconstruction when a bed is given;
 *   - Heun (eq 2.19, default), the three-stage scheme of eq 2.20, or one
 *     forward-Euler stage;
 *   - Delta t from the CFL condition (eq 2.10), reduced over the grid on the
 *     device every step:  dt = cfl / max_i((|u_i|+c_i)/dx + (|v_i|+c_i)/dy).
 *
 * Conventions for every entry point:
 *   - Every call returns fv_status: FV_OK (0) or a negative error code.
 *     fv_last_error() returns a thread-local message describing the last
 *     failing call.  No C++ exception crosses this interface.
 *   - Device pointers are HIP device allocations owned by the caller; the
 *     library never frees them and they must outlive the handle that uses
 *     them.  The library owns only the opaque handles.
 *   - States are structure-of-arrays: var-major, then y (row), then x
 *     (fastest): element (v, j, i) sits at index (v*ny + j)*nx + i, with
 *     element type float (FV_F32) or double (FV_F64).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on that stream; the library
 *     synchronises it only in the calls documented as sync points.
 *   - One handle is used by one host thread at a time; distinct handles are
 *     independent.
 */
#ifndef FV_H
#define FV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FV_OK = 0,
    FV_E_INVALID = -1,      /* bad argument or configuration */
    FV_E_NOMEM = -2,        /* workspace too small */
    FV_E_HIP = -3,          /* a HIP runtime call failed */
    FV_E_INADMISSIBLE = -4, /* a cell reached h <= 0 (rho <= 0, p <= 0) or a non-finite value */
    FV_E_UNSUPPORTED = -5   /* valid but not implemented combination */
} fv_status;

enum { FV_SWE = 0, FV_EULER = 1 };
enum { FV_F32 = 0, FV_F64 = 1 };
enum { FV_BC_PERIODIC = 0, FV_BC_WALL = 1 };
enum { FV_FLUX_HLLE = 0, FV_FLUX_RUSANOV = 1, FV_FLUX_ROE = 2 };
enum { FV_RECON_MINMOD = 0, FV_RECON_FIRST = 1 };

/* Solver configuration (plain data, copied at fv_init). */
typedef struct {
    uint32_t struct_size; /* must be sizeof(fv_config) */
    int32_t eqn;          /* FV_SWE | FV_EULER */
    int32_t prec;         /* FV_F32 | FV_F64: element type of state and bed */
    int32_t nx, ny;       /* cells per axis, each >= 4 */
    int32_t bc_x, bc_y;   /* FV_BC_PERIODIC | FV_BC_WALL (mirror ghosts, normal momentum negated) */
    int32_t flux;         /* FV_FLUX_* */
    int32_t recon;        /* FV_RECON_MINMOD | FV_RECON_FIRST */
    int32_t rk_stages;    /* 1 forward Euler, 2 Heun, 3 three-stage SSP */
    int32_t learned;      /* 1: the workspace also holds the buffers of fv_learned_step */
    double lx, ly;        /* domain [0,lx] x [0,ly], > 0 */
    double cfl;           /* Courant number in (0, 1] */
    double dt_fixed;      /* > 0: fixed Delta t, the CFL reduction is skipped */
    double g;             /* gravity (SWE), > 0 */
    double gamma;         /* ratio of specific heats (Euler), > 1 */
    double h_ref;         /* SWE: reference depth h0 of the pressure term, carried as
                             g (h^2 - h0^2)/2 (a constant shift of every face flux that
                             cancels in each cell's divergence and keeps float rounding
                             proportional to |h^2 - h0^2|); 0 = mean depth of the initial state */
} fv_config;

typedef struct fv_solver fv_solver;

/* Number of variables of the configuration (3 for SWE, 4 for Euler). */
int fv_nvar(const fv_config *cfg);

/* Bytes of device workspace fv_init needs for this configuration (stage
 * buffers, reduction slots, counters); 0 if cfg is invalid.  Used by the
 * caller for memory admission. */
size_t fv_workspace_bytes(const fv_config *cfg);

/* Create a solver over caller-owned device memory.
 *   q         device state, nvar*ny*nx elements, updated in place by the steps;
 *   bathy     device bed b(x,y), ny*nx elements, or NULL for a flat bottom
 *             (SWE only; FV_E_INVALID for Euler);
 *   workspace device memory of at least fv_workspace_bytes(cfg) bytes,
 *             256-byte aligned, private to this solver;
 *   stream    hipStream_t as void*.
 * Validates the configuration (FV_E_INVALID), checks that the initial state
 * is admissible (FV_E_INADMISSIBLE; this check synchronises the stream),
 * resets time and step count to 0 and computes the first CFL rate. */
fv_status fv_init(const fv_config *cfg, void *q, const void *bathy, void *workspace,
                  size_t workspace_bytes, void *stream, fv_solver **out);

/* Enqueue one full time step (all stages) on the solver's stream. */
fv_status fv_step(fv_solver *s);

/* Enqueue nsteps >= 0 full steps; no host synchronisation between steps. */
fv_status fv_run(fv_solver *s, int64_t nsteps);

/* Sync point.  Simulated time and number of completed steps.  Returns
 * FV_E_INADMISSIBLE if a step produced an inadmissible cell: the state is
 * then the one that step produced and later steps were skipped; *step
 * reports the steps completed including the failing one. */
fv_status fv_time(fv_solver *s, double *t, int64_t *step);

/* Sync point.  Conserved totals sum_i q_v dx dy for each of the nvar
 * variables, then the energy sum (g h^2/2 + h|u|^2/2) dx dy (SWE, eq 5.1) or
 * the kinetic energy sum rho|u|^2/2 dx dy (Euler); out holds nvar+1 doubles
 * (host memory), accumulated in double precision in a fixed order. */
fv_status fv_totals(fv_solver *s, double *out);

/* Copy the current state to dst (nvar*ny*nx elements of the solver's
 * precision; host memory if dst_is_host, else device).  Sync point. */
fv_status fv_get_state(fv_solver *s, void *dst, int dst_is_host);

/* Replace the current state (same layout) and recompute the CFL rate;
 * time and step count are kept.  Clears a previous inadmissible flag.
 * Sync point (admissibility of the new state is checked). */
fv_status fv_set_state(fv_solver *s, const void *src, int src_is_host);

/* Reference depth h0 the solver uses (see fv_config.h_ref); a checkpoint
 * that is resumed in a new handle passes it back as h_ref. */
double fv_reference_depth(const fv_solver *s);

/* Device pointer of the current state (the q passed to fv_init). */
void *fv_state_ptr(fv_solver *s);

/* Change the stream later work is enqueued on. */
fv_status fv_set_stream(fv_solver *s, void *stream);

/* Sync point.  Face fluxes of the current state for inspection:
 * fx: nvar x ny x (nx+1) values at faces i-1/2 (i = 0..nx), fy: nvar x (ny+1)
 * x nx at faces j-1/2, as seen by the cell on the right/top, solver
 * precision, device memory.  Flat-bottom configurations only. */
fv_status fv_face_fluxes(fv_solver *s, void *fx, void *fy);

/* Release the handle (not the caller's buffers).  Waits for queued work. */
void fv_destroy(fv_solver *s);

/* ------------------------------------------------------------------------
 * Allocation-free stepping, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  fv_run_noalloc does what fv_init + fv_run + fv_time do, with the
 * same kernels and bit-identical results, but takes its workspace (control
 * block, CFL rate slots, stage buffers, descriptor) from a device array the
 * library holds: FV_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library
 * is loaded and kept until the process ends.  It calls no allocating routine,
 * no memset and no host synchronisation: everything is enqueued on `stream`.
 *
 *   cfg      as for fv_init, with learned = 0; for SWE, h_ref > 0 is required
 *            (the mean-depth default would need a reduction and a host read);
 *   q        device state, updated in place by nsteps full steps;
 *   bathy    device bed or NULL (SWE only);
 *   nsteps   >= 0;
 *   stream   hipStream_t as void*;
 *   info_dev NULL, or a device fv_run_info that receives the simulated time,
 *            the completed steps and the inadmissible flag when the steps end.
 * Errors: FV_E_INVALID (bad configuration or arguments), FV_E_UNSUPPORTED
 * (learned = 0 required), FV_E_NOMEM (the configuration needs more than
 * FV_NOALLOC_SCRATCH_BYTES: see fv_noalloc_bytes), FV_E_HIP.  An initial
 * state that is not admissible is reported through info_dev->inadmissible
 * (the state is then left unchanged), not by the return code.
 * Every call on one GPU uses the same array and leaves its contents behind;
 * each call resets what must start at zero.  Calls that overlap on one GPU
 * (concurrent host threads, or streams that run at the same time) race on
 * the array and must not be issued. */
#define FV_NOALLOC_SCRATCH_BYTES (64u << 20)

typedef struct {
    double t;             /* simulated time */
    int64_t steps;        /* completed steps */
    int32_t inadmissible; /* 1: a cell became inadmissible (h <= 0, rho <= 0, p <= 0 or non-finite) */
    int32_t reserved;
} fv_run_info;

/* Scratch bytes fv_run_noalloc needs for cfg (fv_workspace_bytes of the
 * classic scheme); 0 if cfg is invalid. */
size_t fv_noalloc_bytes(const fv_config *cfg);

fv_status fv_run_noalloc(const fv_config *cfg, void *q, const void *bathy, int64_t nsteps, void *stream,
                         fv_run_info *info_dev);

/* ------------------------------------------------------------------------
 * Learned stencil coefficients (thesis section 2.5.3, fourth approach:
 * a CNN outputs constrained reconstruction coefficients per conserved
 * variable; eq 2.26-2.27 for the pseudo-linear stencil).
 *
 * Network: five 3x3 convolutions 3 -> 32 -> 32 -> 32 -> 32 -> 72, ReLU
 * between layers, periodic padding, input (h, hu, hv) normalised per channel
 * as (q - mean) * inv_std.  BF16 weights and activations, FP32 accumulation
 * on MFMA; the 72 outputs of a cell are raw coefficients z for its +x and +y
 * faces, channel ((axis*2 + side)*3 + var)*6 + k, side 0 = left state, 1 =
 * right state, k over the six cells i-2..i+3 around the face.  They are
 * mapped onto the constraint set alpha = alpha_base + P z, where P projects
 * onto the null space of the moment conditions (the face value is exact for
 * cell averages of polynomials of degree <= order) and alpha_base are
 * Fromm's stencils; the face state is sum_k alpha_k q(i-2+k).  A face side
 * whose learned depth is <= 0 uses the plain MINMOD state; a step that leaves
 * a cell with h <= 0 is redone with the plain scheme.
 *
 * Master parameters: FP32 device vector of fv_model_param_count() floats,
 * layer by layer W_l[co][ci][ky][kx] followed by b_l[co].
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t struct_size; /* sizeof(fv_model_desc) */
    int32_t hidden;       /* hidden channels: 32 */
    int32_t order;        /* constraint order 0 or 1 (1: exact for linear data) */
    int32_t reserved0;    /* must be 0 */
    float mean[3];        /* input normalisation */
    float inv_std[3];
} fv_model_desc;

typedef struct fv_model fv_model;

typedef struct {
    int64_t fallback_faces; /* face sides that used the MINMOD state, cumulative */
    int64_t redone_steps;   /* steps redone with the plain scheme, cumulative */
} fv_learned_stats;

/* Number of FP32 master parameters (49448). */
size_t fv_model_param_count(void);

/* Device bytes a model needs for its packed BF16 weights. */
size_t fv_model_workspace_bytes(const fv_model_desc *desc);

/* Create a model over caller-owned device memory: params (FP32 master
 * vector, read now and by fv_model_update) and workspace (packed weights,
 * 256-byte aligned).  Packing is enqueued on stream. */
fv_status fv_model_create(const fv_model_desc *desc, const float *params, void *workspace, size_t workspace_bytes,
                          void *stream, fv_model **out);

/* Re-pack the weights after the master parameters changed (async). */
fv_status fv_model_update(fv_model *m);

void fv_model_destroy(fv_model *m);

/* Scratch bytes fv_model_forward needs for B solves of ny x nx cells. */
size_t fv_model_forward_scratch_bytes(int B, int nx, int ny);

/* Batched network inference on the model's stream (async):
 *   q       device [B][3][ny][nx] FP32 states (periodic, nx % 16 == 0,
 *           nx*ny % 64 == 0);
 *   z       device [B][ny][nx][72] FP32 raw coefficients (output);
 *   scratch device, >= fv_model_forward_scratch_bytes(B, nx, ny), 256-byte
 *           aligned (BF16 activations). */
fv_status fv_model_forward(const fv_model *m, const float *q, int B, int nx, int ny, float *z, void *scratch,
                           size_t scratch_bytes);

/* The same network pass in one launch, without scratch: each workgroup runs
 * all five layers on an 8x8 tile of pixels, recomputing the halo the 3x3
 * stack needs (thesis section 2.5.3, fourth approach: the network of
 * fv_model_forward).  For small grids, where a launch per layer would
 * dominate.  z is bit-identical to fv_model_forward's.
 *   q  device [B][3][ny][nx] FP32 (periodic, nx % 8 == 0, ny % 8 == 0);
 *   z  device [B][ny][nx][72] FP32 (output).
 * Enqueued on the model's stream; FV_E_UNSUPPORTED for other grid sizes. */
fv_status fv_model_forward_tiled(const fv_model *m, const float *q, int B, int nx, int ny, float *z);

/* Enqueue nsteps learned Heun steps at the fixed step cfg.dt_fixed.
 * Requires a shallow-water FP32 solver with periodic boundaries, no bed,
 * rk_stages = 2, dt_fixed > 0, learned = 1, nx % 16 == 0 and
 * nx*ny % 64 == 0 (FV_E_UNSUPPORTED otherwise).  When stats is not NULL the
 * call synchronises and fills the cumulative counters.  Inadmissible results
 * of the plain redo are reported by fv_time as FV_E_INADMISSIBLE.  The
 * steps' admissibility flags alternate between two slots, so a call
 * captured in a graph for replay should enqueue an even number of steps (a
 * replay starts on the slot its capture started on). */
fv_status fv_learned_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats);

/* Enqueue nsteps Heun steps of the direct face-state scheme (thesis section
 * 5.3, planar shallow water): the network maps the cell averages to the
 * states at the four faces of every cell, and each face's flux (HLLE or
 * Rusanov) is taken between the states its two cells give it, so the scheme
 * is conservative.  The model's output channels 3f + v (f = 0 left, 1 right,
 * 2 bottom, 3 top; v = h, hu, hv) are corrections to the cell average in the
 * input's normalised units, Q^f_v = q_v + z_{3f+v} / inv_std_v (a zero head
 * is the first-order scheme); channels 12..71 are not used.  A face side
 * whose depth is not positive takes its MINMOD state (counted as a fallback
 * face); a step with a non-positive depth after either stage is redone with
 * the plain scheme (counted).  Same solver requirements, statistics and
 * error reporting as fv_learned_step, whose counters it shares. */
fv_status fv_direct_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats);

/* Enqueue nsteps learned Heun steps (the coefficient network of
 * fv_learned_step) with the flux-limiter blend of thesis section 2.5.3
 * (second approach): the flux of face i+1/2 is
 *   F = F_low - phi(r_i) (F_low - F_high),
 * F_high the learned face states' flux (MINMOD fallback as fv_learned_step),
 * F_low the flux of the two cell averages, phi the MINMOD flux limiter
 * max(0, min(1, r)) of r_i = (q_i - q_{i-1}) / (q_{i+1} - q_i) per conserved
 * variable at the face's low-index cell i (phi = 0 where q_{i+1} = q_i).
 * Same solver requirements, statistics and error reporting as
 * fv_learned_step, whose counters it shares. */
fv_status fv_blend_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats);

/* ------------------------------------------------------------------------
 * Learned stencil coefficients for the Euler equations.  Thesis section 6.2
 * names a data-driven Euler discretisation with positive density and energy
 * as future work; this is the construction of section 2.5.3 (fourth
 * approach) on the system of section 4.2, q = (rho, rho u, rho v, E),
 * p = (gamma - 1)(E - |m|^2 / 2 rho):
 *   - network 4 -> 32 -> 32 -> 32 -> 32 -> 96 (3x3 convolutions, periodic
 *     padding, ReLU; BF16 weights and activations on MFMA, FP32
 *     accumulation); per cell and axis the left and right state
 *     coefficients of the cell's high face for the four variables, raw
 *     channel ((axis*2 + side)*4 + var)*6 + k; alpha = Fromm base + P z per
 *     group of six (exact for linear data at order 1);
 *   - positivity: a learned face state with rho <= 0, p <= 0 or a non-finite
 *     value takes its MINMOD state (the cell average where MINMOD itself is
 *     inadmissible), counted per face side; a stage that leaves a cell with
 *     rho <= 0 or p <= 0 makes that solve redo its step with the plain
 *     MINMOD scheme;
 *   - HLLE or Rusanov in the face's normal frame, Heun at a fixed step,
 *     periodic domain; B solves of one size per object.
 * Master parameters (FP32, caller-owned, fv_euler_net_param_count() floats):
 * W_l[co][ci][ky][kx] then b_l, layer by layer.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t struct_size;     /* sizeof(fv_euler_learned_config) */
    int32_t B;                /* solves */
    int32_t nx, ny;           /* periodic grid, nx % 16 == 0, ny >= 4 */
    int32_t flux;             /* FV_FLUX_HLLE | FV_FLUX_RUSANOV */
    int32_t order;            /* constraint order 0 or 1 */
    double lx, ly;            /* domain side lengths */
    double gamma;             /* ratio of specific heats, > 1 */
    double dt;                /* the fixed step, > 0 */
    float mean[4], inv_std[4]; /* input normalisation per variable */
} fv_euler_learned_config;

typedef struct fv_euler_learned fv_euler_learned;

/* Number of FP32 master parameters (56672). */
size_t fv_euler_net_param_count(void);

/* Device bytes of the workspace: packed weights, two BF16 activation
 * buffers, the raw coefficients, two stage buffers, per-solve flags and
 * counters. */
size_t fv_euler_learned_workspace_bytes(const fv_euler_learned_config *cfg);

/* Create over caller-owned device memory: params (read now and by
 * fv_euler_learned_update) and workspace (256-byte aligned, >=
 * fv_euler_learned_workspace_bytes); work is enqueued on stream.  Packs
 * the weights and clears the counters (async).  FV_E_INVALID for a bad
 * configuration, FV_E_NOMEM for a small workspace. */
fv_status fv_euler_learned_create(const fv_euler_learned_config *cfg, const float *params, void *workspace,
                                  size_t workspace_bytes, void *stream, fv_euler_learned **out);

/* Re-pack the weights after the master parameters changed (async). */
fv_status fv_euler_learned_update(fv_euler_learned *e);

/* Raw coefficients z (device [B][ny][nx][96] FP32, written) of the states
 * q (device [B][4][ny][nx] FP32), layer by layer through the workspace's
 * activation buffers (async). */
fv_status fv_euler_learned_forward(fv_euler_learned *e, const float *q, float *z);

/* The same network pass in one launch: each workgroup runs all five layers
 * on 8 x 8 tiles in LDS (recomputing the halo the 3x3 stack needs); z is
 * bit-identical to fv_euler_learned_forward's.  Needs nx % 8 == 0 and
 * ny % 8 == 0 (FV_E_UNSUPPORTED otherwise).  fv_euler_learned_step uses it
 * on such grids. */
fv_status fv_euler_learned_forward_tiled(fv_euler_learned *e, const float *q, float *z);

/* nsteps learned Heun steps of the B solves in q (device [B][4][ny][nx]
 * FP32, updated in place) (async).  A solve whose plain redo is still
 * inadmissible is frozen at that state and reported by
 * fv_euler_learned_stats. */
fv_status fv_euler_learned_step(fv_euler_learned *e, float *q, int64_t nsteps);

/* Synchronise the stream and copy the per-solve counters since creation
 * (host arrays of B entries, each nullable): face sides that fell back,
 * steps redone with the plain scheme, frozen flags.  FV_E_INADMISSIBLE if
 * any solve is frozen. */
fv_status fv_euler_learned_stats(fv_euler_learned *e, int64_t *fallback_faces, int64_t *redone_steps,
                                 int32_t *frozen);

void fv_euler_learned_destroy(fv_euler_learned *e);

/* Training of the Euler network with the unrolled loss of eq 2.28 (the
 * planar trainer's construction): T learned Heun steps at a fixed step from
 * the initial states, kept with their activations and coefficients; loss =
 * sum over t of the MSE against targets, variable v divided by scale[v];
 * the reverse pass runs the Heun adjoint, the finite-volume adjoint (Euler
 * flux Jacobians of the branch taken by forward-mode duals, MINMOD
 * derivative on fallback sides, plain adjoint for redone steps) and the
 * network's BF16 MFMA backward.  Gradient reductions in a fixed order. */
typedef struct {
    uint32_t struct_size;  /* sizeof(fv_euler_train_config) */
    int32_t B;             /* windows per batch */
    int32_t nx, ny;        /* periodic grid, nx % 16 == 0, ny >= 4 */
    int32_t T;             /* largest number of unrolled steps */
    int32_t flux;          /* FV_FLUX_HLLE | FV_FLUX_RUSANOV */
    double lx, ly, gamma, dt;
    float scale[4];        /* loss scale of rho, rho u, rho v, E */
    float lr, beta1, beta2, eps; /* Adam */
} fv_euler_train_config;

typedef struct fv_euler_trainer fv_euler_trainer;

size_t fv_euler_train_workspace_bytes(const fv_euler_train_config *cfg);

/* net: its master parameters are trained in place (Adam re-packs its
 * weights) and its stream is used; grads, adam_m, adam_v: device FP32
 * vectors of fv_euler_net_param_count() entries (caller-owned, Adam moments
 * zeroed by the caller); workspace 256-byte aligned. */
fv_status fv_euler_train_create(const fv_euler_train_config *cfg, fv_euler_learned *net, float *grads,
                                float *adam_m, float *adam_v, void *workspace, size_t workspace_bytes,
                                fv_euler_trainer **out);

/* Loss and gradients (grads overwritten) of one batch: q0 device
 * [B][4][ny][nx], targets device [T][B][4][ny][nx], 1 <= T <= cfg T.
 * Synchronises; loss and, when not NULL, the summed counters of the
 * forward rollout are returned. */
fv_status fv_euler_train_step(fv_euler_trainer *tr, const float *q0, const float *targets, int T, double *loss,
                              fv_learned_stats *stats);

/* d loss / d q0 of the last step (device [B][4][ny][nx]); synchronises. */
fv_status fv_euler_train_input_grad(fv_euler_trainer *tr, float *dst);

/* One Adam update of the net's master parameters from grads, then re-pack. */
fv_status fv_euler_adam_step(fv_euler_trainer *tr);

fv_status fv_euler_train_set_lr(fv_euler_trainer *tr, float lr);

void fv_euler_train_destroy(fv_euler_trainer *tr);

/* Message of the last failing call on this thread ("" if none). */
const char *fv_last_error(void);

/* ------------------------------------------------------------------------
 * Training of the coefficient network (thesis eq 2.28, section 2.5.3):
 * Loss = sum_{t=1..T} MSE(Q_ref(t), Q_pred(t)) over T learned Heun steps at
 * a fixed step from the coarse initial states, the MSE averaged over cells
 * and variables with variable v divided by scale[v].  The forward keeps
 * every stage's input, activations and coefficients; the reverse pass runs
 * the Heun adjoint, the finite-volume adjoint (flux Jacobians of the branch
 * taken, MINMOD derivative on fallback faces, plain-scheme adjoint for
 * redone steps) and the network's BF16 MFMA backward with FP32 accumulation.
 * Gradient reductions are in a fixed order (run-to-run identical).
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t struct_size; /* sizeof(fv_train_config) */
    int32_t B;            /* windows per batch */
    int32_t nx, ny;       /* periodic coarse grid (nx % 16 == 0, nx*ny % 64 == 0) */
    int32_t T;            /* largest number of unrolled steps */
    int32_t flux;         /* FV_FLUX_HLLE | FV_FLUX_RUSANOV */
    double lx, ly;        /* domain size */
    double dt;            /* fixed step */
    double g;             /* gravity */
    double h_ref;         /* reference depth of the pressure term, > 0 */
    float scale[3];       /* loss scale of h, hu, hv */
    float lr, beta1, beta2, eps; /* Adam */
    int32_t direct;       /* 0: the learned stencil-coefficient scheme (fv_learned_step); 1: the
                             direct face-state scheme (fv_direct_step, section 5.3) */
    int32_t blend;        /* 1 (with direct = 0): the stencil-coefficient scheme with the
                             flux-limiter blend of its face fluxes (fv_blend_step, section 2.5.3
                             second approach), differentiated through the limiter and the
                             low-resolution flux; 0 otherwise */
} fv_train_config;

typedef struct fv_trainer fv_trainer;

/* Device workspace of a trainer (saved states, activations, coefficients,
 * adjoints); 0 if the configuration is invalid. */
size_t fv_train_workspace_bytes(const fv_train_config *cfg);

/* Create a trainer for model m (its stream is used).  grads, adam_m, adam_v:
 * caller-owned device FP32 vectors of fv_model_param_count() elements
 * (grads is overwritten by each fv_train_step; the Adam moments must start
 * at zero).  workspace: >= fv_train_workspace_bytes, 256-byte aligned. */
fv_status fv_train_create(const fv_train_config *cfg, fv_model *m, float *grads, float *adam_m, float *adam_v,
                          void *workspace, size_t workspace_bytes, fv_trainer **out);

/* One loss/gradient evaluation.  q0: device [B][3][ny][nx] FP32 initial
 * states; targets: device [T][B][3][ny][nx] reference states after steps
 * 1..T (1 <= T <= cfg.T).  Writes d loss / d theta into grads.  Sync point:
 * *loss (host) receives the loss; stats (nullable) the fallback faces and
 * redone steps of the rollout. */
fv_status fv_train_step(fv_trainer *tr, const float *q0, const float *targets, int T, double *loss,
                        fv_learned_stats *stats);

/* d loss / d q0 of the last fv_train_step, copied to dst (device,
 * [B][3][ny][nx]). */
fv_status fv_train_input_grad(fv_trainer *tr, float *dst);

/* State after step t (0..T) of the last fv_train_step's rollout (device). */
fv_status fv_train_state(fv_trainer *tr, int t, float *dst);

/* Adam update of the model's master parameters from grads, then re-pack
 * the model's weights (async on the model's stream). */
fv_status fv_adam_step(fv_trainer *tr);

/* Learning rate of the following fv_adam_step calls (a schedule is the
 * caller's; the loss of eq 2.28 is minimised with Adam).  lr must be > 0. */
fv_status fv_train_set_lr(fv_trainer *tr, float lr);

void fv_train_destroy(fv_trainer *tr);

/* Block-average coarsening (exact cell averages): coarse[v][J][I] = mean of
 * the factor x factor block of fine[v] (FP32 device arrays, nx and ny
 * multiples of factor), FP64 accumulation.  Async on stream. */
fv_status fv_coarsen(const float *fine, int nvar, int nx, int ny, int factor, float *coarse, void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent FP32 solves (shallow water
 * over a bed, or Euler; HLLE, MINMOD, Heun, CFL time step; square grids on
 * a square domain), and of learned shallow-water solves (the network of the
 * thesis's section 2.5.3 with the server's model, periodic, flat bed, fixed
 * Delta t, Heun; the plain scheme redoes inadmissible steps).  Requests wait
 * in a FIFO queue; at each round boundary
 * those whose device footprint (fv_request_bytes) fits the free part of the
 * caller's memory pool are admitted (a later request may pass one that does
 * not fit).  A round advances every active solve by up to steps_per_round
 * steps, each stage of each step being one batched launch over the tiles of
 * all active solves of an equation type; for the learned solves each step
 * is four batched launches (per stage, one launch runs the network pass
 * (BF16 MFMA) and the learned stage of every learned solve, the
 * coefficients staying on chip; then commit-or-redo and redo), or, in rounds
 * with many learned tiles (learned_split), six (the network pass and the
 * learned stage as separate launches), the network pass itself running
 * layer by layer in rounds with more learned cells still (learned_layered).  A round's launches are recorded once, per kinds of work present
 * and number of steps, into a hipGraph that every later round replays: the
 * kernels read their tile counts from the device work-lists, and between
 * replays the host rewrites those lists and sets each launch's grid to its
 * list's tiles.
 * Finished solves are copied back and their memory returns to the pool.
 * The single-solve calls (fv_run, fv_learned_step) run the same kernels as a
 * batch of one, so a solve's result is bit-identical alone and in any mix.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t struct_size;    /* sizeof(fv_server_config) */
    int32_t max_solves;      /* solve slots */
    int32_t steps_per_round; /* K: steps between admission/retirement points */
    int32_t direct;          /* 0: replay captured graphs; 1: launch every kernel directly (same
                                results; for comparison) */
    uint64_t max_items;      /* most tiles (workgroups) one batched launch may hold: admission keeps
                                every launch within it; a request that alone needs more is rejected */
    const fv_model *model;   /* network of the learned requests (NULL: none accepted); its
                                packed weights must be ready (its stream synchronised) */
    int32_t learned_split;   /* network tiles (8 x 8 cells) in a round's first step from which the
                                round runs the network pass and the learned stage as separate
                                launches (throughput) instead of one launch per stage that keeps
                                the coefficients on chip (latency); 0: 4 x the workgroups of the
                                network pass resident at once.  Same results either way. */
    int32_t learned_layered; /* 16 x 16-cell tiles in a round's first step from which a round with
                                separate launches runs the network pass layer by layer (five
                                launches per stage on 16 x 16 tiles, activations in the pool's
                                scratch; all learned sides multiples of 16) instead of as one
                                launch; 0: 768; -1: never.  Same results either way. */
    uint64_t act_pixels;     /* capacity in cells of that activation scratch (128 bytes per cell,
                                counted in fv_server_pool_overhead); rounds with more learned cells
                                use the one-launch network pass; 0: no scratch (never layer by
                                layer) */
    int32_t max_bypass;      /* admission ageing: after a queued request has not fitted in this many
                                rounds, no request queued behind it is admitted until it is, so a
                                large request waits a bounded number of rounds (the running solves'
                                remaining rounds plus max_bypass); 0: 8; -1: never (plain first fit,
                                later requests may pass it indefinitely) */
    int32_t reserved0;       /* must be 0 */
} fv_server_config;

typedef struct {
    uint32_t struct_size;    /* sizeof(fv_request) */
    int32_t eqn;             /* FV_SWE (with the given bed, or a zero bed) | FV_EULER */
    int32_t n;               /* cells per side, >= 8 */
    int32_t bc;              /* FV_BC_PERIODIC | FV_BC_WALL on both axes */
    int64_t steps;           /* time steps to run */
    double cfl, g, gamma;
    double h_ref;            /* SWE pressure reference depth, 0 = mean initial depth */
    const float *q0;         /* host [nvar][n][n]; copied by fv_server_submit */
    const float *bed;        /* host [n][n] (SWE, nullable); copied */
    int32_t learned;         /* 1: learned solve (SWE, periodic, no bed, n % 16 == 0) */
    int32_t reserved1;       /* must be 0 */
    double dt_fixed;         /* learned: the fixed time step (> 0); `steps` learned steps */
    double lx;               /* side of the square domain (0: the unit square) */
} fv_request;

typedef struct {
    int32_t state;           /* 0 queued, 1 running, 2 done, 3 failed (inadmissible) */
    int32_t rounds_queued;   /* rounds the request stayed queued before its admission */
    int64_t steps_done;
    double t_submit, t_admit, t_done; /* seconds since fv_server_create */
    double sim_time;         /* simulated time reached (done requests) */
    int64_t fallback_faces;  /* learned: face sides that fell back to MINMOD */
    int64_t redone_steps;    /* learned: steps redone with the plain scheme */
} fv_request_info;

typedef struct fv_server fv_server;

typedef struct {
    int64_t rounds;          /* rounds that launched work */
    int64_t graph_replays;   /* of which replayed from a captured graph */
    int64_t grid_updates;    /* launch grids reset before replays */
    int32_t graphs_captured; /* distinct graphs captured so far */
    int32_t layered_rounds;  /* rounds whose network pass ran layer by layer */
    double host_launch_s;    /* host seconds spent enqueueing rounds' launches (or graphs) */
    double host_wait_s;      /* host seconds spent waiting for rounds' work to finish */
    double host_capture_s;   /* host seconds spent capturing and instantiating graphs */
    double host_admit_s;     /* host seconds spent admitting requests (uploads, first CFL rates) */
    double host_retire_s;    /* host seconds spent copying back finished requests */
} fv_server_stats;

/* Pool bytes taken by the server's tables (solve table, work-lists). */
size_t fv_server_pool_overhead(const fv_server_config *cfg);

/* Device bytes one request occupies while admitted; 0 if invalid. */
size_t fv_request_bytes(const fv_request *r);

/* Create a server over a caller-owned device pool (256-byte aligned); its
 * work is enqueued on stream.  A NULL stream (where graphs cannot be
 * captured) makes the server create a non-blocking stream of its own, which
 * fv_server_destroy destroys; every round ends synchronised either way. */
fv_status fv_server_create(const fv_server_config *cfg, void *pool, size_t pool_bytes, void *stream,
                           fv_server **out);

/* Queue a request (inputs are copied); *id identifies it. */
fv_status fv_server_submit(fv_server *s, const fv_request *r, int64_t *id);

/* Admit what fits, run one round, retire finished solves.  Sync point.
 * Reports the running and queued request counts after the round. */
fv_status fv_server_round(fv_server *s, int32_t *n_active, int32_t *n_queued);

fv_status fv_server_info(fv_server *s, int64_t id, fv_request_info *info);

/* Round and graph counters. */
fv_status fv_server_get_stats(fv_server *s, fv_server_stats *out);

/* Copy a finished request's final state to dst (host, [nvar][n][n]);
 * FV_E_INADMISSIBLE if it failed (dst then holds the failing state). */
fv_status fv_server_result(fv_server *s, int64_t id, float *dst);

/* Forget a finished request (frees its host copy). */
fv_status fv_server_release(fv_server *s, int64_t id);

void fv_server_destroy(fv_server *s);

/* ------------------------------------------------------------------------
 * Shallow water on the sphere (thesis section 3.3, on the logically
 * rectangular grid of section 2.4).
 *
 * Grid: 2n x n cells on the computational rectangle [-3,1] x [-1,1] (cell
 * (i, j) spans x in [-3 + 2i/n, -3 + 2(i+1)/n], y in [-1 + 2j/n, ...]); the
 * square [-1,1]^2 maps to the northern hemisphere (the disk mapping of
 * section 2.4 with R = 1, D(d) = d/sqrt 2, lifted by z = sqrt(1 - x^2 - y^2)),
 * the square [-3,-1] x [-1,1] reflected (x -> -2 - x) to the southern one.
 * Neighbours: periodic in x; across y = -+1 the cell of column 2n-1-i.
 * Unit sphere; time in the unit of the configured g and omega.
 *
 * State: [4][n][2n] (h, hu, hv, hw) with Cartesian momenta, element type of
 * prec.  Per face a unit normal n and tangent t in the tangent plane at the
 * edge midpoint (great-circle edge length); face states (MINMOD along the
 * index lines, eq 2.18, or first order) rotated into (n, t, r), the 1D
 * Riemann problem (HLLE, Rusanov or Roe; eq 2.12-2.16) along n, the flux
 * rotated back (eq 2.24); every cell's momentum equation subtracts its own
 * flux against the sum of its outward edge normals times lengths (eq 3.1)
 * and adds the Coriolis force -2 omega z (x cross m) (eq 3.2); after every
 * stage the momentum is projected onto the tangent plane at the cell centre
 * (the tangency forcing of eq 3.2).  Delta t from the CFL condition: cfl /
 * max over cells of (|m|/h + sqrt(g h)) perimeter / (2 area), reduced on the
 * device every step, or dt_fixed.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t struct_size; /* sizeof(fv_sphere_config) */
    int32_t prec;         /* FV_F32 | FV_F64 */
    int32_t n;            /* cells per hemisphere side, 4..8192: grid 2n x n */
    int32_t flux;         /* FV_FLUX_* */
    int32_t recon;        /* FV_RECON_MINMOD | FV_RECON_FIRST */
    int32_t rk_stages;    /* 1, 2 (Heun) or 3 */
    int32_t reserved0;    /* must be 0 */
    int32_t pad;
    double cfl;           /* in (0, 1] unless dt_fixed > 0 */
    double dt_fixed;      /* > 0: fixed Delta t */
    double g;             /* gravity, > 0 */
    double omega;         /* rotation rate of the Coriolis term */
} fv_sphere_config;

typedef struct fv_sphere fv_sphere;

/* Device workspace bytes (geometry, face fluxes, stage buffers, reduction
 * slots); 0 if cfg is invalid. */
size_t fv_sphere_workspace_bytes(const fv_sphere_config *cfg);

/* Create a solver over caller-owned device memory: q [4][n][2n] updated in
 * place, workspace (256-byte aligned) of fv_sphere_workspace_bytes.
 * Computes the grid geometry on the device and checks that the initial
 * state is admissible (FV_E_INADMISSIBLE; this synchronises the stream). */
fv_status fv_sphere_init(const fv_sphere_config *cfg, void *q, void *workspace, size_t workspace_bytes, void *stream,
                         fv_sphere **out);

/* Enqueue nsteps >= 0 full steps (no host synchronisation). */
fv_status fv_sphere_run(fv_sphere *s, int64_t nsteps);

/* Sync point: simulated time and completed steps; FV_E_INADMISSIBLE if a
 * cell reached h <= 0 or a non-finite value (later steps were skipped). */
fv_status fv_sphere_time(fv_sphere *s, double *t, int64_t *steps);

/* Sync point: copy the cell centres (unit vectors, [3][n][2n], solver
 * precision) to the device buffer dst, e.g. to sample initial states. */
fv_status fv_sphere_centres(fv_sphere *s, void *dst);

/* Sync point: total mass sum h A and energy sum (g h^2/2 + |m|^2/(2h)) A
 * (eq 5.1) in double precision, fixed summation order; out holds 2 doubles. */
fv_status fv_sphere_totals(fv_sphere *s, double *out);

void fv_sphere_destroy(fv_sphere *s);

#ifdef __cplusplus
}
#endif

#endif /* FV_H */
