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
    int32_t reserved0;    /* must be 0 */
    double lx, ly;        /* domain [0,lx] x [0,ly], > 0 */
    double cfl;           /* Courant number in (0, 1] */
    double dt_fixed;      /* > 0: fixed Delta t, the CFL reduction is skipped */
    double g;             /* gravity (SWE), > 0 */
    double gamma;         /* ratio of specific heats (Euler), > 1 */
    double h_ref;         /* SWE: reference depth h0 of the pressure term, carried as
                             g (h - h0)(h + h0)/2 (a constant shift of every face flux that
                             cancels in each cell's divergence and keeps float rounding
                             proportional to |h - h0|); 0 = mean depth of the initial state */
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

/* Message of the last failing call on this thread ("" if none). */
const char *fv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FV_H */
