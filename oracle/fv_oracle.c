/*
 * Reference finite-volume solver, double precision, plain loops.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no source, header, table or helper with the HIP library.
 *
 * What it computes (thesis "A Machine Learning accelerated geophysical fluid
 * solver", section 2):
 *   - 2D shallow-water equations, eq 2.3, state (h, hu, hv), optional bed b
 *     entering through the bed-slope source of eq 2.3;
 *   - 2D Euler equations with the ideal-gas law of eq 2.4, state
 *     (rho, rho u, rho v, E), flux matrix of section 4.2;
 *   - cell averages on a uniform grid (section 2.3.1, eq 2.6), conservative
 *     update eq 2.9 / eq 2.23 summed over the four faces of each cell;
 *   - MINMOD slope-limited face states (eq 2.18) or first-order states;
 *   - numerical fluxes: HLLE (eq 2.16), Rusanov (eq 2.12), Roe (eq 2.14),
 *     each solved in the face-normal frame (eq 2.24: for axis-aligned faces
 *     the rotation swaps the two momentum components);
 *   - time integration: Heun (eq 2.19), the three-stage SSP scheme (eq 2.20)
 *     or one forward-Euler stage;
 *   - time step from the CFL condition (eq 2.10) evaluated every step;
 *   - conserved totals and the total energy of eq 5.1.
 *
 * Readings where the thesis is silent or garbled (each one is listed in the
 * design notes of the repository):
 *   - N cells of width L/N (the grid paragraph of section 2.3.1 has N+1);
 *   - MINMOD second case compares |b| with |a|; the face state on the right
 *     of face i+1/2 extrapolates cell i+1 towards the face (minus sign);
 *   - Delta t = CFL / max_i ((|u_i|+c_i)/dx + (|v_i|+c_i)/dy), once per step;
 *   - HLLE speeds: s_L = min(u_L - c_L, u~ - c~, 0), s_R = max(u_R + c_R,
 *     u~ + c~, 0) with Roe averages (Einfeldt);
 *   - Rusanov speed from the reconstructed face states;
 *   - Roe flux without entropy fix;
 *   - bed source: hydrostatic reconstruction of Audusse et al. (2004),
 *     second-order form, which keeps a lake at rest exactly;
 *   - wall boundary: mirrored ghost cells with the normal momentum negated;
 *   - face states with h <= 0 (or rho <= 0, p <= 0) fall back to the cell
 *     average of that side.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_SWE = 0, ORC_EULER = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1 };
enum { ORC_FLUX_HLLE = 0, ORC_FLUX_RUSANOV = 1, ORC_FLUX_ROE = 2 };
enum { ORC_RECON_MINMOD = 0, ORC_RECON_FIRST = 1 };

typedef struct {
    int32_t eqn;        /* ORC_SWE or ORC_EULER */
    int32_t nx, ny;     /* cells */
    int32_t bc_x, bc_y; /* boundary per axis */
    int32_t flux;       /* numerical flux */
    int32_t recon;      /* face-state reconstruction */
    int32_t rk_stages;  /* 1, 2 (Heun) or 3 (SSP three-stage) */
    int32_t shadow_f32; /* 1: round the state to float after every stage */
    int32_t nthreads;   /* OpenMP threads for the row loops */
    double lx, ly;      /* domain [0,lx] x [0,ly] */
    double cfl;         /* Courant number */
    double dt_fixed;    /* > 0: use this step instead of the CFL rule */
    double g, gamma;
} orc_config;

static int nvar_of(const orc_config *c) { return c->eqn == ORC_SWE ? 3 : 4; }

/* ---------------------------------------------------------------- ghosts */

/* Map a possibly out-of-range index along one axis.  Returns the interior
 * index and sets *flip when the ghost is a wall mirror image. */
static int map_index(int i, int n, int bc, int *flip)
{
    if (i >= 0 && i < n) return i;
    if (bc == ORC_BC_PERIODIC) return ((i % n) + n) % n;
    *flip = 1;
    return i < 0 ? -1 - i : 2 * n - 1 - i;
}

/* Cell value of variable v at (i,j); (i,j) may lie in the ghost layer of one
 * axis.  Wall ghosts negate the momentum normal to that wall. */
static double cellv(const orc_config *c, const double *q, int v, int i, int j)
{
    int fx = 0, fy = 0;
    int ii = map_index(i, c->nx, c->bc_x, &fx);
    int jj = map_index(j, c->ny, c->bc_y, &fy);
    double s = 1.0;
    if (fx && v == 1) s = -s;
    if (fy && v == 2) s = -s;
    return s * q[(size_t)v * c->nx * c->ny + (size_t)jj * c->nx + ii];
}

static double bedv(const orc_config *c, const double *b, int i, int j)
{
    int f = 0;
    int ii = map_index(i, c->nx, c->bc_x, &f);
    int jj = map_index(j, c->ny, c->bc_y, &f);
    return b[(size_t)jj * c->nx + ii];
}

/* ------------------------------------------------------ physics, 1D normal */

/* Pressure of a normal-frame Euler state s = (rho, rho n, rho t, E), eq 2.4. */
static double euler_p(const orc_config *c, const double *s)
{
    return (c->gamma - 1.0) * (s[3] - 0.5 * (s[1] * s[1] + s[2] * s[2]) / s[0]);
}

/* Velocity component m/h; a dry SWE state (h == 0, reachable only through
 * the hydrostatic reconstruction) has zero velocity. */
static double vel(double m, double h) { return h > 0.0 ? m / h : 0.0; }

/* Physical flux in the normal direction of a normal-frame state:
 * SWE (eq 2.3): (hn, hn u + g h^2/2, ht u); Euler (section 4.2):
 * (rho n, rho n u + p, rho t u, u (E + p)), u = normal velocity. */
static void phys_flux(const orc_config *c, const double *s, double *f)
{
    if (c->eqn == ORC_SWE) {
        double u = vel(s[1], s[0]);
        f[0] = s[1];
        f[1] = s[1] * u + 0.5 * c->g * s[0] * s[0];
        f[2] = s[2] * u;
    } else {
        double u = s[1] / s[0];
        double p = euler_p(c, s);
        f[0] = s[1];
        f[1] = s[1] * u + p;
        f[2] = s[2] * u;
        f[3] = u * (s[3] + p);
    }
}

static double sound_speed(const orc_config *c, const double *s)
{
    if (c->eqn == ORC_SWE) return sqrt(c->g * s[0]);
    return sqrt(c->gamma * euler_p(c, s) / s[0]);
}

/* Roe-averaged normal velocity, tangential velocity, sound speed (and
 * enthalpy for Euler) of two normal-frame states. */
typedef struct { double u, v, c, H; } roe_avg;

static roe_avg roe_average(const orc_config *c, const double *sl, const double *sr)
{
    roe_avg a;
    double wl = sqrt(sl[0]), wr = sqrt(sr[0]);
    double ul = vel(sl[1], sl[0]), ur = vel(sr[1], sr[0]);
    double vl = vel(sl[2], sl[0]), vr = vel(sr[2], sr[0]);
    a.u = (wl * ul + wr * ur) / (wl + wr);
    a.v = (wl * vl + wr * vr) / (wl + wr);
    if (c->eqn == ORC_SWE) {
        a.c = sqrt(c->g * 0.5 * (sl[0] + sr[0]));
        a.H = 0.0;
    } else {
        double Hl = (sl[3] + euler_p(c, sl)) / sl[0];
        double Hr = (sr[3] + euler_p(c, sr)) / sr[0];
        a.H = (wl * Hl + wr * Hr) / (wl + wr);
        double c2 = (c->gamma - 1.0) * (a.H - 0.5 * (a.u * a.u + a.v * a.v));
        a.c = sqrt(c2 > 0.0 ? c2 : 0.0);
    }
    return a;
}

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* HLLE, eq 2.16, Einfeldt speeds clamped with zero. */
static void flux_hlle(const orc_config *c, const double *sl, const double *sr, double *F)
{
    int nv = nvar_of(c);
    double fl[4], fr[4];
    phys_flux(c, sl, fl);
    phys_flux(c, sr, fr);
    roe_avg a = roe_average(c, sl, sr);
    double cl = sound_speed(c, sl), cr = sound_speed(c, sr);
    double ul = vel(sl[1], sl[0]), ur = vel(sr[1], sr[0]);
    double sL = dmin(dmin(ul - cl, a.u - a.c), 0.0);
    double sR = dmax(dmax(ur + cr, a.u + a.c), 0.0);
    if (sR - sL == 0.0) {
        for (int k = 0; k < nv; k++) F[k] = 0.5 * (fl[k] + fr[k]);
        return;
    }
    for (int k = 0; k < nv; k++)
        F[k] = (sR * fl[k] - sL * fr[k] + sL * sR * (sr[k] - sl[k])) / (sR - sL);
}

/* Rusanov, eq 2.12: one half of the largest |eigenvalue| of the two face
 * states multiplies the jump. */
static void flux_rusanov(const orc_config *c, const double *sl, const double *sr, double *F)
{
    int nv = nvar_of(c);
    double fl[4], fr[4];
    phys_flux(c, sl, fl);
    phys_flux(c, sr, fr);
    double al = fabs(vel(sl[1], sl[0])) + sound_speed(c, sl);
    double ar = fabs(vel(sr[1], sr[0])) + sound_speed(c, sr);
    double a = dmax(al, ar);
    for (int k = 0; k < nv; k++) F[k] = 0.5 * (fl[k] + fr[k]) - 0.5 * a * (sr[k] - sl[k]);
}

/* Roe, eq 2.13/2.14: F = (F_L + F_R)/2 - 1/2 sum_p |lambda_p| alpha_p r_p with
 * the Roe-averaged eigen-system of the normal-frame Jacobian. */
static void flux_roe(const orc_config *c, const double *sl, const double *sr, double *F)
{
    int nv = nvar_of(c);
    double fl[4], fr[4], d[4];
    phys_flux(c, sl, fl);
    phys_flux(c, sr, fr);
    for (int k = 0; k < nv; k++) d[k] = sr[k] - sl[k];
    roe_avg a = roe_average(c, sl, sr);
    double u = a.u, v = a.v, cc = a.c;
    for (int k = 0; k < nv; k++) F[k] = 0.5 * (fl[k] + fr[k]);
    if (c->eqn == ORC_SWE) {
        /* waves: u-c (acoustic), u (shear), u+c (acoustic) */
        double a1 = ((u + cc) * d[0] - d[1]) / (2.0 * cc);
        double a3 = (d[1] - (u - cc) * d[0]) / (2.0 * cc);
        double a2 = d[2] - v * d[0];
        double l1 = fabs(u - cc), l2 = fabs(u), l3 = fabs(u + cc);
        double r1[3] = {1.0, u - cc, v};
        double r2[3] = {0.0, 0.0, 1.0};
        double r3[3] = {1.0, u + cc, v};
        for (int k = 0; k < 3; k++)
            F[k] -= 0.5 * (l1 * a1 * r1[k] + l2 * a2 * r2[k] + l3 * a3 * r3[k]);
    } else {
        double H = a.H, gm1 = c->gamma - 1.0;
        double a3 = d[2] - v * d[0];                       /* shear */
        double d5 = d[3] - a3 * v;                         /* energy jump minus shear part */
        double a2 = gm1 / (cc * cc) * (d[0] * (H - u * u) + u * d[1] - d5); /* entropy */
        double a1 = (d[0] * (u + cc) - d[1] - cc * a2) / (2.0 * cc);
        double a4 = d[0] - (a1 + a2);
        double l1 = fabs(u - cc), l2 = fabs(u), l4 = fabs(u + cc);
        double r1[4] = {1.0, u - cc, v, H - u * cc};
        double r2[4] = {1.0, u, v, 0.5 * (u * u + v * v)};
        double r3[4] = {0.0, 0.0, 1.0, v};
        double r4[4] = {1.0, u + cc, v, H + u * cc};
        for (int k = 0; k < 4; k++)
            F[k] -= 0.5 * (l1 * a1 * r1[k] + l2 * a2 * r2[k] + l2 * a3 * r3[k] + l4 * a4 * r4[k]);
    }
}

static void numflux(const orc_config *c, const double *sl, const double *sr, double *F)
{
    if (c->flux == ORC_FLUX_RUSANOV) flux_rusanov(c, sl, sr, F);
    else if (c->flux == ORC_FLUX_ROE) flux_roe(c, sl, sr, F);
    else flux_hlle(c, sl, sr, F);
}

/* ------------------------------------------------------ reconstruction */

/* MINMOD limiter of eq 2.18 (second case read as |b| < |a|). */
static double minmod(double a, double b)
{
    if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0.0;
    return fabs(a) <= fabs(b) ? a : b;
}

/* Is a Cartesian-frame cell/face state admissible (h > 0; rho > 0, p > 0)? */
static int admissible(const orc_config *c, const double *s)
{
    if (!(s[0] > 0.0)) return 0;
    if (c->eqn == ORC_EULER) {
        double p = (c->gamma - 1.0) * (s[3] - 0.5 * (s[1] * s[1] + s[2] * s[2]) / s[0]);
        if (!(p > 0.0)) return 0;
    }
    return 1;
}

/* Face data of one face: the numerical flux seen by the cell on the left
 * (Fl) and by the cell on the right (Fr), Cartesian frame.  They differ only
 * by the hydrostatic correction when a bed is present.  Also returns the
 * reconstructed depth and bed on both sides (used by the bed source). */
typedef struct {
    double Fl[4], Fr[4];
    double hl, zl, hr, zr;
} face_data;

/* Compute the face between cell (i,j) and its neighbour along axis
 * (0: x, neighbour (i+1,j); 1: y, neighbour (i,j+1)). */
static void face(const orc_config *c, const double *q, const double *b, int axis, int i, int j,
                 face_data *fd)
{
    int nv = nvar_of(c);
    int di = axis == 0 ? 1 : 0, dj = axis == 0 ? 0 : 1;
    double m1[5], c0[5], c1[5], p2[5];   /* conserved vars + (bathy) eta */
    double QL[5], QR[5];
    int nrec = nv + (b ? 1 : 0);
    for (int v = 0; v < nv; v++) {
        m1[v] = cellv(c, q, v, i - di, j - dj);
        c0[v] = cellv(c, q, v, i, j);
        c1[v] = cellv(c, q, v, i + di, j + dj);
        p2[v] = cellv(c, q, v, i + 2 * di, j + 2 * dj);
    }
    if (b) {
        m1[nv] = m1[0] + bedv(c, b, i - di, j - dj);
        c0[nv] = c0[0] + bedv(c, b, i, j);
        c1[nv] = c1[0] + bedv(c, b, i + di, j + dj);
        p2[nv] = p2[0] + bedv(c, b, i + 2 * di, j + 2 * dj);
    }
    for (int v = 0; v < nrec; v++) {
        if (c->recon == ORC_RECON_FIRST) {
            QL[v] = c0[v];
            QR[v] = c1[v];
        } else {
            QL[v] = c0[v] + 0.5 * minmod(c0[v] - m1[v], c1[v] - c0[v]);
            QR[v] = c1[v] - 0.5 * minmod(c1[v] - c0[v], p2[v] - c1[v]);
        }
    }
    if (!admissible(c, QL)) for (int v = 0; v < nrec; v++) QL[v] = c0[v];
    if (!admissible(c, QR)) for (int v = 0; v < nrec; v++) QR[v] = c1[v];

    double sl[4], sr[4], F[4];
    int nm = axis == 0 ? 1 : 2, tm = axis == 0 ? 2 : 1; /* normal / tangential momentum */

    if (!b) {
        /* rotate into the face-normal frame (eq 2.24) */
        sl[0] = QL[0]; sl[1] = QL[nm]; sl[2] = QL[tm];
        sr[0] = QR[0]; sr[1] = QR[nm]; sr[2] = QR[tm];
        if (nv == 4) { sl[3] = QL[3]; sr[3] = QR[3]; }
        numflux(c, sl, sr, F);
        for (int k = 0; k < 4; k++) fd->Fl[k] = fd->Fr[k] = 0.0;
        fd->Fl[0] = F[0]; fd->Fl[nm] = F[1]; fd->Fl[tm] = F[2];
        if (nv == 4) fd->Fl[3] = F[3];
        for (int k = 0; k < nv; k++) fd->Fr[k] = fd->Fl[k];
        fd->hl = fd->zl = fd->hr = fd->zr = 0.0;
        return;
    }

    /* Hydrostatic reconstruction (Audusse et al. 2004), SWE with bed. */
    double hl = QL[0], hr = QR[0];
    double zl = QL[3] - QL[0], zr = QR[3] - QR[0];   /* bed = eta - h at the face */
    double zf = dmax(zl, zr);
    double hls = dmax(0.0, QL[3] - zf), hrs = dmax(0.0, QR[3] - zf);
    double ul = QL[nm] / hl, vl = QL[tm] / hl;
    double ur = QR[nm] / hr, vr = QR[tm] / hr;
    sl[0] = hls; sl[1] = hls * ul; sl[2] = hls * vl;
    sr[0] = hrs; sr[1] = hrs * ur; sr[2] = hrs * vr;
    if (hls > 0.0 || hrs > 0.0) numflux(c, sl, sr, F);
    else F[0] = F[1] = F[2] = 0.0;
    for (int k = 0; k < 4; k++) fd->Fl[k] = fd->Fr[k] = 0.0;
    fd->Fl[0] = F[0]; fd->Fl[nm] = F[1]; fd->Fl[tm] = F[2];
    for (int k = 0; k < 3; k++) fd->Fr[k] = fd->Fl[k];
    fd->Fl[nm] += 0.5 * c->g * (hl * hl - hls * hls);
    fd->Fr[nm] += 0.5 * c->g * (hr * hr - hrs * hrs);
    fd->hl = hl; fd->zl = zl; fd->hr = hr; fd->zr = zr;
}

/* --------------------------------------------------------- spatial operator */

/* L(q) of the semi-discrete scheme: minus the flux divergence over the four
 * faces of every cell (eq 2.23 with unit-normal axis faces) plus the bed
 * source.  The x part and the y part are formed separately and then added. */
void orc_rhs(const orc_config *c, const double *q, const double *b, double *L)
{
    int nx = c->nx, ny = c->ny, nv = nvar_of(c);
    double dx = c->lx / nx, dy = c->ly / ny;
    size_t plane = (size_t)nx * ny;
    int nth = c->nthreads > 0 ? c->nthreads : 1;
    (void)nth;
#pragma omp parallel for schedule(static) num_threads(nth)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            face_data xm, xp, ym, yp;  /* faces i-1/2, i+1/2, j-1/2, j+1/2 */
            face(c, q, b, 0, i - 1, j, &xm);
            face(c, q, b, 0, i, j, &xp);
            face(c, q, b, 1, i, j - 1, &ym);
            face(c, q, b, 1, i, j, &yp);
            for (int v = 0; v < nv; v++) {
                /* cell (i,j) is on the right of face i-1/2 and on the left of i+1/2 */
                double lx = -(xp.Fl[v] - xm.Fr[v]) / dx;
                double ly = -(yp.Fl[v] - ym.Fr[v]) / dy;
                L[v * plane + (size_t)j * nx + i] = lx + ly;
            }
            if (b) {
                /* centred bed source of the hydrostatic reconstruction:
                 * -g (h_{i-1/2+} + h_{i+1/2-})/2 (z_{i+1/2-} - z_{i-1/2+}) / dx */
                double sx = -c->g * 0.5 * (xm.hr + xp.hl) * (xp.zl - xm.zr) / dx;
                double sy = -c->g * 0.5 * (ym.hr + yp.hl) * (yp.zl - ym.zr) / dy;
                L[1 * plane + (size_t)j * nx + i] += sx;
                L[2 * plane + (size_t)j * nx + i] += sy;
            }
        }
    }
}

/* Face fluxes for inspection: Fx[v][j][i] for faces i-1/2 (i = 0..nx),
 * Fy[v][j][i] for faces j-1/2 (j = 0..ny), as seen from the cell on the
 * right/top (flat bottom: both sides see the same flux). */
void orc_face_fluxes(const orc_config *c, const double *q, const double *b, double *Fx, double *Fy)
{
    int nx = c->nx, ny = c->ny, nv = nvar_of(c);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i <= nx; i++) {
            face_data fd;
            face(c, q, b, 0, i - 1, j, &fd);
            for (int v = 0; v < nv; v++) Fx[(size_t)v * (nx + 1) * ny + (size_t)j * (nx + 1) + i] = fd.Fr[v];
        }
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i < nx; i++) {
            face_data fd;
            face(c, q, b, 1, i, j - 1, &fd);
            for (int v = 0; v < nv; v++) Fy[(size_t)v * nx * (ny + 1) + (size_t)j * nx + i] = fd.Fr[v];
        }
}

/* One numerical flux on normal-frame states (for brute-force checks). */
void orc_numflux(const orc_config *c, const double *sl, const double *sr, double *F)
{
    numflux(c, sl, sr, F);
}

void orc_physflux(const orc_config *c, const double *s, double *F) { phys_flux(c, s, F); }

/* ------------------------------------------------------------- time step */

/* Largest a_i = (|u_i| + c_i)/dx + (|v_i| + c_i)/dy over the cells (eq 2.10
 * applied to both axes of the unsplit scheme). */
double orc_max_rate(const orc_config *c, const double *q)
{
    int nx = c->nx, ny = c->ny;
    double dx = c->lx / nx, dy = c->ly / ny;
    size_t plane = (size_t)nx * ny;
    double amax = 0.0;
    for (size_t k = 0; k < plane; k++) {
        double s[4];
        for (int v = 0; v < nvar_of(c); v++) s[v] = q[v * plane + k];
        double u = s[1] / s[0], w = s[2] / s[0];
        double cs = sound_speed(c, s);
        double a = (fabs(u) + cs) / dx + (fabs(w) + cs) / dy;
        if (a > amax) amax = a;
    }
    return amax;
}

double orc_dt(const orc_config *c, const double *q)
{
    if (c->dt_fixed > 0.0) return c->dt_fixed;
    return c->cfl / orc_max_rate(c, q);
}

/* ---------------------------------------------------------------- stepping */

static void round_to_float(double *x, size_t n)
{
    for (size_t k = 0; k < n; k++) x[k] = (double)(float)x[k];
}

/* Advance q by one full step in place; returns 0, or -4 if a cell became
 * inadmissible (q then holds that state).  *dt_used receives Delta t. */
int orc_step(const orc_config *c, double *q, const double *b, double *dt_used)
{
    size_t n = (size_t)nvar_of(c) * c->nx * c->ny;
    double dt = orc_dt(c, q);
    double *L = (double *)malloc(n * sizeof(double));
    double *q1 = (double *)malloc(n * sizeof(double));
    double *q2 = (double *)malloc(n * sizeof(double));
    if (!L || !q1 || !q2) { free(L); free(q1); free(q2); return -2; }

    /* stage 1 (all schemes): q1 = q + dt L(q) */
    orc_rhs(c, q, b, L);
    for (size_t k = 0; k < n; k++) q1[k] = q[k] + dt * L[k];
    if (c->shadow_f32) round_to_float(q1, n);

    if (c->rk_stages == 1) {
        memcpy(q, q1, n * sizeof(double));
    } else if (c->rk_stages == 2) {
        /* Heun, eq 2.19: q^{n+1} = q/2 + (q1 + dt L(q1))/2 */
        orc_rhs(c, q1, b, L);
        for (size_t k = 0; k < n; k++) q[k] = 0.5 * q[k] + 0.5 * (q1[k] + dt * L[k]);
    } else {
        /* eq 2.20: q2 = 3/4 q + 1/4 (q1 + dt L(q1)); q^{n+1} = 1/3 q + 2/3 (q2 + dt L(q2)) */
        orc_rhs(c, q1, b, L);
        for (size_t k = 0; k < n; k++) q2[k] = 0.75 * q[k] + 0.25 * (q1[k] + dt * L[k]);
        if (c->shadow_f32) round_to_float(q2, n);
        orc_rhs(c, q2, b, L);
        for (size_t k = 0; k < n; k++) q[k] = q[k] / 3.0 + 2.0 / 3.0 * (q2[k] + dt * L[k]);
    }
    if (c->shadow_f32) round_to_float(q, n);
    free(L); free(q1); free(q2);
    if (dt_used) *dt_used = dt;

    size_t plane = (size_t)c->nx * c->ny;
    for (size_t k = 0; k < plane; k++) {
        double s[4];
        for (int v = 0; v < nvar_of(c); v++) s[v] = q[v * plane + k];
        if (!admissible(c, s)) return -4;
    }
    return 0;
}

/* Run nsteps steps; writes the simulated time and the smallest/largest step. */
int orc_run(const orc_config *c, double *q, const double *b, int64_t nsteps, double *t_out,
            double *dt_min, double *dt_max)
{
    double t = 0.0, lo = INFINITY, hi = 0.0;
    int rc = 0;
    for (int64_t s = 0; s < nsteps; s++) {
        double dt = 0.0;
        rc = orc_step(c, q, b, &dt);
        t += dt;
        if (dt < lo) lo = dt;
        if (dt > hi) hi = dt;
        if (rc) break;
    }
    if (t_out) *t_out = t;
    if (dt_min) *dt_min = lo;
    if (dt_max) *dt_max = hi;
    return rc;
}

/* Conserved totals sum_i q_v dx dy for every variable, then the total energy
 * of eq 5.1, sum (g h^2/2 + h |u|^2 / 2) dx dy (SWE) or the kinetic energy
 * sum rho |u|^2/2 dx dy (Euler).  Fixed serial order. */
void orc_totals(const orc_config *c, const double *q, double *out)
{
    int nx = c->nx, ny = c->ny, nv = nvar_of(c);
    double dA = (c->lx / nx) * (c->ly / ny);
    size_t plane = (size_t)nx * ny;
    for (int v = 0; v <= nv; v++) out[v] = 0.0;
    for (size_t k = 0; k < plane; k++) {
        for (int v = 0; v < nv; v++) out[v] += q[v * plane + k] * dA;
        double h = q[k], mu = q[plane + k], mv = q[2 * plane + k];
        double kin = 0.5 * (mu * mu + mv * mv) / h;
        if (c->eqn == ORC_SWE) out[nv] += (0.5 * c->g * h * h + kin) * dA;
        else out[nv] += kin * dA;
    }
}
