/*
 * Reference solver for the shallow-water equations on the sphere, double
 * precision, plain loops.
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle the GPU path is checked against; it
 * shares no source, header, table or helper with the HIP library.
 *
 * What it computes (thesis "A Machine Learning accelerated geophysical fluid
 * solver"):
 *   - the logically rectangular sphere grid of section 2.4: computational
 *     domain [-3,1] x [-1,1]; the square [-1,1]^2 is mapped to the unit disk
 *     sector by sector (a vertical segment x_c = d, |y_c| <= d goes to the
 *     arc of radius R(d) = 1 through (D, -D) and (D, D), D(d) = d / sqrt 2;
 *     the other sectors by symmetry) and lifted to the upper hemisphere by
 *     z = sqrt(1 - x^2 - y^2); the square [-3,-1] x [-1,1] is reflected onto
 *     the disk (x -> -2 - x) and lifted to the lower hemisphere;
 *   - the shallow-water equations in three-dimensional Cartesian form
 *     (section 3.3): state (h, hu, hv, hw), flux rows h u and m u^T + g h^2/2 I;
 *   - the discretisation steps listed in section 3.3: great-circle edge
 *     lengths and spherical cell areas; per face a unit normal n and tangent
 *     t in the tangent plane at the edge midpoint; the face states rotated
 *     into (n, t, r) (r: the edge midpoint's radial direction), the 1D
 *     Riemann problem solved along n (eq 2.24 for the rotation), the flux
 *     rotated back; the correction term of eq 3.1 (the cell's own momentum
 *     flux against the sum of its outward edge normals times lengths); the
 *     Coriolis source of eq 3.2; the momentum projected onto the tangent
 *     plane at each cell centre;
 *   - MINMOD face states along the computational index lines (eq 2.18),
 *     HLLE / Rusanov / Roe fluxes, Heun / three-stage / forward-Euler stages
 *     and the CFL time step, as in the planar oracle.
 *
 * Readings where the thesis is silent (listed in the design notes):
 *   - the grid has n cells per hemisphere side: 2n x n cells, dx = dy = 2/n
 *     (corner coordinates formed as exact ratios, coord_x / coord_y);
 *     cell corners are mapped, cell centres are the images of the
 *     computational cell centres;
 *   - neighbours across the domain boundary: x is periodic (x = -3 and x = 1
 *     are the same equator arc); across y = +-1 the neighbour of cell (i, j)
 *     is the cell of column 2n-1-i on the same side (the other hemisphere's
 *     cell sharing that equator arc), row mirrored; momenta are Cartesian, so
 *     no component changes sign;
 *   - the correction of eq 3.1 acts on the momentum equations only (the mass
 *     flux stays exactly conservative); with it a fluid at rest with uniform
 *     depth stays at rest;
 *   - the tangency forcing of eq 3.2 is applied as the projection of the
 *     momentum onto the tangent plane, after every Runge-Kutta stage;
 *   - the Coriolis term uses the unit sphere (a = 1): -2 omega z (x cross m);
 *   - CFL rate of a cell: (|m|/h + sqrt(g h)) times its perimeter over twice
 *     its area (the planar two-axis sum form on a square cell).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { SPH_HLLE = 0, SPH_RUSANOV = 1, SPH_ROE = 2 };
enum { SPH_MINMOD = 0, SPH_FIRST = 1 };

typedef struct {
    int32_t n;          /* cells per hemisphere side: grid 2n x n */
    int32_t flux;
    int32_t recon;
    int32_t rk_stages;  /* 1, 2 (Heun) or 3 */
    int32_t nthreads;
    int32_t pad;
    double cfl;
    double dt_fixed;    /* > 0: fixed step */
    double g;
    double omega;       /* rotation rate of the Coriolis term */
} sph_config;

/* ----------------------------------------------------------- grid mapping */

/* Disk mapping of a point of [-1,1]^2 (section 2.4, R = 1, D(d) = d/sqrt 2). */
static void disk_map(double xc, double yc, double *xp, double *yp)
{
    const int swap = fabs(yc) > fabs(xc);
    const double a = swap ? yc : xc, b = swap ? xc : yc;
    const double d = fabs(a);
    const double D = d / sqrt(2.0);
    const double across = b / sqrt(2.0);                   /* b D(d) / d */
    double along = D - sqrt(1.0 - D * D) + sqrt(1.0 - across * across);
    if (a < 0.0) along = -along;
    if (swap) {
        *xp = across;
        *yp = along;
    } else {
        *xp = along;
        *yp = across;
    }
}

/* Point of the unit sphere for computational (xc, yc) in [-3,1] x [-1,1].
 * Points of the square's boundary map to the equator: they are put there
 * exactly (z = 0, unit length), so that the two hemispheres' cells share
 * their equator corners bit for bit. */
static void sphere_point(double xc, double yc, double p[3])
{
    double xp, yp;
    const int north = xc >= -1.0;
    const double xd = north ? xc : -2.0 - xc;
    disk_map(xd, yc, &xp, &yp);
    if (fmax(fabs(xd), fabs(yc)) >= 1.0) {
        double r = sqrt(xp * xp + yp * yp);
        p[0] = xp / r;
        p[1] = yp / r;
        p[2] = 0.0;
        return;
    }
    double r2 = xp * xp + yp * yp;
    double z = sqrt(1.0 - r2);
    p[0] = xp;
    p[1] = yp;
    p[2] = north ? z : -z;
}

/* Computational coordinates of corner column I and corner row J (twice
 * the index: centres are odd), as one correctly rounded ratio of exact
 * integers, so that the squares' edges x = -3, -1, 1 and y = -1, 1 come out
 * exact for every n (-3 + I * (2/n) misses 1 by an ulp for some n). */
static double coord_x(int nn, int twice_I) { return (double)(twice_I - 3 * nn) / nn; }
static double coord_y(int nn, int twice_J) { return (double)(twice_J - nn) / nn; }

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double *a)
{
    double s = sqrt(dot3(a, a));
    a[0] /= s;
    a[1] /= s;
    a[2] /= s;
}

/* Great-circle distance of two unit vectors. */
static double arc(const double *p, const double *q)
{
    double c[3];
    cross3(p, q, c);
    return atan2(sqrt(dot3(c, c)), dot3(p, q));
}

/* Area of the spherical triangle p, q, r (solid angle, Van Oosterom and
 * Strackee). */
static double tri_area(const double *p, const double *q, const double *r)
{
    double c[3];
    cross3(q, r, c);
    double num = fabs(dot3(p, c));
    double den = 1.0 + dot3(p, q) + dot3(q, r) + dot3(r, p);
    return 2.0 * atan2(num, den);
}

/* Face geometry: unit normal n (from the low-index cell to the high-index
 * one), unit tangent t along the edge, radial r at the edge midpoint, length. */
typedef struct { double n[3], t[3], r[3], len; } face_geom;

/* x face at corner column I (between cells I-1 and I), row j: its edge runs
 * from corner (I, j) to corner (I, j+1). */
static void xface_geom(int nn, int I, int j, face_geom *f)
{
    double a[3], b[3];
    sphere_point(coord_x(nn, 2 * I), coord_y(nn, 2 * j), a);
    sphere_point(coord_x(nn, 2 * I), coord_y(nn, 2 * j + 2), b);
    for (int k = 0; k < 3; k++) {
        f->t[k] = b[k] - a[k];
        f->r[k] = a[k] + b[k];
    }
    normalize3(f->t);
    normalize3(f->r);
    cross3(f->t, f->r, f->n);  /* points towards increasing computational x */
    normalize3(f->n);
    f->len = arc(a, b);
}

/* y face at corner row J (between rows J-1 and J), column i: its edge runs
 * from corner (i, J) to corner (i+1, J). */
static void yface_geom(int nn, int i, int J, face_geom *f)
{
    double a[3], b[3];
    sphere_point(coord_x(nn, 2 * i), coord_y(nn, 2 * J), a);
    sphere_point(coord_x(nn, 2 * i + 2), coord_y(nn, 2 * J), b);
    for (int k = 0; k < 3; k++) {
        f->t[k] = b[k] - a[k];
        f->r[k] = a[k] + b[k];
    }
    normalize3(f->t);
    normalize3(f->r);
    cross3(f->r, f->t, f->n);  /* points towards increasing computational y */
    normalize3(f->n);
    f->len = arc(a, b);
}

/* Per-cell geometry. */
typedef struct { double c[3], area, perim, N[3]; } cell_geom;

static void cell_geometry(int nn, int i, int j, cell_geom *g)
{
    double p00[3], p10[3], p11[3], p01[3];
    sphere_point(coord_x(nn, 2 * i), coord_y(nn, 2 * j), p00);
    sphere_point(coord_x(nn, 2 * i + 2), coord_y(nn, 2 * j), p10);
    sphere_point(coord_x(nn, 2 * i + 2), coord_y(nn, 2 * j + 2), p11);
    sphere_point(coord_x(nn, 2 * i), coord_y(nn, 2 * j + 2), p01);
    sphere_point(coord_x(nn, 2 * i + 1), coord_y(nn, 2 * j + 1), g->c);
    g->area = tri_area(p00, p10, p11) + tri_area(p00, p11, p01);
    face_geom L, R, B, T;
    xface_geom(nn, i, j, &L);
    xface_geom(nn, i + 1, j, &R);
    yface_geom(nn, i, j, &B);
    yface_geom(nn, i, j + 1, &T);
    g->perim = L.len + R.len + B.len + T.len;
    /* sum of outward normals times edge lengths */
    for (int k = 0; k < 3; k++)
        g->N[k] = R.len * R.n[k] - L.len * L.n[k] + T.len * T.n[k] - B.len * B.n[k];
}

/* --------------------------------------------------------------- indexing */

/* Cell (i, j) of the infinite index plane -> interior cell, across the
 * periodic x boundary and the mirrored y boundaries. */
static void wrap(int nn, int i, int j, int *ii, int *jj)
{
    const int nx = 2 * nn, ny = nn;
    if (j >= ny) {
        j = 2 * ny - 1 - j;
        i = nx - 1 - i;
    } else if (j < 0) {
        j = -1 - j;
        i = nx - 1 - i;
    }
    i = ((i % nx) + nx) % nx;
    *ii = i;
    *jj = j;
}

static void cell_state(int nn, const double *q, int i, int j, double s[4])
{
    int ii, jj;
    wrap(nn, i, j, &ii, &jj);
    const size_t plane = (size_t)2 * nn * nn;
    for (int v = 0; v < 4; v++) s[v] = q[v * plane + (size_t)jj * 2 * nn + ii];
}

/* ------------------------------------------------------------------ fluxes */

/* 1D shallow water along the normal with two passively transported momenta:
 * state (h, m_n, m_t, m_r), flux (m_n, m_n u + g h^2/2, m_t u, m_r u). */
static void phys(const double *s, double g, double *f)
{
    double u = s[0] > 0.0 ? s[1] / s[0] : 0.0;
    f[0] = s[1];
    f[1] = s[1] * u + 0.5 * g * s[0] * s[0];
    f[2] = s[2] * u;
    f[3] = s[3] * u;
}

static void numflux(const sph_config *c, const double *L, const double *R, double *F)
{
    const double g = c->g;
    double fl[4], fr[4];
    phys(L, g, fl);
    phys(R, g, fr);
    double ul = L[1] / L[0], ur = R[1] / R[0];
    double cl = sqrt(g * L[0]), cr = sqrt(g * R[0]);
    if (c->flux == SPH_RUSANOV) {
        double a = fmax(fabs(ul) + cl, fabs(ur) + cr);
        for (int k = 0; k < 4; k++) F[k] = 0.5 * (fl[k] + fr[k]) - 0.5 * a * (R[k] - L[k]);
        return;
    }
    double wl = sqrt(L[0]), wr = sqrt(R[0]);
    double ua = (wl * ul + wr * ur) / (wl + wr);
    double ca = sqrt(0.5 * g * (L[0] + R[0]));
    if (c->flux == SPH_HLLE) {
        double sL = fmin(fmin(ul - cl, ua - ca), 0.0);
        double sR = fmax(fmax(ur + cr, ua + ca), 0.0);
        for (int k = 0; k < 4; k++) F[k] = (sR * fl[k] - sL * fr[k] + sL * sR * (R[k] - L[k])) / (sR - sL);
        return;
    }
    /* Roe: acoustic waves u -+ c, a shear wave for each transported momentum */
    double d[4];
    for (int k = 0; k < 4; k++) d[k] = R[k] - L[k];
    double va = (wl * L[2] / L[0] + wr * R[2] / R[0]) / (wl + wr);
    double wa = (wl * L[3] / L[0] + wr * R[3] / R[0]) / (wl + wr);
    double a1 = ((ua + ca) * d[0] - d[1]) / (2.0 * ca);
    double a3 = (d[1] - (ua - ca) * d[0]) / (2.0 * ca);
    double at = d[2] - va * d[0], ar = d[3] - wa * d[0];
    double l1 = fabs(ua - ca), l2 = fabs(ua), l3 = fabs(ua + ca);
    double r1[4] = {1.0, ua - ca, va, wa}, r3[4] = {1.0, ua + ca, va, wa};
    for (int k = 0; k < 4; k++) {
        double diss = l1 * a1 * r1[k] + l3 * a3 * r3[k];
        if (k == 2) diss += l2 * at;
        if (k == 3) diss += l2 * ar;
        F[k] = 0.5 * (fl[k] + fr[k]) - 0.5 * diss;
    }
}

static double minmod(double a, double b)
{
    if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0.0;
    return fabs(a) <= fabs(b) ? a : b;
}

/* Flux through the face between cell (i, j) and its neighbour along axis
 * (0: x, 1: y), in Cartesian components, directed along the face normal
 * (from the low-index cell to the high-index one); multiplied by nothing. */
static void face_flux(const sph_config *c, const double *q, int axis, int i, int j, const face_geom *fg, double *F)
{
    const int nn = c->n;
    const int di = axis == 0 ? 1 : 0, dj = axis == 0 ? 0 : 1;
    double m1[4], c0[4], c1[4], p2[4], QL[4], QR[4];
    cell_state(nn, q, i - di, j - dj, m1);
    cell_state(nn, q, i, j, c0);
    cell_state(nn, q, i + di, j + dj, c1);
    cell_state(nn, q, i + 2 * di, j + 2 * dj, p2);
    for (int v = 0; v < 4; v++) {
        if (c->recon == SPH_FIRST) {
            QL[v] = c0[v];
            QR[v] = c1[v];
        } else {
            QL[v] = c0[v] + 0.5 * minmod(c0[v] - m1[v], c1[v] - c0[v]);
            QR[v] = c1[v] - 0.5 * minmod(c1[v] - c0[v], p2[v] - c1[v]);
        }
    }
    if (!(QL[0] > 0.0)) for (int v = 0; v < 4; v++) QL[v] = c0[v];
    if (!(QR[0] > 0.0)) for (int v = 0; v < 4; v++) QR[v] = c1[v];
    /* rotate the momenta into (n, t, r) */
    double sl[4] = {QL[0], dot3(QL + 1, fg->n), dot3(QL + 1, fg->t), dot3(QL + 1, fg->r)};
    double sr[4] = {QR[0], dot3(QR + 1, fg->n), dot3(QR + 1, fg->t), dot3(QR + 1, fg->r)};
    double G[4];
    numflux(c, sl, sr, G);
    F[0] = G[0];
    for (int k = 0; k < 3; k++) F[1 + k] = G[1] * fg->n[k] + G[2] * fg->t[k] + G[3] * fg->r[k];
}

/* Momentum flux of a cell state against a vector N: m (u . N) + g h^2/2 N. */
static void cell_momentum_flux(const double *s, const double *N, double g, double *out)
{
    double un = dot3(s + 1, N) / s[0];
    for (int k = 0; k < 3; k++) out[k] = s[1 + k] * un + 0.5 * g * s[0] * s[0] * N[k];
}

/* ---------------------------------------------------------------- operator */

/* L(q): flux divergence over the four faces with the eq 3.1 correction on
 * the momenta, plus the Coriolis source of eq 3.2. */
void sph_rhs(const sph_config *c, const double *q, double *L)
{
    const int nn = c->n, nx = 2 * nn, ny = nn;
    const size_t plane = (size_t)nx * ny;
    int nth = c->nthreads > 0 ? c->nthreads : 1;
    (void)nth;
#pragma omp parallel for schedule(static) num_threads(nth)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            cell_geom cg;
            cell_geometry(nn, i, j, &cg);
            face_geom fl, fr, fb, ft;
            xface_geom(nn, i, j, &fl);
            xface_geom(nn, i + 1, j, &fr);
            yface_geom(nn, i, j, &fb);
            yface_geom(nn, i, j + 1, &ft);
            double Fl[4], Fr[4], Fb[4], Ft[4];
            face_flux(c, q, 0, i - 1, j, &fl, Fl);
            face_flux(c, q, 0, i, j, &fr, Fr);
            face_flux(c, q, 1, i, j - 1, &fb, Fb);
            face_flux(c, q, 1, i, j, &ft, Ft);
            double s[4];
            cell_state(nn, q, i, j, s);
            double corr[3];
            cell_momentum_flux(s, cg.N, c->g, corr);
            double cor[3];
            cross3(cg.c, s + 1, cor);
            for (int v = 0; v < 4; v++) {
                double out = fr.len * Fr[v] - fl.len * Fl[v] + ft.len * Ft[v] - fb.len * Fb[v];
                if (v > 0) out -= corr[v - 1];
                double Lv = -out / cg.area;
                if (v > 0) Lv += -2.0 * c->omega * cg.c[2] * cor[v - 1];
                L[v * plane + (size_t)j * nx + i] = Lv;
            }
        }
    }
}

/* Remove the momentum's component along each cell centre's radial direction. */
static void project(const sph_config *c, double *q)
{
    const int nn = c->n, nx = 2 * nn, ny = nn;
    const size_t plane = (size_t)nx * ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double x[3];
            sphere_point(coord_x(nn, 2 * i + 1), coord_y(nn, 2 * j + 1), x);
            size_t k = (size_t)j * nx + i;
            double m[3] = {q[plane + k], q[2 * plane + k], q[3 * plane + k]};
            double mr = dot3(m, x);
            for (int d = 0; d < 3; d++) q[(1 + d) * plane + k] = m[d] - mr * x[d];
        }
}

double sph_max_rate(const sph_config *c, const double *q)
{
    const int nn = c->n, nx = 2 * nn, ny = nn;
    const size_t plane = (size_t)nx * ny;
    double amax = 0.0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            cell_geom cg;
            cell_geometry(nn, i, j, &cg);
            size_t k = (size_t)j * nx + i;
            double h = q[k];
            double m2 = q[plane + k] * q[plane + k] + q[2 * plane + k] * q[2 * plane + k] + q[3 * plane + k] * q[3 * plane + k];
            double a = (sqrt(m2) / h + sqrt(c->g * h)) * cg.perim / (2.0 * cg.area);
            if (a > amax) amax = a;
        }
    return amax;
}

double sph_dt(const sph_config *c, const double *q)
{
    if (c->dt_fixed > 0.0) return c->dt_fixed;
    return c->cfl / sph_max_rate(c, q);
}

/* One full step in place; returns 0, or -4 if a depth became non-positive. */
int sph_step(const sph_config *c, double *q, double *dt_used)
{
    const size_t n = (size_t)4 * 2 * c->n * c->n;
    double dt = sph_dt(c, q);
    double *L = malloc(n * sizeof(double)), *q1 = malloc(n * sizeof(double)), *q2 = malloc(n * sizeof(double));
    if (!L || !q1 || !q2) {
        free(L);
        free(q1);
        free(q2);
        return -2;
    }
    sph_rhs(c, q, L);
    for (size_t k = 0; k < n; k++) q1[k] = q[k] + dt * L[k];
    project(c, q1);
    if (c->rk_stages == 1) {
        memcpy(q, q1, n * sizeof(double));
    } else if (c->rk_stages == 2) {
        sph_rhs(c, q1, L);
        for (size_t k = 0; k < n; k++) q[k] = 0.5 * q[k] + 0.5 * (q1[k] + dt * L[k]);
        project(c, q);
    } else {
        sph_rhs(c, q1, L);
        for (size_t k = 0; k < n; k++) q2[k] = 0.75 * q[k] + 0.25 * (q1[k] + dt * L[k]);
        project(c, q2);
        sph_rhs(c, q2, L);
        for (size_t k = 0; k < n; k++) q[k] = q[k] / 3.0 + 2.0 / 3.0 * (q2[k] + dt * L[k]);
        project(c, q);
    }
    free(L);
    free(q1);
    free(q2);
    if (dt_used) *dt_used = dt;
    const size_t plane = (size_t)2 * c->n * c->n;
    for (size_t k = 0; k < plane; k++)
        if (!(q[k] > 0.0)) return -4;
    return 0;
}

int sph_run(const sph_config *c, double *q, int64_t nsteps, double *t_out)
{
    double t = 0.0;
    int rc = 0;
    for (int64_t s = 0; s < nsteps; s++) {
        double dt = 0.0;
        rc = sph_step(c, q, &dt);
        t += dt;
        if (rc) break;
    }
    if (t_out) *t_out = t;
    return rc;
}

/* Geometry export: centres [3][ny][nx], areas [ny][nx], perimeters,
 * normal sums [3][ny][nx]. */
void sph_geometry(const sph_config *c, double *centres, double *areas, double *perims, double *nsum)
{
    const int nn = c->n, nx = 2 * nn, ny = nn;
    const size_t plane = (size_t)nx * ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            cell_geom cg;
            cell_geometry(nn, i, j, &cg);
            size_t k = (size_t)j * nx + i;
            for (int d = 0; d < 3; d++) {
                centres[d * plane + k] = cg.c[d];
                nsum[d * plane + k] = cg.N[d];
            }
            areas[k] = cg.area;
            perims[k] = cg.perim;
        }
}

/* Face geometry of x face (I, j) or y face (i, J): n[3], t[3], r[3], length. */
void sph_face(const sph_config *c, int axis, int i, int j, double *out)
{
    face_geom f;
    if (axis == 0) xface_geom(c->n, i, j, &f);
    else yface_geom(c->n, i, j, &f);
    for (int k = 0; k < 3; k++) {
        out[k] = f.n[k];
        out[3 + k] = f.t[k];
        out[6 + k] = f.r[k];
    }
    out[9] = f.len;
}

void sph_point(double xc, double yc, double *p) { sphere_point(xc, yc, p); }

/* Total mass sum h A and energy sum (g h^2/2 + |m|^2/(2h)) A. */
void sph_totals(const sph_config *c, const double *q, double *out)
{
    const int nn = c->n, nx = 2 * nn, ny = nn;
    const size_t plane = (size_t)nx * ny;
    out[0] = out[1] = 0.0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            cell_geom cg;
            cell_geometry(nn, i, j, &cg);
            size_t k = (size_t)j * nx + i;
            double h = q[k];
            double m2 = q[plane + k] * q[plane + k] + q[2 * plane + k] * q[2 * plane + k] + q[3 * plane + k] * q[3 * plane + k];
            out[0] += h * cg.area;
            out[1] += (0.5 * c->g * h * h + 0.5 * m2 / h) * cg.area;
        }
}
