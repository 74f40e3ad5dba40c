// Shallow water on the sphere (thesis sections 2.4 and 3.3), GPU kernels.
//
// Grid: the logically rectangular sphere grid of section 2.4, 2n x n cells
// on the computational rectangle [-3,1] x [-1,1]; the square [-1,1]^2 is
// mapped to the unit disk sector by sector (a vertical segment x_c = d goes
// to the arc of radius 1 through (d/sqrt2, -+d/sqrt2)) and lifted to the
// upper hemisphere, the square [-3,-1] x [-1,1] is reflected onto the disk
// and lifted to the lower hemisphere.  Neighbours: x periodic; across
// y = -+1 the cell of the mirrored column (2n-1-i) of the same row range.
//
// Equations (section 3.3): state (h, hu, hv, hw) with Cartesian momenta.
// Per face a unit normal n (towards increasing computational index), the
// edge tangent t and the edge midpoint's radial direction r; face states
// (MINMOD along the index lines, eq 2.18) are rotated into (n, t, r), the
// 1D Riemann problem is solved along n with t and r momenta transported,
// and the flux is rotated back (eq 2.24).  Each cell subtracts its own
// momentum flux against the sum of its outward edge normals times lengths
// (eq 3.1), adds the Coriolis force -2 omega z (x cross m) (eq 3.2, unit
// sphere), and after every stage its momentum is projected onto the tangent
// plane at its centre (the tangency forcing of eq 3.2).
//
// Kernels: geometry (once, in double precision); one launch per stage on
// tiles of cells, the state and a two-cell halo in LDS, each face of the tile
// evaluated once into LDS (fluxes times edge length), then the cell update
// (divergence, correction, source, Runge-Kutta combine, projection; on the
// last stage the CFL rate of the new state, reduced on the device as in the
// planar stage kernels).
#include <hip/hip_runtime.h>

#include "fv_device.hpp"
#include "fv_internal.hpp"
#include "sphere_internal.hpp"

namespace sph {

using fvk::Ctl;
using fvk::rate_slot;
using fvk::RATE_SUB;

// ------------------------------------------------------------- geometry
// Computed without contracting products and sums into FMAs (the rounding of
// the plain C formulas).  A corner that missed a square's edge by an ulp
// would be lifted to z = sqrt(1 - r^2) ~ 1e-8 instead of lying exactly on
// the equator, hence the exact-ratio coordinates below.

__device__ void disk(double xc, double yc, double &xp, double &yp)
{
#pragma clang fp contract(off)
    const bool swap = __builtin_fabs(yc) > __builtin_fabs(xc);
    const double a = swap ? yc : xc, b = swap ? xc : yc;
    const double D = __builtin_fabs(a) * 0.70710678118654752440;
    const double across = b * 0.70710678118654752440;
    double along = D - __builtin_sqrt(1.0 - D * D) + __builtin_sqrt(1.0 - across * across);
    along = a < 0.0 ? -along : along;
    xp = swap ? across : along;
    yp = swap ? along : across;
}

// Point of the unit sphere for computational coordinates; the squares'
// boundaries are put exactly on the equator.
__device__ void spoint(double xc, double yc, double *p)
{
#pragma clang fp contract(off)
    const bool north = xc >= -1.0;
    const double xd = north ? xc : -2.0 - xc;
    double xp, yp;
    disk(xd, yc, xp, yp);
    if (__builtin_fmax(__builtin_fabs(xd), __builtin_fabs(yc)) >= 1.0) {
        const double r = __builtin_sqrt(xp * xp + yp * yp);
        p[0] = xp / r;
        p[1] = yp / r;
        p[2] = 0.0;
        return;
    }
    const double z = __builtin_sqrt(1.0 - (xp * xp + yp * yp));
    p[0] = xp;
    p[1] = yp;
    p[2] = north ? z : -z;
}

__device__ __forceinline__ double dot3(const double *a, const double *b)
{
#pragma clang fp contract(off)
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ void cross3(const double *a, const double *b, double *c)
{
#pragma clang fp contract(off)
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ void unit3(double *a)
{
#pragma clang fp contract(off)
    const double s = 1.0 / __builtin_sqrt(dot3(a, a));
    a[0] *= s;
    a[1] *= s;
    a[2] *= s;
}

// Face from corner a to corner b; xface: the normal is t x r (towards
// increasing computational x), else r x t (towards increasing y).
__device__ void face_frame(const double *a, const double *b, bool xface, double *n, double *t, double *r, double &len)
{
#pragma clang fp contract(off)
    for (int k = 0; k < 3; k++) {
        t[k] = b[k] - a[k];
        r[k] = a[k] + b[k];
    }
    unit3(t);
    unit3(r);
    if (xface) cross3(t, r, n);
    else cross3(r, t, n);
    unit3(n);
    double c[3];
    cross3(a, b, c);
    len = atan2(__builtin_sqrt(dot3(c, c)), dot3(a, b));
}

// Solid angle of the spherical triangle p, q, r.
__device__ double tri(const double *p, const double *q, const double *r)
{
#pragma clang fp contract(off)
    double c[3];
    cross3(q, r, c);
    return 2.0 * atan2(__builtin_fabs(dot3(p, c)), 1.0 + dot3(p, q) + dot3(q, r) + dot3(r, p));
}

// Computational coordinate of twice a corner index (centres: odd), one
// rounding of a ratio of exact integers: the edges x = -3, -1, 1 and
// y = -1, 1 are exact for every n.
__device__ __forceinline__ double cx(int n, int twice_i) { return (double)(twice_i - 3 * n) / n; }
__device__ __forceinline__ double cy(int n, int twice_j) { return (double)(twice_j - n) / n; }

template <typename T>
__global__ __launch_bounds__(256) void geometry_kernel(Geometry<T> G, int n)
{
#pragma clang fp contract(off)
    const int nx = 2 * n, ny = n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int ncell = nx * ny, nyface = nx * (ny + 1);
    if (k < ncell) {
        const int j = k / nx, i = k - j * nx;
        double p00[3], p10[3], p11[3], p01[3], c[3];
        spoint(cx(n, 2 * i), cy(n, 2 * j), p00);
        spoint(cx(n, 2 * i + 2), cy(n, 2 * j), p10);
        spoint(cx(n, 2 * i + 2), cy(n, 2 * j + 2), p11);
        spoint(cx(n, 2 * i), cy(n, 2 * j + 2), p01);
        spoint(cx(n, 2 * i + 1), cy(n, 2 * j + 1), c);
        const double area = tri(p00, p10, p11) + tri(p00, p11, p01);
        double nL[3], tL[3], rL[3], lL, nR[3], tR[3], rR[3], lR, nB[3], tB[3], rB[3], lB, nT[3], tT[3], rT[3], lT;
        face_frame(p00, p01, true, nL, tL, rL, lL);
        face_frame(p10, p11, true, nR, tR, rR, lR);
        face_frame(p00, p10, false, nB, tB, rB, lB);
        face_frame(p01, p11, false, nT, tT, rT, lT);
        const size_t plane = (size_t)ncell;
        for (int d = 0; d < 3; d++) {
            G.cen[d * plane + k] = (T)c[d];
            G.nsum[d * plane + k] = (T)(lR * nR[d] - lL * nL[d] + lT * nT[d] - lB * nB[d]);
        }
        G.inv_area[k] = (T)(1.0 / area);
        G.rate_fac[k] = (T)((lL + lR + lB + lT) / (2.0 * area));
        G.area[k] = area;
        // the cell's low x face (between columns i-1 and i)
        for (int d = 0; d < 3; d++) {
            G.xf[d * plane + k] = (T)nL[d];
            G.xf[(3 + d) * plane + k] = (T)tL[d];
            G.xf[(6 + d) * plane + k] = (T)rL[d];
        }
        G.xf[9 * plane + k] = (T)lL;
    }
    if (k < nyface) {
        // y face row J (between rows J-1 and J), column i
        const int J = k / nx, i = k - J * nx;
        double a[3], b[3], nn[3], t[3], r[3], len;
        spoint(cx(n, 2 * i), cy(n, 2 * J), a);
        spoint(cx(n, 2 * i + 2), cy(n, 2 * J), b);
        face_frame(a, b, false, nn, t, r, len);
        const size_t fplane = (size_t)nyface;
        for (int d = 0; d < 3; d++) {
            G.yf[d * fplane + k] = (T)nn[d];
            G.yf[(3 + d) * fplane + k] = (T)t[d];
            G.yf[(6 + d) * fplane + k] = (T)r[d];
        }
        G.yf[9 * fplane + k] = (T)len;
    }
}

// ------------------------------------------------------------ face fluxes

// Interior cell of (i, j) across the periodic x and mirrored y boundaries.
__device__ __forceinline__ int cell_of(int i, int j, int nx, int ny)
{
    if (j >= ny) {
        j = 2 * ny - 1 - j;
        i = nx - 1 - i;
    } else if (j < 0) {
        j = -1 - j;
        i = nx - 1 - i;
    }
    i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
    return j * nx + i;
}

// Numerical flux along the normal of two face-frame states (h, m_n, m_t,
// m_r): shallow water with two transported momenta.
template <typename T, int FLUX>
__device__ __forceinline__ void numflux4(const T *L, const T *R, T g, T *F)
{
    using fvk::fsqrt;
    using fvk::rcp;
    using fvk::tabs;
    using fvk::tmax;
    using fvk::tmin;
    const T il = rcp(L[0]), ir = rcp(R[0]);
    const T ul = L[1] * il, ur = R[1] * ir;
    const T hg = T(0.5) * g;
    T fl[4] = {L[1], L[1] * ul + hg * L[0] * L[0], L[2] * ul, L[3] * ul};
    T fr[4] = {R[1], R[1] * ur + hg * R[0] * R[0], R[2] * ur, R[3] * ur};
    T dq[4] = {R[0] - L[0], R[1] - L[1], R[2] - L[2], R[3] - L[3]};
    const T wl = fsqrt(L[0]), wr = fsqrt(R[0]);
    const T sg = fsqrt(g);
    const T cl = sg * wl, cr = sg * wr;
    if (FLUX == fvk::RUSANOV) {
        const T a = tmax(tabs(ul) + cl, tabs(ur) + cr);
#pragma unroll
        for (int k = 0; k < 4; k++) F[k] = T(0.5) * (fl[k] + fr[k]) - T(0.5) * a * dq[k];
        return;
    }
    const T iw = rcp(wl + wr);
    const T ua = (wl * ul + wr * ur) * iw;
    const T ca = fsqrt(hg * (L[0] + R[0]));
    if (FLUX == fvk::HLLE) {
        const T sL = tmin(tmin(ul - cl, ua - ca), T(0));
        const T sR = tmax(tmax(ur + cr, ua + ca), T(0));
        const T id = rcp(sR - sL);
#pragma unroll
        for (int k = 0; k < 4; k++) F[k] = (sR * fl[k] - sL * fr[k] + sL * sR * dq[k]) * id;
        return;
    }
    const T va = (wl * L[2] * il + wr * R[2] * ir) * iw;
    const T wa = (wl * L[3] * il + wr * R[3] * ir) * iw;
    const T i2c = rcp(T(2) * ca);
    const T a1 = ((ua + ca) * dq[0] - dq[1]) * i2c;
    const T a3 = (dq[1] - (ua - ca) * dq[0]) * i2c;
    const T at = dq[2] - va * dq[0], ar = dq[3] - wa * dq[0];
    const T l1 = tabs(ua - ca) * a1, l2 = tabs(ua), l3 = tabs(ua + ca) * a3;
    F[0] = T(0.5) * (fl[0] + fr[0]) - T(0.5) * (l1 + l3);
    F[1] = T(0.5) * (fl[1] + fr[1]) - T(0.5) * (l1 * (ua - ca) + l3 * (ua + ca));
    F[2] = T(0.5) * (fl[2] + fr[2]) - T(0.5) * (l1 * va + l2 * at + l3 * va);
    F[3] = T(0.5) * (fl[3] + fr[3]) - T(0.5) * (l1 * wa + l2 * ar + l3 * wa);
}

// ------------------------------------------------------------ stage tiles

__device__ __forceinline__ unsigned long long dmax_bits(double v) { return (unsigned long long)__double_as_longlong(v); }

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fvk::tmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Flux of one face from the four stencil values c[v][0..3] along its index
// line (low-1, low, high, high+1) and its frame F9 (n, t, r, length at
// entry f of planes fp apart): MINMOD (or first-order) face states rotated
// into (n, t, r), the 1D numerical flux along n with the t and r momenta
// transported, rotated back and multiplied by the edge length.
template <typename T, int FLUX, int RECON>
__device__ __forceinline__ void face_flux(const T (*c)[4], const T *__restrict__ F9, size_t fp, int f, T g, T *out)
{
    T QL[4], QR[4];
#pragma unroll
    for (int v = 0; v < 4; v++) fvk::recon_pair<T, RECON>(c[v][0], c[v][1], c[v][2], c[v][3], QL[v], QR[v]);
    T nn[3], t[3], r[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        nn[d] = F9[d * fp + f];
        t[d] = F9[(3 + d) * fp + f];
        r[d] = F9[(6 + d) * fp + f];
    }
    const T len = F9[9 * fp + f];
    T sl[4] = {QL[0], QL[1] * nn[0] + QL[2] * nn[1] + QL[3] * nn[2], QL[1] * t[0] + QL[2] * t[1] + QL[3] * t[2],
               QL[1] * r[0] + QL[2] * r[1] + QL[3] * r[2]};
    T sr[4] = {QR[0], QR[1] * nn[0] + QR[2] * nn[1] + QR[3] * nn[2], QR[1] * t[0] + QR[2] * t[1] + QR[3] * t[2],
               QR[1] * r[0] + QR[2] * r[1] + QR[3] * r[2]};
    T F[4];
    numflux4<T, FLUX>(sl, sr, g, F);
    out[0] = len * F[0];
#pragma unroll
    for (int d = 0; d < 3; d++) out[1 + d] = len * (F[1] * nn[d] + F[2] * t[d] + F[3] * r[d]);
}

// One Runge-Kutta stage, out = a0 q0 + a1 (qs + dt L(qs)) with the momentum
// then projected onto the tangent plane, on an STX x STY tile of cells per
// workgroup: the state with a two-cell halo (periodic in x, mirrored across
// y = -+1, as cell_of) staged in LDS; every face of the tile evaluated once
// into LDS (a face on a tile edge is evaluated by both tiles: the same
// value); then one cell per thread: flux divergence, eq 3.1 correction
// against the cell's summed edge normals, Coriolis (eq 3.2), the combine and
// the projection.  Face fluxes never reach HBM.  The last stage reduces the
// CFL rate of out into slot rate_out, clears slot rate_clear, flags
// inadmissible cells and advances time and step count.
constexpr int STX = 32, STY = 8, SNT = STX * STY;

// Workgroups are handed to the eight XCDs in turn: for a grid that is a
// multiple of 8, XCD k gets the contiguous k-th eighth of the tiles, so that
// neighbouring tiles, which re-read each other's halo cells, share one L2.
__device__ __forceinline__ int xcd_tile(int w, int grid)
{
    return (grid & 7) ? w : (w & 7) * (grid >> 3) + (w >> 3);
}

template <typename T, int FLUX, int RECON>
__global__ __launch_bounds__(SNT) void tile_kernel(CellArgs<T> a, int tiles_x)
{
    constexpr int HX = STX + 4, HY = STY + 4;
    __shared__ T s_q[4][HY][HX];
    __shared__ T s_fx[4][STY][STX + 1];
    __shared__ T s_fy[4][STY + 1][STX];
    __shared__ double s_dt;
    const int nx = 2 * a.n, ny = a.n;
    const int ncell = nx * ny, nyface = nx * (ny + 1);
    const size_t plane = (size_t)ncell;
    const int tid = threadIdx.x;
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int ty = w / tiles_x, tx = w - ty * tiles_x;
    const int x0 = tx * STX, y0 = ty * STY;
    const int tw = nx - x0 < STX ? nx - x0 : STX, th = ny - y0 < STY ? ny - y0 : STY;  // cells of this tile
    const bool frozen = a.ctl->bad != 0;
    // the state on the tile and its two-cell ring: x in [x0 - 2, x0 + tw + 2),
    // y in [y0 - 2, y0 + th + 2), each within one period or mirror of the grid
    for (int e = tid; e < HY * HX; e += SNT) {
        const int ly = e / HX, lx = e - ly * HX;
        if (lx >= tw + 4 || ly >= th + 4) continue;
        const int k = cell_of(x0 - 2 + lx, y0 - 2 + ly, nx, ny);
#pragma unroll
        for (int v = 0; v < 4; v++) s_q[v][ly][lx] = a.qs[v * plane + k];
    }
    if (tid < 64) {
        const int lane = tid;
        double m = 0.0;
        if (!(a.dt_fixed > 0.0)) m = __longlong_as_double((long long)*rate_slot(a.rates, a.rate_in, lane));
        m = wave_max(m);
        if (lane == 0) s_dt = a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl / m;
    }
    __syncthreads();
    const T g = a.g;
    // x faces (fi, fj): between cells x0 + fi - 1 and x0 + fi of row y0 + fj;
    // the x-face arrays index it by cell (x0 + fi) mod nx
    for (int f = tid; f < (STX + 1) * STY; f += SNT) {
        const int fj = f / (STX + 1), fi = f - fj * (STX + 1);
        if (fi > tw || fj >= th) continue;
        const int i = x0 + fi < nx ? x0 + fi : x0 + fi - nx;
        T c[4][4];
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int s = 0; s < 4; s++) c[v][s] = s_q[v][fj + 2][fi + s];
        T o[4];
        face_flux<T, FLUX, RECON>(c, a.G.xf, plane, (y0 + fj) * nx + i, g, o);
#pragma unroll
        for (int v = 0; v < 4; v++) s_fx[v][fj][fi] = o[v];
    }
    // y faces (fi, fj): row y0 + fj of the y-face arrays (between cell rows
    // y0 + fj - 1 and y0 + fj), column x0 + fi
    for (int f = tid; f < (STY + 1) * STX; f += SNT) {
        const int fj = f / STX, fi = f - fj * STX;
        if (fi >= tw || fj > th) continue;
        T c[4][4];
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int s = 0; s < 4; s++) c[v][s] = s_q[v][fj + s][fi + 2];
        T o[4];
        face_flux<T, FLUX, RECON>(c, a.G.yf, (size_t)nyface, (y0 + fj) * nx + x0 + fi, g, o);
#pragma unroll
        for (int v = 0; v < 4; v++) s_fy[v][fj][fi] = o[v];
    }
    __syncthreads();
    const T dt = (T)s_dt;
    const int cj = tid / STX, ci = tid - cj * STX;
    T rate = T(0);
    bool bad = false;
    if (ci < tw && cj < th && !frozen) {
        const int k = (y0 + cj) * nx + x0 + ci;
        T s[4];
#pragma unroll
        for (int v = 0; v < 4; v++) s[v] = s_q[v][cj + 2][ci + 2];
        const T ih = fvk::rcp(s[0]);
        const T N[3] = {a.G.nsum[k], a.G.nsum[plane + k], a.G.nsum[2 * plane + k]};
        const T x[3] = {a.G.cen[k], a.G.cen[plane + k], a.G.cen[2 * plane + k]};
        const T un = (s[1] * N[0] + s[2] * N[1] + s[3] * N[2]) * ih;
        const T pres = T(0.5) * a.g * s[0] * s[0];
        const T ia = a.G.inv_area[k];
        T o[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            T div = (s_fx[v][cj][ci + 1] - s_fx[v][cj][ci]) + (s_fy[v][cj + 1][ci] - s_fy[v][cj][ci]);
            if (v > 0) div = div - (s[v] * un + pres * N[v - 1]);
            o[v] = -div * ia;
        }
        // Coriolis: -2 omega z (x cross m)
        const T c2 = T(-2) * a.omega * x[2];
        o[1] += c2 * (x[1] * s[3] - x[2] * s[2]);
        o[2] += c2 * (x[2] * s[1] - x[0] * s[3]);
        o[3] += c2 * (x[0] * s[2] - x[1] * s[1]);
#pragma unroll
        for (int v = 0; v < 4; v++) {
            T r = a.a1 * (s[v] + dt * o[v]);
            if (a.a0 != T(0)) r = a.a0 * a.q0[v * plane + k] + r;
            o[v] = r;
        }
        const T mr = o[1] * x[0] + o[2] * x[1] + o[3] * x[2];
#pragma unroll
        for (int d = 0; d < 3; d++) o[1 + d] = o[1 + d] - mr * x[d];
#pragma unroll
        for (int v = 0; v < 4; v++) a.out[v * plane + k] = o[v];
        if (a.last) {
            const T speed = fvk::fsqrt(o[1] * o[1] + o[2] * o[2] + o[3] * o[3]) * fvk::rcp(o[0]);
            rate = (speed + fvk::fsqrt(a.g * o[0])) * a.G.rate_fac[k];
            bad = !(o[0] > T(0)) || !(rate < T(__builtin_inf()));
            if (bad) rate = T(0);
        }
    }
    if (!a.last || frozen) return;
    if (bad) atomicExch(&a.ctl->bad, 1);
    if (a.rate_out >= 0) {
        const T m = wave_max(rate);
        if ((tid & 63) == 0)
            atomicMax(rate_slot(a.rates, a.rate_out, (blockIdx.x * 4 + (tid >> 6)) & (RATE_SUB - 1)),
                      dmax_bits((double)m));
    }
    if (blockIdx.x == 0) {
        if (tid == 0) {
            a.ctl->t += s_dt;
            a.ctl->step += 1;
        }
        if (a.rate_clear >= 0 && tid < RATE_SUB) *rate_slot(a.rates, a.rate_clear, tid) = 0ull;
    }
}

// CFL rate of a state into slot `slot` (initialisation) and admissibility.
template <typename T>
__global__ __launch_bounds__(256) void rate_kernel(const T *q, Geometry<T> G, int n, T g, Ctl *ctl,
                                                   unsigned long long *rates, int slot)
{
    const int ncell = 2 * n * n;
    const size_t plane = (size_t)ncell;
    const int k = blockIdx.x * 256 + threadIdx.x;
    T rate = T(0);
    bool bad = false;
    if (k < ncell) {
        const T h = q[k], m1 = q[plane + k], m2 = q[2 * plane + k], m3 = q[3 * plane + k];
        rate = (fvk::fsqrt(m1 * m1 + m2 * m2 + m3 * m3) * fvk::rcp(h) + fvk::fsqrt(g * h)) * G.rate_fac[k];
        bad = !(h > T(0)) || !(rate < T(__builtin_inf()));
        if (bad) rate = T(0);
    }
    if (bad) atomicExch(&ctl->bad, 1);
    const T m = wave_max(rate);
    if ((threadIdx.x & 63) == 0)
        atomicMax(rate_slot(rates, slot, (blockIdx.x * 4 + (threadIdx.x >> 6)) & (RATE_SUB - 1)), dmax_bits((double)m));
}

// Totals: per-block partial sums of h A and (g h^2/2 + |m|^2/(2h)) A in a
// fixed order, then one block adds the partials in index order.
template <typename T>
__global__ __launch_bounds__(256) void totals_kernel(const T *q, const double *area, int n, double g, double *partials)
{
    __shared__ double s[2][256];
    const int ncell = 2 * n * n;
    const size_t plane = (size_t)ncell;
    double acc[2] = {0.0, 0.0};
    for (int k = blockIdx.x * 256 + threadIdx.x; k < ncell; k += gridDim.x * 256) {
        const double h = (double)q[k], m1 = (double)q[plane + k], m2 = (double)q[2 * plane + k],
                     m3 = (double)q[3 * plane + k];
        acc[0] += h * area[k];
        acc[1] += (0.5 * g * h * h + 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / h) * area[k];
    }
    s[0][threadIdx.x] = acc[0];
    s[1][threadIdx.x] = acc[1];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0][0];
        partials[2 * blockIdx.x + 1] = s[1][0];
    }
}

__global__ void totals_final_kernel(const double *partials, int nblocks, double *out)
{
    if (threadIdx.x < 2) {
        double acc = 0.0;
        for (int b = 0; b < nblocks; b++) acc += partials[2 * b + threadIdx.x];
        out[threadIdx.x] = acc;
    }
}

// ------------------------------------------------------------- launchers

template <typename T> hipError_t geometry(const Geometry<T> &G, int n, hipStream_t st)
{
    const int nfaces = 2 * n * (n + 1);
    hipLaunchKernelGGL((geometry_kernel<T>), dim3((nfaces + 255) / 256), dim3(256), 0, st, G, n);
    return hipGetLastError();
}

template <typename T> hipError_t stage(int flux, int recon, const CellArgs<T> &a, hipStream_t st)
{
    const int nx = 2 * a.n, ny = a.n;
    const int tiles_x = (nx + STX - 1) / STX, tiles = tiles_x * ((ny + STY - 1) / STY);
    const dim3 grid(tiles), blk(SNT);
#define SPH_TILE(FL, RC) hipLaunchKernelGGL((tile_kernel<T, FL, RC>), grid, blk, 0, st, a, tiles_x)
    if (recon == fvk::FIRST) {
        if (flux == fvk::RUSANOV) SPH_TILE(fvk::RUSANOV, fvk::FIRST);
        else if (flux == fvk::ROE) SPH_TILE(fvk::ROE, fvk::FIRST);
        else SPH_TILE(fvk::HLLE, fvk::FIRST);
    } else {
        if (flux == fvk::RUSANOV) SPH_TILE(fvk::RUSANOV, fvk::MINMOD);
        else if (flux == fvk::ROE) SPH_TILE(fvk::ROE, fvk::MINMOD);
        else SPH_TILE(fvk::HLLE, fvk::MINMOD);
    }
#undef SPH_TILE
    return hipGetLastError();
}

template <typename T>
hipError_t rate(const T *q, const Geometry<T> &G, int n, double g, Ctl *ctl, unsigned long long *rates, int slot,
                hipStream_t st)
{
    const int ncell = 2 * n * n;
    hipLaunchKernelGGL((rate_kernel<T>), dim3((ncell + 255) / 256), dim3(256), 0, st, q, G, n, (T)g, ctl, rates, slot);
    return hipGetLastError();
}

template <typename T>
hipError_t totals(const T *q, const double *area, int n, double g, double *partials, int max_blocks, double *out,
                  hipStream_t st)
{
    const int ncell = 2 * n * n;
    int blocks = (ncell + 255) / 256;
    if (blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL((totals_kernel<T>), dim3(blocks), dim3(256), 0, st, q, area, n, g, partials);
    hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(64), 0, st, partials, blocks, out);
    return hipGetLastError();
}

#define SPH_INST(T)                                                                                                   \
    template hipError_t geometry<T>(const Geometry<T> &, int, hipStream_t);                                        \
    template hipError_t stage<T>(int, int, const CellArgs<T> &, hipStream_t);                                      \
    template hipError_t rate<T>(const T *, const Geometry<T> &, int, double, Ctl *, unsigned long long *, int,      \
                                hipStream_t);                                                                      \
    template hipError_t totals<T>(const T *, const double *, int, double, double *, int, double *, hipStream_t);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
