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
// Kernels: geometry (once, in double precision), face fluxes (one thread
// per face, each face once per stage, fluxes times edge length to a buffer),
// cell update (divergence, correction, source, Runge-Kutta combine,
// projection; on the last stage the CFL rate of the new state, reduced on
// the device as in the planar stage kernels).
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

// One thread per face: x faces k < nx*ny (the low face of cell k), then y
// faces (nx*(ny+1), row J between rows J-1 and J).  Writes the flux times the
// edge length, Cartesian, along the face's normal.
template <typename T, int FLUX, int RECON>
__global__ __launch_bounds__(256) void face_kernel(const T *__restrict__ q, Geometry<T> G, T *__restrict__ fx,
                                                   T *__restrict__ fy, int n, T g)
{
    const int nx = 2 * n, ny = n;
    const int ncell = nx * ny, nyface = nx * (ny + 1);
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= ncell + nyface) return;
    const bool xface = k < ncell;
    const int f = xface ? k : k - ncell;
    const int j = f / nx, i = f - j * nx;
    // stencil cells along the normal index line: low-1, low, high, high+1
    int idx[4];
    if (xface) {
#pragma unroll
        for (int s = 0; s < 4; s++) idx[s] = cell_of(i - 2 + s, j, nx, ny);
    } else {
#pragma unroll
        for (int s = 0; s < 4; s++) idx[s] = cell_of(i, j - 2 + s, nx, ny);
    }
    const size_t plane = (size_t)ncell;
    T QL[4], QR[4];
#pragma unroll
    for (int v = 0; v < 4; v++) {
        T c[4];
#pragma unroll
        for (int s = 0; s < 4; s++) c[s] = q[v * plane + idx[s]];
        fvk::recon_pair<T, RECON>(c[0], c[1], c[2], c[3], QL[v], QR[v]);
    }
    const T *F9 = xface ? G.xf : G.yf;
    const size_t fp = xface ? plane : (size_t)nyface;
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
    T *out = xface ? fx : fy;
    out[f] = len * F[0];
#pragma unroll
    for (int d = 0; d < 3; d++) out[(1 + d) * fp + f] = len * (F[1] * nn[d] + F[2] * t[d] + F[3] * r[d]);
}

// ------------------------------------------------------------ cell update

__device__ __forceinline__ unsigned long long dmax_bits(double v) { return (unsigned long long)__double_as_longlong(v); }

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fvk::tmax(v, __shfl_xor(v, off, 64));
    return v;
}

// out = a0 q0 + a1 (qs + dt L(qs)) with the momentum then projected onto the
// tangent plane; the last stage reduces the CFL rate of out into slot
// rate_out, clears slot rate_clear, flags inadmissible cells and advances
// time and step count.
template <typename T>
__global__ __launch_bounds__(256) void cell_kernel(CellArgs<T> a)
{
    __shared__ double s_dt;
    const int nx = 2 * a.n, ny = a.n;
    const int ncell = nx * ny, nyface = nx * (ny + 1);
    const size_t plane = (size_t)ncell;
    const bool frozen = a.ctl->bad != 0;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        double m = 0.0;
        if (!(a.dt_fixed > 0.0)) m = __longlong_as_double((long long)*rate_slot(a.rates, a.rate_in, lane));
        m = wave_max(m);
        if (lane == 0) s_dt = a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl / m;
    }
    __syncthreads();
    const T dt = (T)s_dt;
    const int k = blockIdx.x * 256 + threadIdx.x;
    T rate = T(0);
    bool bad = false;
    if (k < ncell && !frozen) {
        const int j = k / nx, i = k - j * nx;
        const int kr = j * nx + (i + 1 == nx ? 0 : i + 1);  // the high x face is the low face of the right cell
        const int fb = j * nx + i, ft = (j + 1) * nx + i;
        T s[4];
#pragma unroll
        for (int v = 0; v < 4; v++) s[v] = a.qs[v * plane + k];
        const T ih = fvk::rcp(s[0]);
        const T N[3] = {a.G.nsum[k], a.G.nsum[plane + k], a.G.nsum[2 * plane + k]};
        const T x[3] = {a.G.cen[k], a.G.cen[plane + k], a.G.cen[2 * plane + k]};
        const T un = (s[1] * N[0] + s[2] * N[1] + s[3] * N[2]) * ih;
        const T pres = T(0.5) * a.g * s[0] * s[0];
        const T ia = a.G.inv_area[k];
        T o[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            T div = (a.fx[v * plane + kr] - a.fx[v * plane + k]) + (a.fy[v * (size_t)nyface + ft] - a.fy[v * (size_t)nyface + fb]);
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
        if ((threadIdx.x & 63) == 0)
            atomicMax(rate_slot(a.rates, a.rate_out, (blockIdx.x * 4 + (threadIdx.x >> 6)) & (RATE_SUB - 1)),
                      dmax_bits((double)m));
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            a.ctl->t += s_dt;
            a.ctl->step += 1;
        }
        if (a.rate_clear >= 0 && threadIdx.x < RATE_SUB) *rate_slot(a.rates, a.rate_clear, threadIdx.x) = 0ull;
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

template <typename T>
hipError_t faces(int flux, int recon, const T *q, const Geometry<T> &G, T *fx, T *fy, int n, double g, hipStream_t st)
{
    const int total = 2 * n * n + 2 * n * (n + 1);
    const dim3 grid((total + 255) / 256), blk(256);
    const T gg = (T)g;
#define SPH_FACE(FL, RC) hipLaunchKernelGGL((face_kernel<T, FL, RC>), grid, blk, 0, st, q, G, fx, fy, n, gg)
    if (recon == fvk::FIRST) {
        if (flux == fvk::RUSANOV) SPH_FACE(fvk::RUSANOV, fvk::FIRST);
        else if (flux == fvk::ROE) SPH_FACE(fvk::ROE, fvk::FIRST);
        else SPH_FACE(fvk::HLLE, fvk::FIRST);
    } else {
        if (flux == fvk::RUSANOV) SPH_FACE(fvk::RUSANOV, fvk::MINMOD);
        else if (flux == fvk::ROE) SPH_FACE(fvk::ROE, fvk::MINMOD);
        else SPH_FACE(fvk::HLLE, fvk::MINMOD);
    }
#undef SPH_FACE
    return hipGetLastError();
}

template <typename T> hipError_t cells(const CellArgs<T> &a, hipStream_t st)
{
    const int ncell = 2 * a.n * a.n;
    hipLaunchKernelGGL((cell_kernel<T>), dim3((ncell + 255) / 256), dim3(256), 0, st, a);
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
    template hipError_t faces<T>(int, int, const T *, const Geometry<T> &, T *, T *, int, double, hipStream_t);      \
    template hipError_t cells<T>(const CellArgs<T> &, hipStream_t);                                                 \
    template hipError_t rate<T>(const T *, const Geometry<T> &, int, double, Ctl *, unsigned long long *, int,      \
                                hipStream_t);                                                                      \
    template hipError_t totals<T>(const T *, const double *, int, double, double *, int, double *, hipStream_t);
SPH_INST(float)
SPH_INST(double)
#undef SPH_INST

}  // namespace sph
