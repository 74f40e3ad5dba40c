// Device-side physics of the finite-volume step: face-state reconstruction,
// normal-frame numerical fluxes and the hydrostatic bed treatment.
//
// Thesis "A Machine Learning accelerated geophysical fluid solver":
//   shallow-water flux, eq 2.3; Euler flux with the ideal-gas law, eq 2.4 and
//   section 4.2; MINMOD face states, eq 2.18; HLLE, eq 2.16; Rusanov, eq 2.12;
//   Roe, eq 2.13/2.14; axis-aligned rotation into the face frame, eq 2.24.
// The bed source follows the hydrostatic reconstruction of Audusse et al.
// (2004), the reading taken where the thesis leaves the discretisation open.
//
// The step is bound by vector-ALU issue, so the code is written branch-free:
// min/max/abs map to single instructions (v_min3/v_max3, |x| source
// modifiers), MINMOD is one v_med3_f32, guards are selects, and every face
// evaluates one reciprocal per side, one for the Roe weight and one for the
// HLLE denominator, plus three square roots.
#pragma once

#include <hip/hip_runtime.h>

namespace fvk {

enum { SWE = 0, EULER = 1 };
enum { HLLE = 0, RUSANOV = 1, ROE = 2 };
enum { MINMOD = 0, FIRST = 1 };

// ---------------------------------------------------------------- arithmetic
// Single precision uses the hardware reciprocal and square root (about 1 ulp);
// double precision keeps IEEE division and square root.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float tmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double tmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float tmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double tmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float tabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double tabs(double a) { return __builtin_fabs(a); }

// MINMOD(a, b): 0 unless a and b share a sign, else the one of smaller
// magnitude -- which is the median of (a, b, 0).
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b)
{
    return __builtin_fmax(__builtin_fmin(a, b), __builtin_fmin(__builtin_fmax(a, b), 0.0));
}

// 1/x for x > 0, else 0 (a dry state has zero velocity).
template <typename T> __device__ __forceinline__ T rcp_pos(T x) { return x > T(0) ? rcp(x) : T(0); }

// A positive power of two far below any wave speed or sqrt(h) of interest:
// the floor that keeps HLLE's denominator and the Roe weight positive.
template <typename T> __device__ __forceinline__ T tiny() { return T(0x1p-60f); }

template <typename T> struct Phys {
    T g;      // gravity
    T sqg;    // sqrt(g)
    T gamma;  // ratio of specific heats
    T h0;     // reference depth: the SWE pressure is carried as g (h^2 - h0^2) / 2
};

// ------------------------------------------------------------ shallow water
// Normal-frame state given by depth and velocities: (h, u normal, v tangential).
template <typename T> struct SweV { T h, u, v; };

// Numerical flux of two normal-frame shallow-water states.  The pressure
// g h^2/2 is carried relative to the constant g c/2, c = h0^2 rounded to the
// working precision: every flux below is affine in (F_L, F_R) with weights
// summing to one (and equal to F_L when both sides are dry), so the constant
// shifts all face fluxes equally and cancels in every cell's divergence,
// while h^2 - c, formed as one fused multiply-add, carries a rounding error
// that scales with |h^2 - h0^2| instead of h^2.
template <typename T, int FLUX>
__device__ __forceinline__ void swe_numflux(const SweV<T> &L, const SweV<T> &R, const Phys<T> &ph, T F[3])
{
    const T hg = T(0.5) * ph.g;
    const T c0 = ph.h0 * ph.h0;
    T ml = L.h * L.u, mr = R.h * R.u;
    T fl[3] = {ml, ml * L.u + hg * (L.h * L.h - c0), ml * L.v};
    T fr[3] = {mr, mr * R.u + hg * (R.h * R.h - c0), mr * R.v};
    T dq[3] = {R.h - L.h, mr - ml, R.h * R.v - L.h * L.v};
    T wl = fsqrt(L.h), wr = fsqrt(R.h);
    T cl = ph.sqg * wl, cr = ph.sqg * wr;
    if (FLUX == RUSANOV) {
        T a = tmax(tabs(L.u) + cl, tabs(R.u) + cr);
#pragma unroll
        for (int k = 0; k < 3; k++) F[k] = T(0.5) * (fl[k] + fr[k]) - T(0.5) * a * dq[k];
        return;
    }
    // Roe averages: sqrt(h)-weighted velocities (zero when both sides are
    // dry), c~ = sqrt(g (hL + hR) / 2)
    T iw = rcp(tmax(wl + wr, tiny<T>()));
    T ua = (wl * L.u + wr * R.u) * iw;
    T ca = fsqrt(hg * (L.h + R.h));
    if (FLUX == HLLE) {
        // sR is floored at a tiny power of two instead of 0.  The denominator
        // is then never zero: where it would be (both sides dry, sL = sR = 0)
        // the formula returns F_L exactly, which equals (F_L + F_R)/2 there;
        // elsewhere the floor moves the flux by a relative 2^-60 at most.
        // (sR F_L - sL F_R + sL sR dQ) / (sR - sL) = F_L + t (sR dQ - (F_R - F_L)),
        // t = sL / (sR - sL)
        T sL = tmin(tmin(L.u - cl, ua - ca), T(0));
        T sR = tmax(tmax(R.u + cr, ua + ca), tiny<T>());
        T t = sL * rcp(sR - sL);
#pragma unroll
        for (int k = 0; k < 3; k++) F[k] = fl[k] + t * (sR * dq[k] - (fr[k] - fl[k]));
        return;
    }
    // Roe: three waves u-c, u (shear), u+c
    T va = (wl * L.v + wr * R.v) * iw;
    T i2c = rcp_pos(T(2) * ca);
    T a1 = ((ua + ca) * dq[0] - dq[1]) * i2c;
    T a3 = (dq[1] - (ua - ca) * dq[0]) * i2c;
    T a2 = dq[2] - va * dq[0];
    T l1 = tabs(ua - ca) * a1, l2 = tabs(ua) * a2, l3 = tabs(ua + ca) * a3;
    F[0] = T(0.5) * (fl[0] + fr[0]) - T(0.5) * (l1 + l3);
    F[1] = T(0.5) * (fl[1] + fr[1]) - T(0.5) * (l1 * (ua - ca) + l3 * (ua + ca));
    F[2] = T(0.5) * (fl[2] + fr[2]) - T(0.5) * (l1 * va + l2 + l3 * va);
}

// ----------------------------------------------------------------- Euler
template <typename T> struct EulS { T r, m, t, E; };

template <typename T> __device__ __forceinline__ T eul_p(const EulS<T> &s, T gamma)
{
    return (gamma - T(1)) * (s.E - T(0.5) * (s.m * s.m + s.t * s.t) * rcp(s.r));
}

template <typename T, int FLUX>
__device__ __forceinline__ void eul_numflux(const EulS<T> &L, const EulS<T> &R, T gamma, T F[4])
{
    T irl = rcp(L.r), irr = rcp(R.r);
    T ul = L.m * irl, ur = R.m * irr;
    T vl = L.t * irl, vr = R.t * irr;
    T pl = (gamma - T(1)) * (L.E - T(0.5) * (L.m * ul + L.t * vl));
    T pr = (gamma - T(1)) * (R.E - T(0.5) * (R.m * ur + R.t * vr));
    T fl[4] = {L.m, L.m * ul + pl, L.t * ul, ul * (L.E + pl)};
    T fr[4] = {R.m, R.m * ur + pr, R.t * ur, ur * (R.E + pr)};
    T dq[4] = {R.r - L.r, R.m - L.m, R.t - L.t, R.E - L.E};
    T cl = fsqrt(gamma * pl * irl), cr = fsqrt(gamma * pr * irr);
    if (FLUX == RUSANOV) {
        T a = tmax(tabs(ul) + cl, tabs(ur) + cr);
#pragma unroll
        for (int k = 0; k < 4; k++) F[k] = T(0.5) * (fl[k] + fr[k]) - T(0.5) * a * dq[k];
        return;
    }
    T wl = fsqrt(L.r), wr = fsqrt(R.r);
    T iw = rcp(wl + wr);
    T ua = (wl * ul + wr * ur) * iw;
    T va = (wl * vl + wr * vr) * iw;
    T Ha = (wl * ((L.E + pl) * irl) + wr * ((R.E + pr) * irr)) * iw;
    T c2 = (gamma - T(1)) * (Ha - T(0.5) * (ua * ua + va * va));
    T ca = fsqrt(tmax(c2, T(0)));
    if (FLUX == HLLE) {
        T sL = tmin(tmin(ul - cl, ua - ca), T(0));
        T sR = tmax(tmax(ur + cr, ua + ca), T(0));
        T id = rcp(sR - sL), ss = sL * sR;  // sR - sL >= c~ > 0 for admissible states
#pragma unroll
        for (int k = 0; k < 4; k++) F[k] = (sR * fl[k] - sL * fr[k] + ss * dq[k]) * id;
        return;
    }
    // Roe: acoustic u-c, entropy u, shear u, acoustic u+c (normal frame)
    T gm1 = gamma - T(1);
    T a3 = dq[2] - va * dq[0];
    T d5 = dq[3] - a3 * va;
    T a2 = gm1 * rcp(ca * ca) * (dq[0] * (Ha - ua * ua) + ua * dq[1] - d5);
    T a1 = (dq[0] * (ua + ca) - dq[1] - ca * a2) * rcp(T(2) * ca);
    T a4 = dq[0] - (a1 + a2);
    T w1 = tabs(ua - ca) * a1, w2 = tabs(ua) * a2, w3 = tabs(ua) * a3, w4 = tabs(ua + ca) * a4;
    F[0] = T(0.5) * (fl[0] + fr[0]) - T(0.5) * (w1 + w2 + w4);
    F[1] = T(0.5) * (fl[1] + fr[1]) - T(0.5) * (w1 * (ua - ca) + w2 * ua + w4 * (ua + ca));
    F[2] = T(0.5) * (fl[2] + fr[2]) - T(0.5) * (w1 * va + w2 * va + w3 + w4 * va);
    F[3] = T(0.5) * (fl[3] + fr[3]) -
           T(0.5) * (w1 * (Ha - ua * ca) + w2 * T(0.5) * (ua * ua + va * va) + w3 * va + w4 * (Ha + ua * ca));
}

// --------------------------------------------------------- face states

// Face states on both sides of face i+1/2 from the four cells i-1, i, i+1, i+2
// along the face normal, for one scalar: MINMOD (eq 2.18, right state taken
// towards the face) or first order.
template <typename T, int RECON>
__device__ __forceinline__ void recon_pair(T m1, T c0, T c1, T p2, T &ql, T &qr)
{
    if (RECON == FIRST) {
        ql = c0;
        qr = c1;
    } else {
        ql = c0 + T(0.5) * minmod(c0 - m1, c1 - c0);
        qr = c1 - T(0.5) * minmod(c1 - c0, p2 - c1);
    }
}

template <typename T> __device__ __forceinline__ bool eul_admissible(T r, T m, T t, T E, T gamma)
{
    T p = (gamma - T(1)) * (E - T(0.5) * (m * m + t * t) * rcp(r));
    return r > T(0) && p > T(0);
}

// CFL rate (|u|+c)/dx + (|v|+c)/dy of a cell and whether the cell is
// admissible (finite, h > 0; or rho > 0 and p > 0).  A non-finite or
// non-positive depth, or a non-finite momentum or energy, makes the rate NaN
// or infinite, so one comparison of the rate covers finiteness; the
// comparison is false for NaN.  (A positive depth so small that the rate
// overflows is reported inadmissible too: it would stall Delta t at 0.)
template <typename T, int EQN>
__device__ __forceinline__ bool cell_rate_ok(const T *s, const Phys<T> &ph, T rdx, T rdy, T &rate)
{
    const T ir = rcp(s[0]);
    const T u = s[1] * ir, v = s[2] * ir;
    T c;
    bool pos = true;
    if (EQN == SWE) {
        c = ph.sqg * fsqrt(s[0]);
    } else {
        const T p = (ph.gamma - T(1)) * (s[3] - T(0.5) * (s[1] * u + s[2] * v));
        c = fsqrt(ph.gamma * p * ir);
        pos = s[0] > T(0) && p > T(0);
    }
    rate = (tabs(u) + c) * rdx + (tabs(v) + c) * rdy;
    return pos && rate < T(__builtin_inf());
}

// Full face computation.  Inputs: the four cells along the normal for each
// variable, in Cartesian order (v = 0..NV-1, plus the free surface eta = h + b
// as the last entry when BATHY).  Output: flux seen by the cell on the left
// (FlC, NV values, Cartesian order) and the normal-momentum flux seen by the
// cell on the right (frn) -- they differ only by the hydrostatic correction.
// With a bed, `sd` receives the two face states the centred bed source needs:
// {h, z} of the left state and {h, z} of the right state (z = eta - h), after
// the positivity fallback.
// AXIS 0: x face (normal momentum is variable 1), AXIS 1: y face (variable 2).
template <typename T, int EQN, bool BATHY, int FLUX, int RECON, int AXIS>
__device__ __forceinline__ void face_flux(const T (*st)[4], const Phys<T> &ph, T *FlC, T &frn, T *sd)
{
    constexpr int NV = EQN == SWE ? 3 : 4;
    constexpr int NR = NV + (BATHY ? 1 : 0);
    constexpr int NM = AXIS == 0 ? 1 : 2, TM = AXIS == 0 ? 2 : 1;
    T QL[NR], QR[NR];
#pragma unroll
    for (int v = 0; v < NR; v++) recon_pair<T, RECON>(st[v][0], st[v][1], st[v][2], st[v][3], QL[v], QR[v]);
    // Face states that are not admissible fall back to the cell average.  A
    // MINMOD (or first-order) face depth of positive cell averages is at
    // least half the cell's own depth, so for shallow water the fallback can
    // only act where a cell average is already non-positive, which the step
    // reports as a failure anyway: the check is kept for Euler only, where a
    // reconstructed pressure can turn negative.
    if (EQN == EULER) {
        const bool okl = eul_admissible(QL[0], QL[1], QL[2], QL[3], ph.gamma);
        const bool okr = eul_admissible(QR[0], QR[1], QR[2], QR[3], ph.gamma);
#pragma unroll
        for (int v = 0; v < NR; v++) {
            QL[v] = okl ? QL[v] : st[v][1];
            QR[v] = okr ? QR[v] : st[v][2];
        }
    }
    if (EQN == EULER) {
        EulS<T> L{QL[0], QL[NM], QL[TM], QL[3]}, R{QR[0], QR[NM], QR[TM], QR[3]};
        T F[4];
        eul_numflux<T, FLUX>(L, R, ph.gamma, F);
        FlC[0] = F[0];
        FlC[NM] = F[1];
        FlC[TM] = F[2];
        FlC[3] = F[3];
        frn = F[1];
        return;
    }
    T il = rcp(QL[0]), ir = rcp(QR[0]);  // face depths are positive here
    if (!BATHY) {
        SweV<T> L{QL[0], QL[NM] * il, QL[TM] * il}, R{QR[0], QR[NM] * ir, QR[TM] * ir};
        T F[3];
        swe_numflux<T, FLUX>(L, R, ph, F);
        FlC[0] = F[0];
        FlC[NM] = F[1];
        FlC[TM] = F[2];
        frn = F[1];
        return;
    }
    // hydrostatic reconstruction: bed at the face = max of the two sides,
    // depths re-evaluated against it, velocities kept
    T hl = QL[0], hr = QR[0];
    T el = QL[NV], er = QR[NV];
    T zf = tmax(el - hl, er - hr);
    T hls = tmax(T(0), el - zf), hrs = tmax(T(0), er - zf);
    SweV<T> L{hls, QL[NM] * il, QL[TM] * il}, R{hrs, QR[NM] * ir, QR[TM] * ir};
    T F[3];
    swe_numflux<T, FLUX>(L, R, ph, F);
    const T hg = T(0.5) * ph.g;
    FlC[0] = F[0];
    FlC[NM] = F[1] + hg * (hl - hls) * (hl + hls);
    FlC[TM] = F[2];
    frn = F[1] + hg * (hr - hrs) * (hr + hrs);
    sd[0] = hl;
    sd[1] = el - hl;
    sd[2] = hr;
    sd[3] = er - hr;
}

template <typename T, int EQN, bool BATHY, int FLUX, int RECON, int AXIS>
__device__ __forceinline__ void face_flux(const T (*st)[4], const Phys<T> &ph, T *FlC, T &frn)
{
    T sd[4];
    face_flux<T, EQN, BATHY, FLUX, RECON, AXIS>(st, ph, FlC, frn, sd);
}

// What one face hands to its two cells, for kernels that pass face results
// between lanes: TL to the cell on the left (below), TR to the cell on the
// right (above).  Entries 0..NV-1: the flux that cell sees (the two differ
// only in the normal momentum, by the hydrostatic correction); with a bed,
// entries NV and NV+1: depth and bed height of the face state on that side.
template <typename T, int EQN, bool BATHY> struct FaceSide {
    static constexpr int NV = EQN == SWE ? 3 : 4;
    static constexpr int N = NV + (BATHY ? 2 : 0);
};

template <typename T, int EQN, bool BATHY, int FLUX, int RECON, int AXIS>
__device__ __forceinline__ void face_eval(const T (*st)[4], const Phys<T> &ph, T *TL, T *TR)
{
    constexpr int NV = FaceSide<T, EQN, BATHY>::NV;
    constexpr int NM = AXIS == 0 ? 1 : 2;
    T F[NV], frn, sd[4];
    face_flux<T, EQN, BATHY, FLUX, RECON, AXIS>(st, ph, F, frn, sd);
#pragma unroll
    for (int v = 0; v < NV; v++) TL[v] = TR[v] = F[v];
    TR[NM] = frn;
    if (BATHY) {
        TL[NV] = sd[0];
        TL[NV + 1] = sd[1];
        TR[NV] = sd[2];
        TR[NV + 1] = sd[3];
    }
}

// Centred bed source of one cell along one axis (hydrostatic reconstruction),
// times the cell width: -g (h_{i-1/2+} + h_{i+1/2-})/2 (z_{i+1/2-} - z_{i-1/2+}),
// from the face state at the cell's low face (hL, zL) and at its high face
// (hR, zR); it is added to the cell's flux difference along that axis.
template <typename T> __device__ __forceinline__ T bed_term(T hL, T zL, T hR, T zR, T g)
{
    return -g * T(0.5) * (hL + hR) * (zR - zL);
}

}  // namespace fvk
