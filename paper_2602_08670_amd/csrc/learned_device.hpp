// Face states and fluxes of the learned reconstruction (thesis section
// 2.5.3, fourth approach), shared by the learned-stage kernels and the
// network pass that runs a learned stage in the same workgroup.
#pragma once

#include "cnn_internal.hpp"
#include "fv_device.hpp"

namespace cnn {

using fvk::Phys;
using fvk::SweV;

__device__ __forceinline__ int pwrap(int i, int n) { return ((i % n) + n) % n; }

// Face states of one face from the six stencil values st[v][0..5] (cells
// i-2..i+3 along the normal).  MODE 0: learned with fallback; MODE 1: MINMOD.
// AL: zc already holds alpha = base + P z (projected by the network pass).
template <int MODE, bool AL = false>
__device__ __forceinline__ int face_states(const float (*st)[6], const float *zc, const Proj &pr, float *QL,
                                           float *QR)
{
    float ML[3], MR[3];
#pragma unroll
    for (int v = 0; v < 3; v++) fvk::recon_pair<float, fvk::MINMOD>(st[v][1], st[v][2], st[v][3], st[v][4], ML[v], MR[v]);
    bool okl = ML[0] > 0.0f, okr = MR[0] > 0.0f;
#pragma unroll
    for (int v = 0; v < 3; v++) {
        ML[v] = okl ? ML[v] : st[v][2];
        MR[v] = okr ? MR[v] : st[v][3];
    }
    if (MODE == 1) {
#pragma unroll
        for (int v = 0; v < 3; v++) {
            QL[v] = ML[v];
            QR[v] = MR[v];
        }
        return 0;
    }
#pragma unroll
    for (int s = 0; s < 2; s++) {
#pragma unroll
        for (int v = 0; v < 3; v++) {
            const float *zz = zc + (s * 3 + v) * 6;
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < 6; k++) {
                float al;
                if (AL) {
                    al = zz[k];
                } else {
                    al = pr.base[s * 6 + k];
#pragma unroll
                    for (int j = 0; j < 6; j++) al += pr.P[k * 6 + j] * zz[j];
                }
                acc += al * st[v][k];
            }
            (s == 0 ? QL : QR)[v] = acc;
        }
    }
    bool ll = QL[0] > 0.0f, lr = QR[0] > 0.0f;
#pragma unroll
    for (int v = 0; v < 3; v++) {
        QL[v] = ll ? QL[v] : ML[v];
        QR[v] = lr ? QR[v] : MR[v];
    }
    return (ll ? 0 : 1) + (lr ? 0 : 1);
}

// Direct face states (thesis section 2.5.3, third approach; section 5.3):
// the network's output is split into a depth part and a momentum part, and
// the depth part ends in a Softplus so every reconstructed depth is positive.
// The outputs are in the input's normalised units (de-normalised by
// 1 / inv_std): a face state's depth is its cell's depth times
// softplus(z / inv_std + c), with c = ln(e - 1) so that softplus(c) = 1 (a
// zero head is the first-order scheme); its momenta are the cell's plus
// z / inv_std.
constexpr float kSoftplusShift = 0.541324854612918f;  // ln(e - 1)

// ln(1 + e^x) without overflow or loss of the small values.
__device__ __forceinline__ float softplusf(float x)
{
    return __builtin_fmaxf(x, 0.0f) + log1pf(expf(-__builtin_fabsf(x)));
}

// Face states of one face in the direct scheme: the owner cell's high-side
// state and the neighbour's low-side state (zo: the owner's three outputs for
// its right or top side, zn: the neighbour's for its left or bottom side;
// sig = 1 / inv_std).  A side whose depth is not positive (the Softplus
// underflowed) takes its MINMOD state (counted).
__device__ __forceinline__ int face_states_direct(const float (*st)[6], const float *zo, const float *zn,
                                                  const float *sig, float *QL, float *QR)
{
    float ML[3], MR[3];
#pragma unroll
    for (int v = 0; v < 3; v++) fvk::recon_pair<float, fvk::MINMOD>(st[v][1], st[v][2], st[v][3], st[v][4], ML[v], MR[v]);
    bool okl = ML[0] > 0.0f, okr = MR[0] > 0.0f;
#pragma unroll
    for (int v = 0; v < 3; v++) {
        ML[v] = okl ? ML[v] : st[v][2];
        MR[v] = okr ? MR[v] : st[v][3];
    }
    QL[0] = st[0][2] * softplusf(sig[0] * zo[0] + kSoftplusShift);
    QR[0] = st[0][3] * softplusf(sig[0] * zn[0] + kSoftplusShift);
#pragma unroll
    for (int v = 1; v < 3; v++) {
        QL[v] = st[v][2] + sig[v] * zo[v];
        QR[v] = st[v][3] + sig[v] * zn[v];
    }
    bool ll = QL[0] > 0.0f, lr = QR[0] > 0.0f;
#pragma unroll
    for (int v = 0; v < 3; v++) {
        QL[v] = ll ? QL[v] : ML[v];
        QR[v] = lr ? QR[v] : MR[v];
    }
    return (ll ? 0 : 1) + (lr ? 0 : 1);
}

template <int FLUX, int AXIS>
__device__ __forceinline__ void flux3(const float *QL, const float *QR, const Phys<float> &ph, float *F)
{
    constexpr int NM = AXIS == 0 ? 1 : 2, TM = AXIS == 0 ? 2 : 1;
    float il = fvk::rcp(QL[0]), ir = fvk::rcp(QR[0]);
    SweV<float> L{QL[0], QL[NM] * il, QL[TM] * il}, R{QR[0], QR[NM] * ir, QR[TM] * ir};
    float G[3];
    fvk::swe_numflux<float, FLUX>(L, R, ph, G);
    F[0] = G[0];
    F[NM] = G[1];
    F[TM] = G[2];
}

// Flux-limiter blend (thesis section 2.5.3, second approach): the face flux F
// of the learned states is pulled towards the flux of the two cell averages,
// F <- F_low - phi (F_low - F), with phi the MINMOD flux limiter of the ratio
// r = (q_i - q_{i-1}) / (q_{i+1} - q_i) of the face's low-index cell i
// (stencil index 2), per conserved variable; phi = 0 where the ratio is
// undefined.  The limiter is taken without forming r where it is 0 or 1.
template <int FLUX, int AXIS>
__device__ __forceinline__ void blend_flux(const float (*st)[6], const Phys<float> &ph, float *F)
{
    float lo[3], hi[3], Fl[3];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        lo[v] = st[v][2];
        hi[v] = st[v][3];
    }
    flux3<FLUX, AXIS>(lo, hi, ph, Fl);
#pragma unroll
    for (int v = 0; v < 3; v++) {
        const float a = st[v][2] - st[v][1], b = st[v][3] - st[v][2];
        float phi = 0.0f;
        if ((a > 0.0f && b > 0.0f) || (a < 0.0f && b < 0.0f)) phi = __builtin_fabsf(a) >= __builtin_fabsf(b) ? 1.0f : a / b;
        F[v] = Fl[v] - phi * (Fl[v] - F[v]);
    }
}

}  // namespace cnn
