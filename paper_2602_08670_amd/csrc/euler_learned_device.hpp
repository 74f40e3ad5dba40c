// Face states and fluxes of the learned Euler stage (the planar learned
// construction of thesis section 2.5.3, fourth approach, on the system of
// section 4.2), shared by the learned Euler stage kernels and the network
// pass that runs the stage in the same workgroup.
#pragma once

#include "cnn_internal.hpp"
#include "fv_device.hpp"

namespace eln {

using fvk::EulS;

// rho > 0, p > 0 and every component finite.
__device__ __forceinline__ bool admissible(const float *Q, float gamma)
{
    const float p = (gamma - 1.0f) * (Q[3] - 0.5f * (Q[1] * Q[1] + Q[2] * Q[2]) / Q[0]);
    return Q[0] > 0.0f && p > 0.0f && __builtin_isfinite(Q[0]) && __builtin_isfinite(Q[1]) &&
           __builtin_isfinite(Q[2]) && __builtin_isfinite(Q[3]);
}

// Face states from the stencil st[v][0..5] (cells i-2..i+3 along the
// normal); LEARNED: from the owner's 48 raw coefficients of this axis
// (zc[(side*4 + v)*6 + k]), or with AL from its 48 projected ones (alpha =
// base + P z, the same operation order).  Returns the number of sides that
// fell back.
template <bool LEARNED, bool AL = false>
__device__ __forceinline__ int face_states(const float (*st)[6], const float *zc, const cnn::Proj &pr, float gamma,
                                           float *QL, float *QR)
{
    float ML[4], MR[4];
#pragma unroll
    for (int v = 0; v < 4; v++) fvk::recon_pair<float, fvk::MINMOD>(st[v][1], st[v][2], st[v][3], st[v][4], ML[v], MR[v]);
    const bool okl = admissible(ML, gamma), okr = admissible(MR, gamma);
#pragma unroll
    for (int v = 0; v < 4; v++) {
        ML[v] = okl ? ML[v] : st[v][2];
        MR[v] = okr ? MR[v] : st[v][3];
    }
    if (!LEARNED) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            QL[v] = ML[v];
            QR[v] = MR[v];
        }
        return 0;
    }
#pragma unroll
    for (int s = 0; s < 2; s++) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const float *zz = zc + (s * 4 + v) * 6;
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
    const bool ll = admissible(QL, gamma), lr = admissible(QR, gamma);
#pragma unroll
    for (int v = 0; v < 4; v++) {
        QL[v] = ll ? QL[v] : ML[v];
        QR[v] = lr ? QR[v] : MR[v];
    }
    return (ll ? 0 : 1) + (lr ? 0 : 1);
}

template <int FLUX, int AXIS>
__device__ __forceinline__ void flux4(const float *QL, const float *QR, float gamma, float *F)
{
    constexpr int NM = AXIS == 0 ? 1 : 2, TM = AXIS == 0 ? 2 : 1;
    const EulS<float> L{QL[0], QL[NM], QL[TM], QL[3]}, R{QR[0], QR[NM], QR[TM], QR[3]};
    float G[4];
    fvk::eul_numflux<float, FLUX>(L, R, gamma, G);
    F[0] = G[0];
    F[NM] = G[1];
    F[TM] = G[2];
    F[3] = G[3];
}

}  // namespace eln
