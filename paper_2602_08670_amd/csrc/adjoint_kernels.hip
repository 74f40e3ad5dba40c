// Reverse pass of one learned finite-volume stage (training, eq 2.28).
//
// Stage: out = a0*q0 + a1*(qs + dt*L(qs; alpha(qs))).  Given the adjoint of
// out, with w = a1*dt*g_out the adjoint of L:
//   - every face gets g_F = (w(owner+1) - w(owner)) / dx (the face flux
//     leaves the owner cell and enters its neighbour);
//   - the flux Jacobian with respect to the two face states comes from
//     forward-mode duals through the same templated flux code (exact for
//     the branch taken), giving g_QL, g_QR;
//   - a learned face side passes g_Q * alpha_k to its six stencil cells and
//     g_alpha_k = g_Q * q_k to the coefficients, mapped back to the raw
//     network outputs by g_z = P^T g_alpha = P g_alpha; a side that fell
//     back to MINMOD passes the MINMOD derivative (branch taken) instead.
// The face kernel writes each face's 18 stencil contributions next to its
// owner cell; the gather kernel sums, per cell and in a fixed order, the
// contributions of the twelve faces whose stencil contains it, so the
// result does not depend on scheduling.
#include "cnn_internal.hpp"
#include "dual.hpp"
#include "fv_device.hpp"
#include "learned_device.hpp"

namespace cnn {

using fvk::Dual;
using fvk::Phys;
using fvk::SweV;

struct AdjArgs {
    const float *qs;    // stage input [B][3][ny][nx]
    const float *z;     // raw coefficients of this stage [B][ny][nx][72]
    const float *gout;  // adjoint of the stage output [B][3][ny][nx]
    float wscale;       // a1 * dt
    int B, nx, ny;
    float rdx, rdy;
    Phys<float> ph;
    Proj pr;
    const int *plain;   // per solve: 1 = this step ran the plain scheme (or NULL)
    float *contrib;     // [2][B][ny][nx][ADJ_REC] (18 used)
    __bf16 *dz;         // [B][ny][nx][DZ_CH]
    float sig[3];       // direct scheme: 1 / inv_std of the network's input normalisation
};

// Flux-limiter blend of one face (section 2.5.3, second approach), per
// conserved variable v: F_v = (1 - phi_v) F_low,v + phi_v F_high,v with phi_v
// the MINMOD limiter of r = a / b, a = q_i - q_{i-1}, b = q_{i+1} - q_i at the
// face's low-index cell, as in the forward.  The adjoint freezes phi (the
// frozen-limiter adjoint): its derivative, of order 1 / b, is unbounded
// where successive differences vanish and overflows on a flat background.
__device__ __forceinline__ void blend_limiter(const float (*st)[6], float *phi)
{
#pragma unroll
    for (int v = 0; v < 3; v++) {
        const float a = st[v][2] - st[v][1], b = st[v][3] - st[v][2];
        const bool same = (a > 0.f && b > 0.f) || (a < 0.f && b < 0.f);
        const bool frac = same && __builtin_fabsf(a) < __builtin_fabsf(b);
        phi[v] = frac ? a / b : (same ? 1.f : 0.f);
    }
}

__device__ __forceinline__ int pw(int i, int n) { return ((i % n) + n) % n; }

// MINMOD face states of one variable and their derivatives with respect to
// the stencil cells k = 0..5 (only k = 1..4 are touched).  Branch rules as in
// the forward: minmod picks a when |a| <= |b| and both share a sign.
__device__ __forceinline__ void minmod_left(const float *c, float &val, float *dv)
{
    float a = c[2] - c[1], b = c[3] - c[2];
    bool same = (a > 0.f && b > 0.f) || (a < 0.f && b < 0.f);
    bool pa = same && __builtin_fabsf(a) <= __builtin_fabsf(b);
    bool pb = same && !pa;
    val = c[2] + 0.5f * (pa ? a : (pb ? b : 0.f));
    for (int k = 0; k < 6; k++) dv[k] = 0.f;
    dv[2] = 1.f;
    if (pa) { dv[2] += 0.5f; dv[1] -= 0.5f; }
    if (pb) { dv[3] += 0.5f; dv[2] -= 0.5f; }
}
__device__ __forceinline__ void minmod_right(const float *c, float &val, float *dv)
{
    float a = c[3] - c[2], b = c[4] - c[3];
    bool same = (a > 0.f && b > 0.f) || (a < 0.f && b < 0.f);
    bool pa = same && __builtin_fabsf(a) <= __builtin_fabsf(b);
    bool pb = same && !pa;
    val = c[3] - 0.5f * (pa ? a : (pb ? b : 0.f));
    for (int k = 0; k < 6; k++) dv[k] = 0.f;
    dv[3] = 1.f;
    if (pa) { dv[3] -= 0.5f; dv[2] += 0.5f; }
    if (pb) { dv[4] -= 0.5f; dv[3] += 0.5f; }
}

// DIR: the direct face-state scheme (section 5.3): the face's left state is
// the owner's right (top) state and its right state the neighbour's left
// (bottom) state; a side's depth is h_c softplus(sig_h z_h + c) and its
// momenta m_c + sig z_m (h_c, m_c: its own cell's), so a learned side passes
// g_Q softplus(sig_h z_h + c) (depth) and g_Q (momenta) to its own cell, and
// g_Q h_c sig_h sigmoid(sig_h z_h + c) and g_Q sig to its own cell's channels
// of z; this
// face writes the owner's high-side and the neighbour's low-side channels of
// dz (each written by exactly one face).
// BL: the learned face flux is blended with the flux of the two cell
// averages by the flux limiter (blend_limiter, phi frozen): the learned path
// receives phi g_F and the cell averages of the face (stencil entries 2 and
// 3) the low-resolution flux's Jacobian times (1 - phi) g_F.
template <int FLUX, bool DIR, bool BL = false>
__global__ __launch_bounds__(256) void adj_face_kernel(AdjArgs a)
{
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    const size_t nfaces = (size_t)2 * a.B * plane;
    for (size_t f = (size_t)blockIdx.x * 256 + threadIdx.x; f < nfaces; f += (size_t)gridDim.x * 256) {
        const int axis = (int)(f / ((size_t)a.B * plane));
        size_t r = f - (size_t)axis * a.B * plane;
        const int b = (int)(r / plane);
        const int cell = (int)(r - (size_t)b * plane);
        const int y = cell / nx, x = cell - y * nx;
        const int NM = axis == 0 ? 1 : 2, TM = axis == 0 ? 2 : 1;
        const float *q = a.qs + (size_t)b * 3 * plane;
        // stencil cells i-2 .. i+3 along the normal; owner i at k = 2
        int idx[6];
#pragma unroll
        for (int k = 0; k < 6; k++)
            idx[k] = axis == 0 ? y * nx + pw(x - 2 + k, nx) : pw(y - 2 + k, ny) * nx + x;
        float st[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = q[v * plane + idx[k]];
        const bool learned = !(a.plain && a.plain[b]);

        // forward recompute of the face states
        float ML[3], MR[3], dML[3][6], dMR[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            minmod_left(st[v], ML[v], dML[v]);
            minmod_right(st[v], MR[v], dMR[v]);
        }
        if (!(ML[0] > 0.f)) {  // safeguard: cell average of the owner
#pragma unroll
            for (int v = 0; v < 3; v++) {
                ML[v] = st[v][2];
                for (int k = 0; k < 6; k++) dML[v][k] = k == 2 ? 1.f : 0.f;
            }
        }
        if (!(MR[0] > 0.f)) {
#pragma unroll
            for (int v = 0; v < 3; v++) {
                MR[v] = st[v][3];
                for (int k = 0; k < 6; k++) dMR[v][k] = k == 3 ? 1.f : 0.f;
            }
        }
        float al[2][3][6];
        float QS[2][3];
        bool useL[2] = {false, false};
        // the cell across the face (the owner's +x or +y neighbour)
        const int nbc = axis == 0 ? y * nx + pw(x + 1, nx) : pw(y + 1, ny) * nx + x;
        float dsp[2] = {0.f, 0.f};  // direct: d depth / d z_h of each side
        if (DIR && learned) {
            const float *zo = a.z + ((size_t)b * plane + cell) * 72 + (axis == 0 ? 3 : 9);
            const float *zn = a.z + ((size_t)b * plane + nbc) * 72 + (axis == 0 ? 0 : 6);
            const float ao = a.sig[0] * zo[0] + kSoftplusShift, an = a.sig[0] * zn[0] + kSoftplusShift;
            const float so = softplusf(ao), sn = softplusf(an);
            dsp[0] = st[0][2] * a.sig[0] / (1.f + expf(-ao));
            dsp[1] = st[0][3] * a.sig[0] / (1.f + expf(-an));
#pragma unroll
            for (int v = 0; v < 3; v++) {
                QS[0][v] = v == 0 ? st[0][2] * so : st[v][2] + a.sig[v] * zo[v];
                QS[1][v] = v == 0 ? st[0][3] * sn : st[v][3] + a.sig[v] * zn[v];
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    al[0][v][k] = k == 2 ? (v == 0 ? so : 1.f) : 0.f;
                    al[1][v][k] = k == 3 ? (v == 0 ? sn : 1.f) : 0.f;
                }
            }
            useL[0] = QS[0][0] > 0.f;
            useL[1] = QS[1][0] > 0.f;
        } else if (learned) {
            // this face's 36 raw coefficients: nine 16-byte loads
            float zc[36];
            const float4 *z4 = (const float4 *)(a.z + ((size_t)b * plane + cell) * 72 + axis * 36);
#pragma unroll
            for (int q4 = 0; q4 < 9; q4++) {
                const float4 t = z4[q4];
                zc[4 * q4] = t.x;
                zc[4 * q4 + 1] = t.y;
                zc[4 * q4 + 2] = t.z;
                zc[4 * q4 + 3] = t.w;
            }
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int v = 0; v < 3; v++) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < 6; k++) {
                        float t = a.pr.base[s * 6 + k];
#pragma unroll
                        for (int j = 0; j < 6; j++) t += a.pr.P[k * 6 + j] * zc[(s * 3 + v) * 6 + j];
                        al[s][v][k] = t;
                        acc += t * st[v][k];
                    }
                    QS[s][v] = acc;
                }
            useL[0] = QS[0][0] > 0.f;
            useL[1] = QS[1][0] > 0.f;
        }
        float QL[3], QR[3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            QL[v] = useL[0] ? QS[0][v] : ML[v];
            QR[v] = useL[1] ? QS[1][v] : MR[v];
        }

        // flux Jacobian by duals: directions 0..2 = QL (Cartesian), 3..5 = QR
        typedef Dual<6> D;
        D hl = fvk::seed<6>(QL[0], 0), ml = fvk::seed<6>(QL[NM], NM), tl = fvk::seed<6>(QL[TM], TM);
        D hr = fvk::seed<6>(QR[0], 3), mr = fvk::seed<6>(QR[NM], 3 + NM), tr = fvk::seed<6>(QR[TM], 3 + TM);
        D il = fvk::rcp(hl), ir = fvk::rcp(hr);
        SweV<D> L{hl, ml * il, tl * il}, R{hr, mr * ir, tr * ir};
        Phys<D> ph{D(a.ph.g), D(a.ph.sqg), D(a.ph.gamma), D(a.ph.h0)};
        D F[3];
        fvk::swe_numflux<D, FLUX>(L, R, ph, F);
        D Fc[3];
        Fc[0] = F[0];
        Fc[NM] = F[1];
        Fc[TM] = F[2];

        // adjoint of the face flux
        const float rd = axis == 0 ? a.rdx : a.rdy;
        const int nb = nbc;
        const float *go = a.gout + (size_t)b * 3 * plane;
        float gF[3];
#pragma unroll
        for (int c = 0; c < 3; c++) gF[c] = a.wscale * rd * (go[c * plane + nb] - go[c * plane + cell]);
        // blend: the learned flux's share of the adjoint and the adjoint of
        // the low-resolution flux's states (phi frozen)
        float gH[3], gLo[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
        for (int c = 0; c < 3; c++) gH[c] = gF[c];
        if (BL && learned) {
            float phi[3];
            blend_limiter(st, phi);
            D cl[3], cr[3];
#pragma unroll
            for (int v = 0; v < 3; v++) {
                cl[v] = fvk::seed<6>(st[v][2], v);
                cr[v] = fvk::seed<6>(st[v][3], 3 + v);
            }
            D ilo = fvk::rcp(cl[0]), iro = fvk::rcp(cr[0]);
            SweV<D> Lo{cl[0], cl[NM] * ilo, cl[TM] * ilo}, Ro{cr[0], cr[NM] * iro, cr[TM] * iro};
            D Fn[3];
            fvk::swe_numflux<D, FLUX>(Lo, Ro, ph, Fn);
            D Flo[3];
            Flo[0] = Fn[0];
            Flo[NM] = Fn[1];
            Flo[TM] = Fn[2];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                gH[c] = phi[c] * gF[c];
                const float gl = (1.f - phi[c]) * gF[c];
#pragma unroll
                for (int v = 0; v < 3; v++) {
                    gLo[0][v] += gl * Flo[c].d[v];
                    gLo[1][v] += gl * Flo[c].d[3 + v];
                }
            }
        }
        float gQ[2][3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            float sl = 0.f, sr = 0.f;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                sl += gH[c] * Fc[c].d[v];
                sr += gH[c] * Fc[c].d[3 + v];
            }
            gQ[0][v] = sl;
            gQ[1][v] = sr;
        }

        // stencil contributions and coefficient adjoints, stored as 16-byte
        // vectors (the record of a face is ADJ_REC floats)
        float co[ADJ_REC], gzc[36];
#pragma unroll
        for (int v = 0; v < 3; v++) {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                float cL = useL[0] ? al[0][v][k] : dML[v][k];
                float cR = useL[1] ? al[1][v][k] : dMR[v][k];
                co[v * 6 + k] = gQ[0][v] * cL + gQ[1][v] * cR;
                if (BL) {
                    if (k == 2) co[v * 6 + k] += gLo[0][v];
                    if (k == 3) co[v * 6 + k] += gLo[1][v];
                }
            }
#pragma unroll
            for (int s = 0; s < 2; s++) {
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    float t = 0.f;
                    if (!DIR && useL[s]) {
#pragma unroll
                        for (int k = 0; k < 6; k++) t += a.pr.P[k * 6 + j] * (gQ[s][v] * st[v][k]);
                    }
                    gzc[(s * 3 + v) * 6 + j] = t;
                }
            }
        }
#pragma unroll
        for (int k = 18; k < ADJ_REC; k++) co[k] = 0.f;
        float4 *co4 = (float4 *)(a.contrib + (((size_t)axis * a.B + b) * plane + cell) * ADJ_REC);
#pragma unroll
        for (int q4 = 0; q4 < ADJ_REC / 4; q4++)
            co4[q4] = make_float4(co[4 * q4], co[4 * q4 + 1], co[4 * q4 + 2], co[4 * q4 + 3]);
        if (DIR) {
            __bf16 *dzo = a.dz + ((size_t)b * plane + cell) * DZ_CH + (axis == 0 ? 3 : 9);
            __bf16 *dzn = a.dz + ((size_t)b * plane + nbc) * DZ_CH + (axis == 0 ? 0 : 6);
#pragma unroll
            for (int v = 0; v < 3; v++) {
                dzo[v] = (__bf16)(useL[0] ? gQ[0][v] * (v == 0 ? dsp[0] : a.sig[v]) : 0.f);
                dzn[v] = (__bf16)(useL[1] ? gQ[1][v] * (v == 0 ? dsp[1] : a.sig[v]) : 0.f);
            }
        } else {
            typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
            bf16x4 *dz4 = (bf16x4 *)(a.dz + ((size_t)b * plane + cell) * DZ_CH + axis * 36);
#pragma unroll
            for (int q4 = 0; q4 < 9; q4++) {
                bf16x4 o;
#pragma unroll
                for (int e = 0; e < 4; e++) o[e] = (__bf16)gzc[4 * q4 + e];
                dz4[q4] = o;
            }
        }
    }
}

// out = (accumulate ? out : 0) + a1*gout + sum of the stencil contributions
// of the 12 faces around each cell, in a fixed order.
__global__ __launch_bounds__(256) void adj_gather_kernel(float *out, const float *gout, float a1,
                                                         const float *contrib, int B, int nx, int ny, int accumulate)
{
    const size_t plane = (size_t)nx * ny;
    const size_t n = (size_t)B * plane;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int b = (int)(i / plane);
        const int cell = (int)(i - (size_t)b * plane);
        const int y = cell / nx, x = cell - y * nx;
        float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int axis = 0; axis < 2; axis++)
#pragma unroll
            for (int k = 0; k < 6; k++) {
                // this cell is stencil entry k of the face owned by cell - (k - 2)
                int own = axis == 0 ? y * nx + pw(x + 2 - k, nx) : pw(y + 2 - k, ny) * nx + x;
                const float *co = contrib + (((size_t)axis * B + b) * plane + own) * ADJ_REC;
#pragma unroll
                for (int v = 0; v < 3; v++) acc[v] += co[v * 6 + k];
            }
#pragma unroll
        for (int v = 0; v < 3; v++) {
            size_t o = (size_t)b * 3 * plane + v * plane + cell;
            float base = accumulate ? out[o] : 0.f;
            out[o] = base + a1 * gout[o] + acc[v];
        }
    }
}

hipError_t launch_adjoint(int flux, const AdjStage &s, hipStream_t st)
{
    AdjArgs a;
    a.qs = s.qs;
    a.z = s.z;
    a.gout = s.gout;
    a.wscale = s.a1 * s.dt;
    a.B = s.B;
    a.nx = s.nx;
    a.ny = s.ny;
    a.rdx = s.rdx;
    a.rdy = s.rdy;
    a.ph.g = s.g;
    a.ph.sqg = __builtin_sqrtf(s.g);
    a.ph.gamma = 1.4f;
    a.ph.h0 = s.h0;
    a.pr = s.pr;
    a.plain = s.plain;
    a.contrib = s.contrib;
    a.dz = (__bf16 *)s.dz;
    for (int v = 0; v < 3; v++) a.sig[v] = s.sig[v];
    size_t nf = (size_t)2 * s.B * s.nx * s.ny;
    unsigned blocks = (unsigned)((nf + 255) / 256);
    if (s.direct && s.blend) return hipErrorInvalidValue;
    if (s.direct) {
        if (flux == 1) hipLaunchKernelGGL((adj_face_kernel<fvk::RUSANOV, true>), dim3(blocks), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((adj_face_kernel<fvk::HLLE, true>), dim3(blocks), dim3(256), 0, st, a);
    } else if (s.blend) {
        if (flux == 1) hipLaunchKernelGGL((adj_face_kernel<fvk::RUSANOV, false, true>), dim3(blocks), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((adj_face_kernel<fvk::HLLE, false, true>), dim3(blocks), dim3(256), 0, st, a);
    } else {
        if (flux == 1) hipLaunchKernelGGL((adj_face_kernel<fvk::RUSANOV, false>), dim3(blocks), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((adj_face_kernel<fvk::HLLE, false>), dim3(blocks), dim3(256), 0, st, a);
    }
    size_t nc = (size_t)s.B * s.nx * s.ny;
    hipLaunchKernelGGL(adj_gather_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, s.gqs, s.gout, s.a1,
                       (const float *)s.contrib, s.B, s.nx, s.ny, s.accumulate);
    return hipGetLastError();
}

}  // namespace cnn
