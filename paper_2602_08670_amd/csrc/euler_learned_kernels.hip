// Learned stencil-coefficient stage for the 2D Euler equations (the planar
// construction of thesis section 2.5.3, fourth approach, on the system of
// section 4.2; section 6.2 asks for it with positive density and energy).
//
// One workgroup of 256 threads per 32 x 4 cell tile of one solve: the tile
// and a three-cell halo of the four conserved variables are staged in LDS;
// each thread evaluates one x face and one y face (the cell's low faces and
// the tile's high edge), reading the owner cell's 48 raw coefficients of
// that axis, projecting them (alpha = base + P z per group of six) and
// forming both face states; a side whose learned state has rho <= 0, p <= 0
// or a non-finite value takes its MINMOD state (itself the cell average
// where MINMOD is inadmissible).  The Euler flux (HLLE or Rusanov) is taken
// in the face's normal frame, and each thread then updates one cell.
//
// Modes (per solve flags in two slots, the step's parity picking one):
//   0  learned stage: out = a0 q0 + a1 (qs + dt L(qs)), flag bit set when a
//      cell of the result is inadmissible, fallback sides counted (not for
//      stage 2 of a solve whose stage 1 failed);
//   2  solves whose flag is 0 commit S2 -> q (commit_src NULL: nothing to
//      copy); the others run the plain MINMOD first stage S1 = q + dt L(q);
//   3  solves whose flag is set run the plain second stage
//      q = (q + S1 + dt L(S1)) / 2 (a still inadmissible result freezes the
//      solve); bookkeeping: redone count, the other slot cleared.
#include <hip/hip_runtime.h>

#include "cnn_internal.hpp"
#include "dual.hpp"
#include "euler_learned_device.hpp"
#include "euler_learned_internal.hpp"
#include "fv_device.hpp"

namespace eln {

using fvk::EulS;

constexpr int TX = 32, TY = 4, HX = TX + 6, HY = TY + 6;

__device__ __forceinline__ int pwrap(int i, int n) { return ((i % n) + n) % n; }

template <int MODE, int FLUX>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs a)
{
    static_assert(TY * (TX + 1) <= 256 && (TY + 1) * TX <= 256, "one face per axis and thread");
    __shared__ float s_q[4][HY][HX];
    __shared__ float s_fx[4][TY][TX + 1];
    __shared__ float s_fy[4][TY + 1][TX];
    __shared__ int s_cnt, s_bad;
    const int b = blockIdx.z, x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tid = threadIdx.x, nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    int *flag = a.flags + 2 * b + a.parity;
    if (MODE == 3 && a.record && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) a.record[b] = *flag != 0;
    if (a.fatal[b]) return;  // frozen solve
    if (MODE == 3 && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) {
        // this step's flag is read only in this launch; the other slot is
        // not read before the next step
        if (*flag && a.redone) a.redone[b] += 1;
        a.flags[2 * b + (a.parity ^ 1)] = 0;
    }
    const int fl = *flag;
    if (MODE == 2 && fl == 0) {
        if (!a.commit_src) return;  // the result is already in place
        for (int k = tid; k < TX * TY; k += 256) {
            const int cy = k / TX, cx = k - cy * TX;
            if (x0 + cx >= nx || y0 + cy >= ny) continue;
            const size_t idx = (size_t)b * 4 * plane + (size_t)(y0 + cy) * nx + x0 + cx;
#pragma unroll
            for (int v = 0; v < 4; v++) a.commit_dst[idx + v * plane] = a.commit_src[idx + v * plane];
        }
        return;
    }
    if (MODE == 3 && fl == 0) return;
    constexpr bool LEARNED = MODE == 0;
    const float *qs = a.qs + (size_t)b * 4 * plane;
    const bool count = LEARNED && !(a.flagbit == 2 && (fl & 1));
    if (tid == 0) {
        s_cnt = 0;
        s_bad = 0;
    }
    for (int k = tid; k < HY * HX; k += 256) {
        const int ly = k / HX, lx = k - ly * HX;
        const size_t idx = (size_t)pwrap(y0 - 3 + ly, ny) * nx + pwrap(x0 - 3 + lx, nx);
#pragma unroll
        for (int v = 0; v < 4; v++) s_q[v][ly][lx] = qs[v * plane + idx];
    }
    __syncthreads();

    int nfb = 0;
    // x face of thread tid: owner cell (x0 - 1 + xi, y0 + xj) at halo column
    // xi + 2; y face: owner (x0 + yi, y0 - 1 + yj) at halo row yj + 2
    constexpr int NFX = TY * (TX + 1), NFY = (TY + 1) * TX;
    if (tid < NFX) {
        const int xj = tid / (TX + 1), xi = tid - xj * (TX + 1);
        float st[4][6];
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = s_q[v][xj + 3][xi + k];
        float zc[48];
        if (LEARNED) {
            const int gy = y0 + xj < ny ? y0 + xj : ny - 1;
            const float4 *pz =
                (const float4 *)(a.z + (((size_t)b * ny + gy) * nx + pwrap(x0 - 1 + xi, nx)) * cnn::E_COUT);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const float4 u = pz[k];
                zc[4 * k] = u.x;
                zc[4 * k + 1] = u.y;
                zc[4 * k + 2] = u.z;
                zc[4 * k + 3] = u.w;
            }
        }
        float QL[4], QR[4], F[4];
        const int c = face_states<LEARNED>(st, zc, a.pr, a.gamma, QL, QR);
        if (xi < TX && x0 + xi < nx && y0 + xj < ny) nfb += c;  // counted once: as a cell's low face
        flux4<FLUX, 0>(QL, QR, a.gamma, F);
#pragma unroll
        for (int v = 0; v < 4; v++) s_fx[v][xj][xi] = F[v];
    }
    if (tid < NFY) {
        const int yj = tid / TX, yi = tid - yj * TX;
        float st[4][6];
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = s_q[v][yj + k][yi + 3];
        float zc[48];
        if (LEARNED) {
            const int gx = x0 + yi < nx ? x0 + yi : nx - 1;
            const float4 *pz =
                (const float4 *)(a.z + (((size_t)b * ny + pwrap(y0 - 1 + yj, ny)) * nx + gx) * cnn::E_COUT + 48);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const float4 u = pz[k];
                zc[4 * k] = u.x;
                zc[4 * k + 1] = u.y;
                zc[4 * k + 2] = u.z;
                zc[4 * k + 3] = u.w;
            }
        }
        float QL[4], QR[4], F[4];
        const int c = face_states<LEARNED>(st, zc, a.pr, a.gamma, QL, QR);
        if (yj < TY && y0 + yj < ny && x0 + yi < nx) nfb += c;
        flux4<FLUX, 1>(QL, QR, a.gamma, F);
#pragma unroll
        for (int v = 0; v < 4; v++) s_fy[v][yj][yi] = F[v];
    }
    __syncthreads();

    // MODE 0 and 2 (plain first stage): out = a0 q0 + a1 (qs + dt L);
    // MODE 3 (plain second stage): q = q/2 + (S1 + dt L(S1))/2
    bool bad = false;
    if (tid < TX * TY) {
        const int cy = tid / TX, cx = tid - cy * TX, gx = x0 + cx, gy = y0 + cy;
        if (gx < nx && gy < ny) {
            const size_t idx = (size_t)b * 4 * plane + (size_t)gy * nx + gx;
            float qn[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const float L = -(s_fx[v][cy][cx + 1] - s_fx[v][cy][cx]) * a.rdx -
                                (s_fy[v][cy + 1][cx] - s_fy[v][cy][cx]) * a.rdy;
                float o = a.a1 * (s_q[v][cy + 3][cx + 3] + a.dt * L);
                if (a.a0 != 0.0f) o = a.a0 * a.q0[idx + v * plane] + o;
                a.out[idx + v * plane] = o;
                qn[v] = o;
            }
            bad = !admissible(qn, a.gamma);
        }
    }
    if (count && nfb) atomicAdd(&s_cnt, nfb);
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0) {
        if (s_cnt) atomicAdd(&a.nfb[b], (unsigned long long)s_cnt);
        if (s_bad) {
            if (MODE == 0) atomicOr(flag, a.flagbit);
            else if (MODE == 3) atomicExch(&a.fatal[b], 1);
        }
    }
}

hipError_t stage(int mode, int flux, const StageArgs &a, hipStream_t st)
{
    if (a.nx < 1 || a.ny < 1 || a.B < 1) return hipErrorInvalidValue;
    const dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, a.B), blk(256);
    const bool rus = flux == fvk::RUSANOV;
#define ELN_LAUNCH(M)                                                                                                 \
    do {                                                                                                              \
        if (rus) hipLaunchKernelGGL((stage_kernel<M, fvk::RUSANOV>), grid, blk, 0, st, a);                           \
        else hipLaunchKernelGGL((stage_kernel<M, fvk::HLLE>), grid, blk, 0, st, a);                                  \
    } while (0)
    switch (mode) {
    case 0: ELN_LAUNCH(0); break;
    case 2: ELN_LAUNCH(2); break;
    case 3: ELN_LAUNCH(3); break;
    default: return hipErrorInvalidValue;
    }
#undef ELN_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------- adjoint
// Reverse of one learned stage out = a0 q0 + a1 (qs + dt L(qs; z(qs))), as
// the planar adjoint: with w = a1 dt g_out the adjoint of L, every face gets
// g_F = (w(owner + 1) - w(owner)) / dx; the flux Jacobian with respect to the
// two face states comes from forward-mode duals through the same Euler flux
// code (exact for the branch taken); a learned side passes g_Q alpha_k to its
// six stencil cells and g_z = P g_alpha (g_alpha_k = g_Q q_k) to the owner's
// raw coefficients, a side on its MINMOD state the MINMOD derivative (branch
// taken; the cell average where MINMOD was inadmissible).  Each face writes
// its 24 stencil contributions next to its owner; the gather sums, per cell
// and in a fixed order, those of the twelve faces whose stencil holds it.

__device__ __forceinline__ void minmod_d(float a, float b, float &m, float &da, float &db)
{
    const bool same = (a > 0.f && b > 0.f) || (a < 0.f && b < 0.f);
    const bool pa = same && __builtin_fabsf(a) <= __builtin_fabsf(b);
    const bool pb = same && !pa;
    m = pa ? a : (pb ? b : 0.f);
    da = pa ? 1.f : 0.f;
    db = pb ? 1.f : 0.f;
}

template <int FLUX>
__global__ __launch_bounds__(256) void adj_face_kernel(AdjArgs a)
{
    using D = fvk::Dual<8>;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    const size_t nfaces = (size_t)2 * a.B * plane;
    for (size_t f = (size_t)blockIdx.x * 256 + threadIdx.x; f < nfaces; f += (size_t)gridDim.x * 256) {
        const int axis = (int)(f / ((size_t)a.B * plane));
        const size_t r = f - (size_t)axis * a.B * plane;
        const int b = (int)(r / plane);
        const int cell = (int)(r - (size_t)b * plane);
        const int y = cell / nx, x = cell - y * nx;
        const int NM = axis == 0 ? 1 : 2, TM = axis == 0 ? 2 : 1;
        const float *q = a.qs + (size_t)b * 4 * plane;
        int idx[6];
#pragma unroll
        for (int k = 0; k < 6; k++) idx[k] = axis == 0 ? y * nx + pwrap(x - 2 + k, nx) : pwrap(y - 2 + k, ny) * nx + x;
        float st[4][6];
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = q[v * plane + idx[k]];
        const bool learned = !(a.plain && a.plain[b]);

        // MINMOD states (the forward's recon) and their derivatives
        float ML[4], MR[4], dML[4][6], dMR[4][6];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            float m, da, db;
#pragma unroll
            for (int k = 0; k < 6; k++) dML[v][k] = dMR[v][k] = 0.f;
            minmod_d(st[v][2] - st[v][1], st[v][3] - st[v][2], m, da, db);
            ML[v] = st[v][2] + 0.5f * m;
            dML[v][1] = -0.5f * da;
            dML[v][2] = 1.f + 0.5f * (da - db);
            dML[v][3] = 0.5f * db;
            minmod_d(st[v][3] - st[v][2], st[v][4] - st[v][3], m, da, db);
            MR[v] = st[v][3] - 0.5f * m;
            dMR[v][2] = 0.5f * da;
            dMR[v][3] = 1.f - 0.5f * (da - db);
            dMR[v][4] = -0.5f * db;
        }
        if (!admissible(ML, a.gamma)) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                ML[v] = st[v][2];
#pragma unroll
                for (int k = 0; k < 6; k++) dML[v][k] = k == 2 ? 1.f : 0.f;
            }
        }
        if (!admissible(MR, a.gamma)) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                MR[v] = st[v][3];
#pragma unroll
                for (int k = 0; k < 6; k++) dMR[v][k] = k == 3 ? 1.f : 0.f;
            }
        }
        float al[2][4][6], QS[2][4];
        bool useL[2] = {false, false};
        if (learned) {
            const float4 *z4 = (const float4 *)(a.z + ((size_t)b * plane + cell) * cnn::E_COUT + axis * 48);
            float zc[48];
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const float4 t = z4[k];
                zc[4 * k] = t.x;
                zc[4 * k + 1] = t.y;
                zc[4 * k + 2] = t.z;
                zc[4 * k + 3] = t.w;
            }
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < 6; k++) {
                        float t = a.pr.base[s * 6 + k];
#pragma unroll
                        for (int j = 0; j < 6; j++) t += a.pr.P[k * 6 + j] * zc[(s * 4 + v) * 6 + j];
                        al[s][v][k] = t;
                        acc += t * st[v][k];
                    }
                    QS[s][v] = acc;
                }
            useL[0] = admissible(QS[0], a.gamma);
            useL[1] = admissible(QS[1], a.gamma);
        }
        float QL[4], QR[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            QL[v] = useL[0] ? QS[0][v] : ML[v];
            QR[v] = useL[1] ? QS[1][v] : MR[v];
        }
        // flux Jacobian: directions 0..3 = QL, 4..7 = QR (Cartesian order)
        const EulS<D> L{fvk::seed<8>(QL[0], 0), fvk::seed<8>(QL[NM], NM), fvk::seed<8>(QL[TM], TM),
                        fvk::seed<8>(QL[3], 3)};
        const EulS<D> R{fvk::seed<8>(QR[0], 4), fvk::seed<8>(QR[NM], 4 + NM), fvk::seed<8>(QR[TM], 4 + TM),
                        fvk::seed<8>(QR[3], 7)};
        D G[4];
        fvk::eul_numflux<D, FLUX>(L, R, D(a.gamma), G);
        D Fc[4];
        Fc[0] = G[0];
        Fc[NM] = G[1];
        Fc[TM] = G[2];
        Fc[3] = G[3];
        const float rd = axis == 0 ? a.rdx : a.rdy;
        const int nb = axis == 0 ? y * nx + pwrap(x + 1, nx) : pwrap(y + 1, ny) * nx + x;
        const float *go = a.gout + (size_t)b * 4 * plane;
        float gF[4];
#pragma unroll
        for (int c = 0; c < 4; c++) gF[c] = a.wscale * rd * (go[c * plane + nb] - go[c * plane + cell]);
        float gQ[2][4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            float sl = 0.f, sr = 0.f;
#pragma unroll
            for (int c = 0; c < 4; c++) {
                sl += gF[c] * Fc[c].d[v];
                sr += gF[c] * Fc[c].d[4 + v];
            }
            gQ[0][v] = sl;
            gQ[1][v] = sr;
        }
        float co[ADJ_REC];
        __bf16 gz[48];
#pragma unroll
        for (int v = 0; v < 4; v++) {
#pragma unroll
            for (int k = 0; k < 6; k++)
                co[v * 6 + k] = gQ[0][v] * (useL[0] ? al[0][v][k] : dML[v][k]) +
                                gQ[1][v] * (useL[1] ? al[1][v][k] : dMR[v][k]);
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    float t = 0.f;
                    if (useL[s]) {
#pragma unroll
                        for (int k = 0; k < 6; k++) t += a.pr.P[k * 6 + j] * (gQ[s][v] * st[v][k]);
                    }
                    gz[(s * 4 + v) * 6 + j] = (__bf16)t;
                }
        }
        float4 *co4 = (float4 *)(a.contrib + (((size_t)axis * a.B + b) * plane + cell) * ADJ_REC);
#pragma unroll
        for (int k = 0; k < ADJ_REC / 4; k++) co4[k] = make_float4(co[4 * k], co[4 * k + 1], co[4 * k + 2], co[4 * k + 3]);
        typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
        bf16x8 *dz8 = (bf16x8 *)(a.dz + ((size_t)b * plane + cell) * cnn::E_COUT + axis * 48);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; e++) o[e] = gz[8 * k + e];
            dz8[k] = o;
        }
    }
}

// out = (accumulate ? out : 0) + a1 gout + the stencil contributions of the
// twelve faces around each cell, in a fixed order.
__global__ __launch_bounds__(256) void adj_gather_kernel(float *out, const float *gout, float a1,
                                                         const float *contrib, int B, int nx, int ny, int accumulate)
{
    const size_t plane = (size_t)nx * ny;
    const size_t n = (size_t)B * plane;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int b = (int)(i / plane);
        const int cell = (int)(i - (size_t)b * plane);
        const int y = cell / nx, x = cell - y * nx;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int axis = 0; axis < 2; axis++)
#pragma unroll
            for (int k = 0; k < 6; k++) {
                // this cell is stencil entry k of the face owned by cell - (k - 2)
                const int own = axis == 0 ? y * nx + pwrap(x + 2 - k, nx) : pwrap(y + 2 - k, ny) * nx + x;
                const float *co = contrib + (((size_t)axis * B + b) * plane + own) * ADJ_REC;
#pragma unroll
                for (int v = 0; v < 4; v++) acc[v] += co[v * 6 + k];
            }
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const size_t o = (size_t)b * 4 * plane + v * plane + cell;
            out[o] = (accumulate ? out[o] : 0.f) + a1 * gout[o] + acc[v];
        }
    }
}

hipError_t adjoint(int flux, const AdjArgs &a, float *gqs, float a1, int accumulate, hipStream_t st)
{
    const size_t nf = (size_t)2 * a.B * a.nx * a.ny;
    unsigned blocks = (unsigned)((nf + 255) / 256);
    if (flux == fvk::RUSANOV) hipLaunchKernelGGL((adj_face_kernel<fvk::RUSANOV>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((adj_face_kernel<fvk::HLLE>), dim3(blocks), dim3(256), 0, st, a);
    const size_t nc = (size_t)a.B * a.nx * a.ny;
    hipLaunchKernelGGL(adj_gather_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, gqs, a.gout, a1,
                       (const float *)a.contrib, a.B, a.nx, a.ny, accumulate);
    return hipGetLastError();
}

}  // namespace eln
