// Learned-coefficient finite-volume stage for batches of periodic
// shallow-water solves (FP32), thesis section 2.5.3, fourth approach.
//
// Every cell owns its +x and +y face.  For a face the kernel reads the
// owner's 36 raw coefficients z (one axis: 2 sides x 3 variables x 6), maps
// them onto the constraint set, alpha = alpha_base + P z (P: orthogonal
// projector onto the null space of the moment conditions), and forms the two
// face states as sum_k alpha_k q(i-2+k) over the six cells around the face.
// A side whose learned depth is not positive uses its MINMOD state instead
// (counted).  Fluxes, divergence and the Runge-Kutta combine follow the
// classic stage kernel.  MODE 1 runs the plain MINMOD scheme only for the
// solves whose learned step produced an inadmissible cell (the step is redone).
// MODE 2 and 3 end a step in two launches: MODE 2 commits the learned result
// of the admissible solves and runs the plain first stage for the others;
// MODE 3 runs the plain second stage for those and does the step's
// bookkeeping.
#include "cnn_internal.hpp"
#include "fv_device.hpp"
#include "learned_device.hpp"

namespace cnn {

using fvk::Phys;
using fvk::SweV;

struct LearnedArgs {
    const float *qs;  // stage input [B][3][ny][nx]
    const float *q0;  // q^n, read only at the updated cell
    float *out;
    const float *z;   // [B][ny][nx][72]
    int B, nx, ny;
    float rdx, rdy;
    Phys<float> ph;
    float a0, a1;
    const float *dt;         // per solve
    int *bad;                // per solve flag bits
    int flagbit;
    unsigned long long *nfb; // per solve fallback face sides
    int *fatal;              // per solve: the plain redo itself failed
    Proj pr;
    const float *commit_src;
    float *commit_dst;
    int *bad_next;
    unsigned long long *redone;
    double *t;
    long long *steps;
    float sig[3];                // direct scheme: 1 / inv_std of the network's input normalisation
};

// One LTILE_X x LTILE_Y tile of solve b at (x0, y0); `first` marks the
// solve's tile that does the per-step bookkeeping of MODE 3.  The tile is
// small enough for every thread to own at most one x face, one y face and
// one cell: the coefficients of both faces are loaded before any face is
// evaluated, so a stage costs about one global-load latency on the small
// grids of the learned solver.
// DIR (MODE 0 only): the direct face-state scheme of section 5.3, z holding
// the network's raw output (channels 0..11: left, right, bottom, top states'
// corrections); the MINMOD fallback, flags and counters are the learned
// stage's.
// BL (MODE 0 only): every face's flux is the flux-limiter blend of the
// learned flux and the flux of the two cell averages (blend_flux).
template <int MODE, int FLUX, bool AL, bool DIR = false, bool BL = false>
__device__ __forceinline__ void learned_tile(const LearnedArgs &a, const int b, const int x0, const int y0,
                                             const bool first)
{
    constexpr int TX = LTILE_X, TY = LTILE_Y, HX = TX + 6, HY = TY + 6;
    constexpr int NFX = TY * (TX + 1), NFY = (TY + 1) * TX;
    static_assert(NFX <= 256 && NFY <= 256 && TX * TY <= 256, "one face per axis and one cell per thread");
    __shared__ float s_q[3][HY][HX];
    __shared__ float s_fx[3][TY][TX + 1];
    __shared__ float s_fy[3][TY + 1][TX];
    __shared__ int s_cnt;
    __shared__ int s_bad;

    constexpr int FS = MODE == 0 ? 0 : 1;  // face states: learned or plain MINMOD
    const int tid = threadIdx.x;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    if (MODE == 3 && first && tid == 0) {
        // this step's flags are only read in this launch; the next step's
        // flags are not read before the next step
        const int flag = a.bad[b];
        if (flag && a.redone) a.redone[b] += 1;
        a.bad_next[b] = 0;
        if (b == 0 && a.t) {
            *a.t += (double)a.dt[0];
            *a.steps += 1;
        }
    }
    if (MODE == 2 && a.bad[b] == 0) {
        // admissible learned step: q <- S2 on this tile (no source: the
        // result is already in place)
        if (!a.commit_src) return;
        for (int k = tid; k < TX * TY; k += 256) {
            const int cy = k / TX, cx = k - cy * TX;
            if (x0 + cx >= nx || y0 + cy >= ny) continue;
            const size_t idx = (size_t)b * 3 * plane + (size_t)(y0 + cy) * nx + x0 + cx;
#pragma unroll
            for (int v = 0; v < 3; v++) a.commit_dst[idx + v * plane] = a.commit_src[idx + v * plane];
        }
        return;
    }
    if ((MODE == 1 || MODE == 3) && a.bad[b] == 0) return;
    const float *qs = a.qs + (size_t)b * 3 * plane;
    const float dt = a.dt[b];
    // stage 2 of a solve whose stage 1 failed is evaluated (its result is
    // discarded by the redo) but its fallback faces are not counted
    const bool count = MODE == 0 && !(a.flagbit == 2 && (a.bad[b] & 1));
    if (tid == 0) {
        s_cnt = 0;
        s_bad = 0;
    }
    for (int k = tid; k < HY * HX; k += 256) {
        int ly = k / HX, lx = k - ly * HX;
        size_t idx = (size_t)pwrap(y0 - 3 + ly, ny) * nx + pwrap(x0 - 3 + lx, nx);
#pragma unroll
        for (int v = 0; v < 3; v++) s_q[v][ly][lx] = qs[v * plane + idx];
    }
    __syncthreads();

    int nfb = 0;
    // this thread's x face: owner cell (x0 - 1 + xi, y0 + xj) <-> halo
    // column xi + 2; its y face: owner cell (x0 + yi, y0 - 1 + yj) <-> halo
    // row yj + 2.  Threads past a face count read a valid face's
    // coefficients and discard them.
    const bool hx = tid < NFX, hy = tid < NFY;
    const int tx_ = hx ? tid : 0, ty_ = hy ? tid : 0;
    const int xj = tx_ / (TX + 1), xi = tx_ - xj * (TX + 1);
    const int yj = ty_ / TX, yi = ty_ - yj * TX;
    float zx[36], zy[36];
    if (DIR) {
        // x face: the owner's right state (channels 3..5) and the neighbour's
        // left state (0..2); y face: the owner's top state (9..11) and the
        // neighbour's bottom state (6..8)
        const int gy = y0 + xj < ny ? y0 + xj : ny - 1;
        const int gx = x0 + yi < nx ? x0 + yi : nx - 1;
        const float *zb = a.z + (size_t)b * ny * nx * 72;
        const float *ox = zb + ((size_t)gy * nx + pwrap(x0 - 1 + xi, nx)) * 72;
        const float *nxp = zb + ((size_t)gy * nx + pwrap(x0 + xi, nx)) * 72;
        const float *oy = zb + ((size_t)pwrap(y0 - 1 + yj, ny) * nx + gx) * 72;
        const float *nyp = zb + ((size_t)pwrap(y0 + yj, ny) * nx + gx) * 72;
#pragma unroll
        for (int v = 0; v < 3; v++) {
            zx[v] = ox[3 + v];
            zx[3 + v] = nxp[v];
            zy[v] = oy[9 + v];
            zy[3 + v] = nyp[6 + v];
        }
    } else if (FS == 0) {
        const int gy = y0 + xj < ny ? y0 + xj : ny - 1;
        const int gx = x0 + yi < nx ? x0 + yi : nx - 1;
        const float4 *px = (const float4 *)(a.z + (((size_t)b * ny + gy) * nx + pwrap(x0 - 1 + xi, nx)) * 72);
        const float4 *py = (const float4 *)(a.z + (((size_t)b * ny + pwrap(y0 - 1 + yj, ny)) * nx + gx) * 72 + 36);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const float4 u = px[k], w = py[k];
            zx[4 * k] = u.x; zx[4 * k + 1] = u.y; zx[4 * k + 2] = u.z; zx[4 * k + 3] = u.w;
            zy[4 * k] = w.x; zy[4 * k + 1] = w.y; zy[4 * k + 2] = w.z; zy[4 * k + 3] = w.w;
        }
    }
    if (hx) {
        float st[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = s_q[v][xj + 3][xi + k];
        float QL[3], QR[3], F[3];
        int c = DIR ? face_states_direct(st, zx, zx + 3, a.sig, QL, QR) : face_states<FS, AL>(st, zx, a.pr, QL, QR);
        // each face is counted once: as the left face of a cell of this tile
        if (xi < TX && x0 + xi < nx && y0 + xj < ny) nfb += c;
        flux3<FLUX, 0>(QL, QR, a.ph, F);
        if (BL) blend_flux<FLUX, 0>(st, a.ph, F);
#pragma unroll
        for (int v = 0; v < 3; v++) s_fx[v][xj][xi] = F[v];
    }
    if (hy) {
        float st[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = s_q[v][yj + k][yi + 3];
        float QL[3], QR[3], F[3];
        int c = DIR ? face_states_direct(st, zy, zy + 3, a.sig, QL, QR) : face_states<FS, AL>(st, zy, a.pr, QL, QR);
        if (yj < TY && y0 + yj < ny && x0 + yi < nx) nfb += c;
        flux3<FLUX, 1>(QL, QR, a.ph, F);
        if (BL) blend_flux<FLUX, 1>(st, a.ph, F);
#pragma unroll
        for (int v = 0; v < 3; v++) s_fy[v][yj][yi] = F[v];
    }
    __syncthreads();

    bool bad = false;
    for (int k = tid; k < TX * TY; k += 256) {
        int cy = k / TX, cx = k - cy * TX;
        int gx = x0 + cx, gy = y0 + cy;
        if (gx >= nx || gy >= ny) continue;
        size_t idx = (size_t)b * 3 * plane + (size_t)gy * nx + gx;
        float qn[3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            float L = -(s_fx[v][cy][cx + 1] - s_fx[v][cy][cx]) * a.rdx - (s_fy[v][cy + 1][cx] - s_fy[v][cy][cx]) * a.rdy;
            float o = a.a1 * (s_q[v][cy + 3][cx + 3] + dt * L);
            if (a.a0 != 0.0f) o = a.a0 * a.q0[idx + v * plane] + o;
            a.out[idx + v * plane] = o;
            qn[v] = o;
        }
        bool ok = qn[0] > 0.0f && __builtin_isfinite(qn[0]) && __builtin_isfinite(qn[1]) && __builtin_isfinite(qn[2]);
        bad = bad || !ok;
    }
    if (count && nfb) atomicAdd(&s_cnt, nfb);
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0) {
        if (MODE == 0 && s_cnt) atomicAdd(&a.nfb[b], (unsigned long long)s_cnt);
        if (s_bad) {
            if (MODE == 0) atomicOr(&a.bad[b], a.flagbit);
            else atomicExch(&a.fatal[b], 1);
        }
    }
}

template <int MODE, int FLUX, bool AL = false, bool DIR = false, bool BL = false>
__global__ __launch_bounds__(256) void learned_stage_kernel(LearnedArgs a)
{
    learned_tile<MODE, FLUX, AL, DIR, BL>(a, blockIdx.z, blockIdx.x * LTILE_X, blockIdx.y * LTILE_Y,
                                      blockIdx.x == 0 && blockIdx.y == 0);
}

// Work-list form over a table of solves of any size (serving, and single
// solves as a batch of one): workgroup w finds its solve by binary search
// over the items' first stage tile.  MODE 0 with STAGE 1 or 2 (the learned
// stage after a separate network pass that wrote alpha to z), MODE 2 and 3
// (the end of a learned step: commit or plain stage 1; plain stage 2 and
// bookkeeping).  ntiles == 0: the tile count is read from the list header (nitems[2]; graph
// replay).
template <int MODE, int STAGE>
__global__ __launch_bounds__(256) void learned_batch_kernel(const LSolve *__restrict__ tab,
                                                            const LItem *__restrict__ items,
                                                            const int *__restrict__ nitems, int ntiles, int one,
                                                            Proj pr)
{
    const int w = blockIdx.x;
    if (w >= (ntiles > 0 ? ntiles : nitems[2])) return;
    LItem it;
    if (one) {
        it = items[0];
    } else {
        const int n = *nitems;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].tb_st <= w) lo = mid;
            else hi = mid - 1;
        }
        it = items[lo];
    }
    const LSolve &d = tab[it.solve];
    LearnedArgs a;
    a.B = 1;
    a.nx = d.nx;
    a.ny = d.ny;
    a.rdx = d.rdx;
    a.rdy = d.rdy;
    a.ph.g = d.g;
    a.ph.sqg = d.sqg;
    a.ph.gamma = 1.4f;
    a.ph.h0 = d.h0;
    a.z = d.z;
    a.dt = d.dt;
    a.bad = d.flags + it.parity;
    a.bad_next = d.flags + (it.parity ^ 1);
    a.flagbit = STAGE;
    a.nfb = d.nfb;
    a.fatal = d.fatal;
    a.redone = d.redone;
    a.t = d.t;
    a.steps = d.steps;
    a.pr = pr;
    a.commit_src = d.s2;
    a.commit_dst = d.q;
    if (MODE == 0 && STAGE == 2) {
        a.qs = d.s1; a.q0 = d.q; a.out = d.s2; a.a0 = 0.5f; a.a1 = 0.5f;
    } else if (MODE == 3) {
        a.qs = d.s1; a.q0 = d.q; a.out = d.q; a.a0 = 0.5f; a.a1 = 0.5f;
    } else {  // MODE 0 stage 1, MODE 2: q -> S1
        a.qs = d.q; a.q0 = d.q; a.out = d.s1; a.a0 = 0.0f; a.a1 = 1.0f;
    }
    const int tile = w - it.tb_st;
    const int tiles_x = (d.nx + LTILE_X - 1) / LTILE_X;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    learned_tile<MODE, fvk::HLLE, true>(a, 0, tx * LTILE_X, ty * LTILE_Y, tile == 0);
}

static hipError_t learned_batch_go(int mode, int stage, dim3 g, const LSolve *tab, const LItem *items,
                                   const int *nitems, int ntiles, int one, const Proj &pr, hipStream_t st)
{
    const dim3 b(256);
    if (mode == 0 && stage == 1) hipLaunchKernelGGL((learned_batch_kernel<0, 1>), g, b, 0, st, tab, items, nitems, ntiles, one, pr);
    else if (mode == 0 && stage == 2) hipLaunchKernelGGL((learned_batch_kernel<0, 2>), g, b, 0, st, tab, items, nitems, ntiles, one, pr);
    else if (mode == 2) hipLaunchKernelGGL((learned_batch_kernel<2, 0>), g, b, 0, st, tab, items, nitems, ntiles, one, pr);
    else if (mode == 3) hipLaunchKernelGGL((learned_batch_kernel<3, 0>), g, b, 0, st, tab, items, nitems, ntiles, one, pr);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_learned_batch(int mode, int stage, const LSolve *tab, const LItem *items, const int *nitems,
                                int ntiles, const Proj &pr, hipStream_t st, int one)
{
    if (ntiles <= 0) return hipSuccess;
    return learned_batch_go(mode, stage, dim3(ntiles), tab, items, nitems, ntiles, one, pr, st);
}

hipError_t launch_learned_batch_list(int mode, int stage, const LSolve *tab, const LItem *items, const int *list,
                                     int wgs, const Proj &pr, hipStream_t st)
{
    if (wgs <= 0) return hipErrorInvalidValue;
    return learned_batch_go(mode, stage, dim3(wgs), tab, items, list, 0, 0, pr, st);
}

// q[b] <- S2[b] for the solves whose learned step was admissible.
__global__ void commit_kernel(float *q, const float *s2, const int *bad, size_t per_solve, int B)
{
    size_t n = per_solve * B;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        int b = (int)(i / per_solve);
        if (!bad[b]) q[i] = s2[i];
    }
}

// End of step: count redone steps (and record which solves were redone),
// clear the per-step flags, advance time.
__global__ void finish_kernel(int *bad, unsigned long long *redone, int *record, int B, const float *dt, double *t,
                              long long *steps)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) {
        if (bad[b] && redone) redone[b] += 1;
        if (record) record[b] = bad[b] != 0;
        bad[b] = 0;
    }
    if (b == 0 && t) {
        *t += (double)dt[0];
        *steps += 1;
    }
}

hipError_t learned_stage(int mode, int flux, const StageBatch &sb, hipStream_t st)
{
    LearnedArgs a;
    a.qs = sb.qs;
    a.q0 = sb.q0;
    a.out = sb.out;
    a.z = sb.z;
    a.B = sb.B;
    a.nx = sb.nx;
    a.ny = sb.ny;
    a.rdx = sb.rdx;
    a.rdy = sb.rdy;
    a.ph.g = sb.g;
    a.ph.sqg = __builtin_sqrtf(sb.g);
    a.ph.gamma = 1.4f;
    a.ph.h0 = sb.h0;
    a.a0 = sb.a0;
    a.a1 = sb.a1;
    a.dt = sb.dt;
    a.bad = sb.bad;
    a.flagbit = sb.flagbit;
    a.nfb = sb.nfb;
    a.fatal = sb.fatal;
    a.pr = sb.pr;
    a.commit_src = sb.commit_src;
    a.commit_dst = sb.commit_dst;
    a.bad_next = sb.bad_next;
    a.redone = sb.redone;
    a.t = sb.t;
    a.steps = sb.steps;
    for (int v = 0; v < 3; v++) a.sig[v] = sb.sig[v];
    if ((mode == 2 && a.commit_src && !a.commit_dst) || (mode == 3 && !a.bad_next)) return hipErrorInvalidValue;
    if ((sb.direct || sb.blend) && (mode != 0 || sb.alpha)) return hipErrorInvalidValue;
    if (sb.direct && sb.blend) return hipErrorInvalidValue;
    dim3 grid((a.nx + LTILE_X - 1) / LTILE_X, (a.ny + LTILE_Y - 1) / LTILE_Y, a.B), blk(256);
    const bool rus = flux == fvk::RUSANOV;
    switch (mode) {
    case 0:
        if (sb.direct) {
            if (rus) hipLaunchKernelGGL((learned_stage_kernel<0, fvk::RUSANOV, false, true>), grid, blk, 0, st, a);
            else hipLaunchKernelGGL((learned_stage_kernel<0, fvk::HLLE, false, true>), grid, blk, 0, st, a);
        } else if (sb.blend) {
            if (rus) hipLaunchKernelGGL((learned_stage_kernel<0, fvk::RUSANOV, false, false, true>), grid, blk, 0, st, a);
            else hipLaunchKernelGGL((learned_stage_kernel<0, fvk::HLLE, false, false, true>), grid, blk, 0, st, a);
        } else if (sb.alpha) {
            if (rus) hipLaunchKernelGGL((learned_stage_kernel<0, fvk::RUSANOV, true>), grid, blk, 0, st, a);
            else hipLaunchKernelGGL((learned_stage_kernel<0, fvk::HLLE, true>), grid, blk, 0, st, a);
        } else {
            if (rus) hipLaunchKernelGGL((learned_stage_kernel<0, fvk::RUSANOV>), grid, blk, 0, st, a);
            else hipLaunchKernelGGL((learned_stage_kernel<0, fvk::HLLE>), grid, blk, 0, st, a);
        }
        break;
    case 1:
        if (rus) hipLaunchKernelGGL((learned_stage_kernel<1, fvk::RUSANOV>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((learned_stage_kernel<1, fvk::HLLE>), grid, blk, 0, st, a);
        break;
    case 2:
        if (rus) hipLaunchKernelGGL((learned_stage_kernel<2, fvk::RUSANOV>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((learned_stage_kernel<2, fvk::HLLE>), grid, blk, 0, st, a);
        break;
    case 3:
        if (rus) hipLaunchKernelGGL((learned_stage_kernel<3, fvk::RUSANOV>), grid, blk, 0, st, a);
        else hipLaunchKernelGGL((learned_stage_kernel<3, fvk::HLLE>), grid, blk, 0, st, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_commit(float *q, const float *s2, const int *bad, size_t per_solve, int B, hipStream_t st)
{
    size_t n = per_solve * B;
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(commit_kernel, dim3(blocks), dim3(256), 0, st, q, s2, bad, per_solve, B);
    return hipGetLastError();
}

hipError_t launch_finish(int *bad, unsigned long long *redone, int *record, int B, const float *dt, double *t,
                         long long *steps, hipStream_t st)
{
    hipLaunchKernelGGL(finish_kernel, dim3((B + 255) / 256), dim3(256), 0, st, bad, redone, record, B, dt, t, steps);
    return hipGetLastError();
}

Proj make_projection(int order)
{
    // moment matrix A (order+1) x 6: cell averages of x^p over unit cells
    // centred at -2.5 .. 2.5 (the six cells around the face)
    const int m = order + 1;
    double A[3][6];
    for (int p = 0; p < m; p++)
        for (int k = 0; k < 6; k++) {
            double xc = -2.5 + k;
            A[p][k] = (__builtin_pow(xc + 0.5, p + 1) - __builtin_pow(xc - 0.5, p + 1)) / (p + 1);
        }
    // X = (A A^T)^-1 A by Gauss-Jordan on [A A^T | A]
    double M[3][9];
    for (int i = 0; i < m; i++) {
        for (int j = 0; j < m; j++) {
            double s = 0;
            for (int k = 0; k < 6; k++) s += A[i][k] * A[j][k];
            M[i][j] = s;
        }
        for (int k = 0; k < 6; k++) M[i][m + k] = A[i][k];
    }
    for (int c = 0; c < m; c++) {
        int piv = c;
        for (int r = c + 1; r < m; r++)
            if (__builtin_fabs(M[r][c]) > __builtin_fabs(M[piv][c])) piv = r;
        for (int j = 0; j < m + 6; j++) {
            double t = M[c][j];
            M[c][j] = M[piv][j];
            M[piv][j] = t;
        }
        double d = M[c][c];
        for (int j = 0; j < m + 6; j++) M[c][j] /= d;
        for (int r = 0; r < m; r++)
            if (r != c) {
                double f = M[r][c];
                for (int j = 0; j < m + 6; j++) M[r][j] -= f * M[c][j];
            }
    }
    Proj pr;
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int p = 0; p < m; p++) s -= A[p][i] * M[p][m + j];
            pr.P[i * 6 + j] = (float)s;
        }
    const float fromm[12] = {0.f, -0.25f, 1.f, 0.25f, 0.f, 0.f, 0.f, 0.f, 0.25f, 1.f, -0.25f, 0.f};
    for (int i = 0; i < 12; i++) pr.base[i] = fromm[i];
    return pr;
}

}  // namespace cnn
