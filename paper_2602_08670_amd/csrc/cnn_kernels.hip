// Stencil-coefficient network on MFMA (gfx950): 3x3 convolutions as implicit
// GEMMs on v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation.
//
// One wave64 computes 16 consecutive pixels of one row x all output
// channels.  The MFMA product is D(co, pixel) = W(co, k) * X(k, pixel): the
// A operand is a 16-channel slice of the packed weights (staged in LDS), the
// B operand holds 8 consecutive input channels of one pixel per lane -- one
// 16-byte load from the NHWC activations -- and each lane's accumulators are
// four consecutive output channels of one pixel, stored as 8 bytes (BF16) or
// 16 bytes (FP32).  K runs over the 9 taps x 32 input channels.  Lane mapping
// of the 16x16x32 MFMA: A row / B column / D column = lane % 16; D rows
// 4*(lane/16) .. +3; lane group lane/16 carries the same 8 K indices in A
// and B.
#include "cnn_internal.hpp"
#include "learned_device.hpp"
#include "euler_learned_device.hpp"
#include "euler_learned_internal.hpp"

namespace cnn {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

static const int L_CI[NL] = {3, 32, 32, 32, 32};
static const int L_CO[NL] = {32, 32, 32, 32, 72};

MasterLayout master_layout()
{
    MasterLayout m;
    int off = 0;
    for (int l = 0; l < NL; l++) {
        m.w[l] = off;
        off += L_CO[l] * L_CI[l] * 9;
        m.b[l] = off;
        off += L_CO[l];
    }
    return m;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

Packed packed_layout()
{
    Packed p;
    size_t off = 0;
    p.w[0] = off;
    off = al256(off + 32 * 32 * 2);
    for (int l = 1; l < 4; l++) {
        p.w[l] = off;
        off = al256(off + 9 * 32 * 32 * 2);
    }
    p.w[4] = off;
    off = al256(off + 9 * 80 * 32 * 2);
    p.wt[0] = off;  // [9][16 ci (3 used)][32 co]
    off = al256(off + 9 * 16 * 32 * 2);
    for (int l = 1; l < 4; l++) {
        p.wt[l] = off;  // [9][32 ci][32 co]
        off = al256(off + 9 * 32 * 32 * 2);
    }
    p.wt[4] = off;  // [9][32 ci][96 co (72 used)]
    off = al256(off + 9 * 32 * 96 * 2);
    for (int l = 0; l < NL; l++) {
        p.b[l] = off;
        off = al256(off + (l == 4 ? 80 : 32) * 4);
    }
    p.bytes = off;
    return p;
}

// ------------------------------------------------------------------ packing
struct PackArgs {
    MasterLayout m;
    Packed p;
};

// Sections of the packed buffer, in element counts.
__device__ __forceinline__ void pack_one(const float *M, char *P, const PackArgs &a, int e)
{
    const int n0 = 32 * 32, n1 = 9 * 32 * 32, n4 = 9 * 80 * 32, t0 = 9 * 16 * 32, t4 = 9 * 32 * 96;
    const int sizes[10] = {n0, n1, n1, n1, n4, t0, n1, n1, n1, t4};
    int s = 0;
    while (s < 10 && e >= sizes[s]) {
        e -= sizes[s];
        s++;
    }
    if (s >= 10) {  // biases: 4 x 32 then 80
        int l = e / 32;
        if (l > 4) l = 4;
        int co = e - l * 32;
        float v = 0.0f;
        int nco = L_CO[l];
        if (co < nco) v = M[a.m.b[l] + co];
        if (l < 4 || co < 80) ((float *)(P + a.p.b[l]))[co] = v;
        return;
    }
    float v = 0.0f;
    bf16 *dst;
    if (s == 0) {  // [co][k], k = tap*3 + ci
        int co = e / 32, k = e % 32;
        if (k < 27) v = M[a.m.w[0] + (co * 3 + k % 3) * 9 + k / 3];
        dst = (bf16 *)(P + a.p.w[0]);
    } else if (s <= 3) {  // [tap][co][ci]
        int tap = e / 1024, co = (e / 32) % 32, ci = e % 32;
        v = M[a.m.w[s] + (co * 32 + ci) * 9 + tap];
        dst = (bf16 *)(P + a.p.w[s]);
    } else if (s == 4) {  // [tap][co 80][ci]
        int tap = e / 2560, co = (e / 32) % 80, ci = e % 32;
        if (co < 72) v = M[a.m.w[4] + (co * 32 + ci) * 9 + tap];
        dst = (bf16 *)(P + a.p.w[4]);
    } else if (s == 5) {  // [tap][ci 16][co 32], flipped
        int tap = e / 512, ci = (e / 32) % 16, co = e % 32;
        if (ci < 3) v = M[a.m.w[0] + (co * 3 + ci) * 9 + (8 - tap)];
        dst = (bf16 *)(P + a.p.wt[0]);
    } else if (s <= 8) {  // [tap][ci][co], flipped
        int l = s - 5;
        int tap = e / 1024, ci = (e / 32) % 32, co = e % 32;
        v = M[a.m.w[l] + (co * 32 + ci) * 9 + (8 - tap)];
        dst = (bf16 *)(P + a.p.wt[l]);
    } else {  // [tap][ci][co 96], flipped
        int tap = e / 3072, ci = (e / 96) % 32, co = e % 96;
        if (co < 72) v = M[a.m.w[4] + (co * 32 + ci) * 9 + (8 - tap)];
        dst = (bf16 *)(P + a.p.wt[4]);
    }
    dst[e] = (bf16)v;
}

__global__ void pack_kernel(const float *M, char *P, PackArgs a, int total)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) pack_one(M, P, a, e);
}

hipError_t launch_pack(const float *master, void *packed, hipStream_t st)
{
    PackArgs a{master_layout(), packed_layout()};
    int total = 32 * 32 + 3 * 9 * 32 * 32 + 9 * 80 * 32 + 9 * 16 * 32 + 3 * 9 * 32 * 32 + 9 * 32 * 96 + 4 * 32 + 80;
    hipLaunchKernelGGL(pack_kernel, dim3((total + 255) / 256), dim3(256), 0, st, master, (char *)packed, a, total);
    return hipGetLastError();
}

// ----------------------------------------------------------------- forward
__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Workgroup barrier after every global load of this wave (loads straight
// into LDS, global_load_lds, included: the compiler's waits do not track
// those) and its LDS accesses are done.
__device__ __forceinline__ void barrier_after_weights()
{
    __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Constrained coefficients of one group of six (side 0: left state, 1: right
// state), in place: alpha_k = base_k + sum_j P[k][j] z_j.
__device__ __forceinline__ void alpha_group(float *zz, int side, const Proj &pr)
{
    float zv[6], al[6];
#pragma unroll
    for (int j = 0; j < 6; j++) zv[j] = zz[j];
#pragma unroll
    for (int k = 0; k < 6; k++) {
        al[k] = pr.base[side * 6 + k];
#pragma unroll
        for (int j = 0; j < 6; j++) al[k] += pr.P[k * 6 + j] * zv[j];
    }
#pragma unroll
    for (int k = 0; k < 6; k++) zz[k] = al[k];
}

constexpr int HT = 16;  // width of the layer-by-layer pass's tiles

// First layer on a 16-pixel-wide, 4R-row tile (columns x0 .. x0+15, rows
// y0 .. y0+4R-1 of an H x W solve): the normalised, BF16-rounded input of the
// tile's halo is staged in LDS once ([3][4R + 2][18]), then lane (g, px) of
// wave w builds its K = 27 operand from LDS for rows Rw .. Rw+R-1 and
// stores act[(y * W + x) * 32 ..].  Input = states (FP32 planar [3][H][W])
// normalised per channel and rounded to BF16, K = 27 (tap*3 + ci) padded to
// 32; bias, ReLU, BF16 out.  Rows past H are not stored.
template <int R>
__device__ __forceinline__ void first_layer_tile(const float *qb, int H, int W, int x0, int y0, bf16x8 *s_w,
                                                 bf16 *s_q, const float *bias, const Norm &nrm, bf16 *act)
{
    constexpr int HR = 4 * R + 2, HC = HT + 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, px = lane & 15;
    const int hw = H * W;
    for (int i = tid; i < 3 * HR * HC; i += 256) {
        const int ci = i / (HR * HC), r = i - ci * (HR * HC);
        const int hr = r / HC, hc = r - hr * HC;
        int yy = y0 - 1 + hr;
        yy = yy < 0 ? yy + H : yy % H;
        const int xx = wrap(x0 - 1 + hc, W);
        s_q[i] = (bf16)((qb[(size_t)ci * hw + yy * W + xx] - nrm.mean[ci]) * nrm.inv_std[ci]);
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        const int ry = wave * R + rr, y = y0 + ry;
        bf16x8 bx;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int k = 8 * g + e;
            bf16 v = (bf16)0.0f;
            if (k < 27) {
                const int tap = k / 3, ci = k - 3 * tap;
                v = s_q[(ci * HR + ry + tap / 3) * HC + px + tap % 3];
            }
            bx[e] = v;
        }
        if (y >= H) continue;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[(t * 16 + px) * 4 + g], bx,
                                                                        floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            const int co0 = 16 * t + 4 * g;
            bf16x4 o;
#pragma unroll
            for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[i] + bias[co0 + i], 0.0f);
            *(bf16x4 *)(act + ((size_t)y * W + x0 + px) * 32 + co0) = o;
        }
    }
}

// First layer of B solves on 16-pixel-wide, 4R-row tiles (grid: tile
// columns, tile rows, solves); BF16 NHWC out [p][32].
template <int R>
__global__ __launch_bounds__(256) void conv_first_kernel(const float *q, const bf16 *wp, const float *bias, bf16 *out,
                                                         int H, int W, Norm nrm)
{
    __shared__ bf16x8 s_w[32 * 32 / 8];
    __shared__ bf16 s_q[3 * (4 * R + 2) * (HT + 2)];
    const bf16x8 *gw = (const bf16x8 *)wp;
    for (int i = threadIdx.x; i < 32 * 32 / 8; i += 256) s_w[i] = gw[i];
    const int b = blockIdx.z;
    const size_t hw = (size_t)H * W;
    first_layer_tile<R>(q + (size_t)b * 3 * hw, H, W, blockIdx.x * HT, blockIdx.y * 4 * R, s_w, s_q, bias, nrm,
                        out + (size_t)b * hw * 32);
}

// 3x3 convolution over a 16-pixel-wide, 4R-row tile of one solve per
// workgroup (K = KB*32 input channels, NT tiles of 16 output channels):
//   out[p][co] = sum_tap sum_ci Wp[tap][co][ci] in[p + d_tap][ci]
// with the packed layout [9 tap][rows][KB*32] of the forward weights or of
// the transposed, tap-flipped ones.  The workgroup stages the layer's
// weights and the 18 x (4R + 2) halo of its input tile in LDS once; wave w
// computes tile rows Rw .. Rw+R-1 (one 16-pixel MFMA column group each) and
// reuses each weight fragment for its R rows.  R = 4 where the grid still
// has many workgroups per CU, else fewer rows per workgroup keep enough
// workgroups resident to overlap staging with MFMAs.  Per output the MFMAs
// run in the order
// of the per-pixel kernels (taps 0..8, K blocks within a tap), so the results
// are the same bits.  The halo's 16-byte channel octets are XOR-swizzled by
// column so that sixteen consecutive pixels' reads of one octet hit distinct
// banks.  Rows past ny are computed from wrapped rows and not stored.
// EPI 0: forward hidden layer, + bias, ReLU, BF16 [p][32];
// EPI 1: forward last layer, + bias, FP32 [p][72] (NT = 5);
// EPI 2: input gradient of a hidden layer, times the ReLU mask of the
//        previous activation (act > 0), BF16 [p][32];
// EPI 3: forward last layer of the Euler network, + bias, FP32 [p][96]
//        (NT = 6).
template <int KB, int NT, int R>
struct HaloShape {
    static constexpr int CG = KB * 32, OCT = CG / 8;     // channels, 16-byte octets per pixel
    static constexpr int WEL = 9 * NT * 16 * CG;         // packed weights (BF16)
    static constexpr int TR = 4 * R;                     // tile rows
    static constexpr int HP = (TR + 2) * (HT + 2);       // halo pixels
    static constexpr int BYTES = WEL * 2 + HP * OCT * 16;  // LDS: weights, then the halo
};

// The convolution of one tile (columns x0 .. x0+15, rows y0 .. y0+4R-1 of an
// H x W NHWC input src with KB*32 channels) into acc: stage the weights and
// the halo into smem, then lane (g, px) of wave w accumulates output pixel
// (y0 + Rw + r, x0 + px), channels 16 t + 4 g .. +3, in acc[r][t].
template <int KB, int NT, int R>
__device__ __forceinline__ void halo_conv(const bf16 *src, const bf16 *wp, int H, int W, int x0, int y0, char *smem,
                                          floatx4 (&acc)[R][NT])
{
    using S = HaloShape<KB, NT, R>;
    constexpr int OCT = S::OCT, WEL = S::WEL, TR = S::TR, HP = S::HP, CG = S::CG;
    bf16x8 *s_w = (bf16x8 *)smem;
    bf16x8 *s_a = (bf16x8 *)(smem + WEL * 2);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, px = lane & 15;
    {
        // the weights and the halo straight from global memory into LDS
        // (global_load_lds_dwordx4: a wave's 64 lanes fill one 1 KB block,
        // lane l its octet l), waited for at the barrier below
        static_assert(WEL / 8 % 64 == 0, "whole weight blocks");
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const bf16x8 *gw = (const bf16x8 *)wp;
        for (int b = wv; b < WEL / 512; b += 4)  // wave-uniform
            __builtin_amdgcn_global_load_lds((const void *)(gw + b * 64 + lane), (void *)(s_w + b * 64), 16, 0, 0);
        for (int b = wv; b * 64 < HP * OCT; b += 4) {
            // LDS octet j of the halo holds pixel hp's octet o, o the
            // swizzled position (an involution)
            const int j = b * 64 + lane, hp = j / OCT, pos = j - hp * OCT;
            const int hr = hp / (HT + 2), hc = hp - hr * (HT + 2);
            int yy = y0 - 1 + hr;
            yy = yy < 0 ? yy + H : yy % H;
            const int xx = wrap(x0 - 1 + hc, W);
            const int o = (pos & ~3) | ((pos & 3) ^ ((hc >> 2) & 3));
            if (j < HP * OCT)
                __builtin_amdgcn_global_load_lds((const void *)(src + ((size_t)yy * W + xx) * CG + o * 8),
                                                 (void *)(s_a + b * 64), 16, 0, 0);
        }
    }
    barrier_after_weights();
    static_assert(TR == 4 * R, "tile rows");
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int t = 0; t < NT; t++) acc[r][t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        const int dy = tap / 3, dx = tap % 3;  // halo offsets (d + 1)
        const int hc = px + dx;
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            bf16x8 af[NT], bx[R];
#pragma unroll
            for (int t = 0; t < NT; t++) af[t] = s_w[((tap * NT + t) * 16 + px) * OCT + kb * 4 + g];
            const int pos = kb * 4 + (g ^ ((hc >> 2) & 3));
#pragma unroll
            for (int r = 0; r < R; r++) bx[r] = s_a[((wave * R + r + dy) * (HT + 2) + hc) * OCT + pos];
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int t = 0; t < NT; t++)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bx[r], acc[r][t], 0, 0, 0);
        }
    }
}

template <int KB, int NT, int EPI, int R>
__global__ __launch_bounds__(256) void conv_halo_kernel(const bf16 *in, const bf16 *wp, const float *bias,
                                                        const bf16 *mask, void *out, int H, int W)
{
    using S = HaloShape<KB, NT, R>;
    __shared__ __align__(16) char smem[S::BYTES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, px = lane & 15;
    const int x0 = blockIdx.x * HT, y0 = blockIdx.y * S::TR, b = blockIdx.z;
    const size_t hw = (size_t)H * W;
    floatx4 acc[R][NT];
    halo_conv<KB, NT, R>(in + (size_t)b * hw * S::CG, wp, H, W, x0, y0, smem, acc);

#pragma unroll
    for (int r = 0; r < R; r++) {
        const int y = y0 + wave * R + r;
        if (y >= H) break;
        const size_t p = (size_t)b * hw + (size_t)y * W + x0 + px;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int co0 = 16 * t + 4 * g;
            if (EPI == 0) {
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[r][t][i] + bias[co0 + i], 0.0f);
                *(bf16x4 *)((bf16 *)out + p * 32 + co0) = o;
            } else if (EPI == 1) {
                if (co0 < 72) {
                    floatx4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = acc[r][t][i] + bias[co0 + i];
                    *(floatx4 *)((float *)out + p * 72 + co0) = o;
                }
            } else if (EPI == 3) {
                floatx4 o;
#pragma unroll
                for (int i = 0; i < 4; i++) o[i] = acc[r][t][i] + bias[co0 + i];
                *(floatx4 *)((float *)out + p * E_COUT + co0) = o;
            } else {
                const bf16x4 m = *(const bf16x4 *)(mask + p * 32 + co0);
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; i++) o[i] = (bf16)((float)m[i] > 0.0f ? acc[r][t][i] : 0.0f);
                *(bf16x4 *)((bf16 *)out + p * 32 + co0) = o;
            }
        }
    }
}

// Rows per wave of the halo-tile convolutions: 4 while that leaves at least
// 2048 workgroups (eight per CU), else 2, else 1.
static int halo_rows(int B, int nx, int ny)
{
    for (int R = 4; R > 1; R /= 2)
        if ((long)B * (nx / HT) * ((ny + 4 * R - 1) / (4 * R)) >= 2048) return R;
    return 1;
}
static dim3 halo_grid(int B, int nx, int ny, int R)
{
    return dim3((unsigned)(nx / HT), (unsigned)((ny + 4 * R - 1) / (4 * R)), (unsigned)B);
}
template <int KB, int NT, int EPI>
static void launch_halo(const bf16 *in, const bf16 *wp, const float *bias, const bf16 *mask, void *out, int B, int nx,
                        int ny, hipStream_t st)
{
    const int R = halo_rows(B, nx, ny);
    const dim3 grid = halo_grid(B, nx, ny, R), blk(256);
    if (R == 4) hipLaunchKernelGGL((conv_halo_kernel<KB, NT, EPI, 4>), grid, blk, 0, st, in, wp, bias, mask, out, ny, nx);
    else if (R == 2) hipLaunchKernelGGL((conv_halo_kernel<KB, NT, EPI, 2>), grid, blk, 0, st, in, wp, bias, mask, out, ny, nx);
    else hipLaunchKernelGGL((conv_halo_kernel<KB, NT, EPI, 1>), grid, blk, 0, st, in, wp, bias, mask, out, ny, nx);
}

// ------------------------------------------- layer-by-layer work lists
// The network pass of a round's listed learned solves, one launch per layer
// on 16 x 16 tiles (nx, ny multiples of 16): workgroup w is tile w of the
// list (items' tb_h prefix, binary search).  Solve d's activations are NHWC
// [ny][nx][32] BF16 at pixel offset tb_h * 256 of two ping-pong buffers.
// Layer 0 reads q (stage 1) or S1 (stage 2); the last layer writes
// alpha = base + P z (per group of six) to d.z.  Per output the arithmetic is
// the one-launch pass's, so alpha is the same bits.  The tile count is read
// from the list header (list = {items, network tiles, stage tiles, 16 x 16
// tiles}); workgroups past it exit.
__device__ __forceinline__ LItem find_item_h(const LItem *__restrict__ items, int n, int w)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tb_h <= w) lo = mid;
        else hi = mid - 1;
    }
    return items[lo];
}

template <int STAGE>
__global__ __launch_bounds__(256) void conv_first_list_kernel(const LSolve *__restrict__ tab,
                                                              const LItem *__restrict__ items,
                                                              const int *__restrict__ list, const bf16 *wp,
                                                              const float *bias, bf16 *act, Norm nrm)
{
    const int w = blockIdx.x;
    if (w >= list[3]) return;
    __shared__ bf16x8 s_w[32 * 32 / 8];
    __shared__ bf16 s_q[3 * 18 * (HT + 2)];
    const bf16x8 *gw = (const bf16x8 *)wp;
    for (int i = threadIdx.x; i < 32 * 32 / 8; i += 256) s_w[i] = gw[i];
    const LItem it = find_item_h(items, list[0], w);
    const LSolve &d = tab[it.solve];
    const int tile = w - it.tb_h, tx_n = d.nx / HT;
    const int ty = tile / tx_n, tx = tile - ty * tx_n;
    first_layer_tile<4>(STAGE == 1 ? d.q : d.s1, d.ny, d.nx, tx * HT, ty * HT, s_w, s_q, bias, nrm,
                        act + (size_t)it.tb_h * HT * HT * 32);
}

// EPI 0: hidden layer (+ bias, ReLU, BF16 act); EPI 1: last layer (+ bias,
// then alpha through LDS, FP32 [ny][nx][72] to d.z).
template <int NT, int EPI>
__global__ __launch_bounds__(256) void conv_halo_list_kernel(const LSolve *__restrict__ tab,
                                                             const LItem *__restrict__ items,
                                                             const int *__restrict__ list, const bf16 *wp,
                                                             const float *bias, const bf16 *in, bf16 *out, Proj pr)
{
    using S = HaloShape<1, NT, 4>;
    constexpr int ZB = EPI == 1 ? HT * HT * 72 * 4 : 0;  // the tile's z for the alpha epilogue
    __shared__ __align__(16) char smem[S::BYTES > ZB ? S::BYTES : ZB];
    const int w = blockIdx.x;
    if (w >= list[3]) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, px = lane & 15;
    const LItem it = find_item_h(items, list[0], w);
    const LSolve &d = tab[it.solve];
    const int tile = w - it.tb_h, tx_n = d.nx / HT;
    const int ty = tile / tx_n, tx = tile - ty * tx_n;
    const int x0 = tx * HT, y0 = ty * HT;
    const size_t off = (size_t)it.tb_h * HT * HT;  // the solve's first pixel in the activation buffers
    floatx4 acc[4][NT];
    halo_conv<1, NT, 4>(in + off * 32, wp, d.ny, d.nx, x0, y0, smem, acc);
    if (EPI == 0) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const size_t p = off + (size_t)(y0 + wave * 4 + r) * d.nx + x0 + px;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int co0 = 16 * t + 4 * g;
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[r][t][i] + bias[co0 + i], 0.0f);
                *(bf16x4 *)(out + p * 32 + co0) = o;
            }
        }
    } else {
        float *s_z = (float *)smem;  // [256 tile pixels][72]
        __syncthreads();             // the MFMAs' LDS reads are done
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int pl = (wave * 4 + r) * HT + px;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int co0 = 16 * t + 4 * g;
                if (co0 < 72) {
                    floatx4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = acc[r][t][i] + bias[co0 + i];
                    *(floatx4 *)(s_z + pl * 72 + co0) = o;
                }
            }
        }
        __syncthreads();
        for (int task = threadIdx.x; task < HT * HT * 12; task += 256) {
            const int pl = task / 12, grp = task - pl * 12;
            alpha_group(s_z + pl * 72 + grp * 6, (grp / 3) & 1, pr);
        }
        __syncthreads();
        // each tile row's 16 x 72 values are contiguous in d.z
        constexpr int RV = HT * 72 / 4;  // float4 per tile row
        for (int i = threadIdx.x; i < HT * RV; i += 256) {
            const int row = i / RV, c = i - row * RV;
            ((float4 *)(d.z + ((size_t)(y0 + row) * d.nx + x0) * 72))[c] = ((const float4 *)(s_z + row * HT * 72))[c];
        }
    }
}

hipError_t launch_layer_list(int layer, int stage, const void *packed, const Norm &nrm, const Proj &pr,
                             const LSolve *tab, const LItem *items, const int *list, int wgs, void *act0, void *act1,
                             hipStream_t st)
{
    const Packed pk = packed_layout();
    const char *P = (const char *)packed;
    const dim3 grid((unsigned)(wgs > 0 ? wgs : 1)), blk(256);
    bf16 *a[2] = {(bf16 *)act0, (bf16 *)act1};
    const bf16 *w = (const bf16 *)(P + pk.w[layer]);
    const float *b = (const float *)(P + pk.b[layer]);
    if (layer == 0) {
        if (stage == 1) hipLaunchKernelGGL(conv_first_list_kernel<1>, grid, blk, 0, st, tab, items, list, w, b, a[0], nrm);
        else hipLaunchKernelGGL(conv_first_list_kernel<2>, grid, blk, 0, st, tab, items, list, w, b, a[0], nrm);
    } else if (layer < 4) {
        hipLaunchKernelGGL((conv_halo_list_kernel<2, 0>), grid, blk, 0, st, tab, items, list, w, b,
                           (const bf16 *)a[(layer - 1) & 1], a[layer & 1], pr);
    } else {
        hipLaunchKernelGGL((conv_halo_list_kernel<5, 1>), grid, blk, 0, st, tab, items, list, w, b,
                           (const bf16 *)a[1], (bf16 *)nullptr, pr);
    }
    return hipGetLastError();
}

hipError_t launch_forward(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny,
                          void *const acts[4], float *z, hipStream_t st)
{
    const Packed pk = packed_layout();
    const char *P = (const char *)packed;
    if (nx % HT) return hipErrorInvalidValue;
    const dim3 blk(256);
    {
        const int R = halo_rows(B, nx, ny);
        const dim3 fg = halo_grid(B, nx, ny, R);
        const bf16 *w0 = (const bf16 *)(P + pk.w[0]);
        const float *b0 = (const float *)(P + pk.b[0]);
        if (R == 4) hipLaunchKernelGGL(conv_first_kernel<4>, fg, blk, 0, st, q, w0, b0, (bf16 *)acts[0], ny, nx, nrm);
        else if (R == 2) hipLaunchKernelGGL(conv_first_kernel<2>, fg, blk, 0, st, q, w0, b0, (bf16 *)acts[0], ny, nx, nrm);
        else hipLaunchKernelGGL(conv_first_kernel<1>, fg, blk, 0, st, q, w0, b0, (bf16 *)acts[0], ny, nx, nrm);
    }
    for (int l = 1; l < 4; l++)
        launch_halo<1, 2, 0>((const bf16 *)acts[l - 1], (const bf16 *)(P + pk.w[l]), (const float *)(P + pk.b[l]),
                             nullptr, acts[l], B, nx, ny, st);
    launch_halo<1, 5, 1>((const bf16 *)acts[3], (const bf16 *)(P + pk.w[4]), (const float *)(P + pk.b[4]), nullptr,
                         (void *)z, B, nx, ny, st);
    return hipGetLastError();
}

// ---------------------------------------------------- Euler network pass
EPacked euler_packed_layout()
{
    EPacked p;
    size_t off = 0;
    p.w[0] = off;
    off = al256(off + 32 * 64 * 2);
    for (int l = 1; l < 4; l++) {
        p.w[l] = off;
        off = al256(off + 9 * 32 * 32 * 2);
    }
    p.w[4] = off;
    off = al256(off + 9 * E_COUT * 32 * 2);
    p.wt[0] = off;  // [9][16 ci (4 used)][32 co]
    off = al256(off + 9 * 16 * 32 * 2);
    for (int l = 1; l < 4; l++) {
        p.wt[l] = off;  // [9][32 ci][32 co]
        off = al256(off + 9 * 32 * 32 * 2);
    }
    p.wt[4] = off;  // [9][32 ci][96 co]
    off = al256(off + 9 * 32 * E_COUT * 2);
    for (int l = 0; l < NL; l++) {
        p.b[l] = off;
        off = al256(off + (l == 4 ? E_COUT : 32) * 4);
    }
    p.bytes = off;
    return p;
}

// Master offsets of the Euler network (W_l then b_l).
struct EMaster {
    int w[NL], b[NL];
};
static EMaster euler_master()
{
    static const int ci[NL] = {E_CIN, 32, 32, 32, 32}, co[NL] = {32, 32, 32, 32, E_COUT};
    EMaster m;
    int off = 0;
    for (int l = 0; l < NL; l++) {
        m.w[l] = off;
        off += co[l] * ci[l] * 9;
        m.b[l] = off;
        off += co[l];
    }
    return m;
}

// Element e of the packed buffer's sections: layer 0 [32][64], layers 1-3
// [9][32][32], layer 4 [9][96][32], the transposed tap-flipped copies
// (layer 0 [9][16][32], layers 1-3 [9][32][32], layer 4 [9][32][96]), then
// the biases 4 x 32 + 96.
__global__ void pack_euler_kernel(const float *M, char *P, EPacked p, EMaster m, int total)
{
    constexpr int n0 = 32 * 64, n1 = 9 * 32 * 32, n4 = 9 * E_COUT * 32, t0 = 9 * 16 * 32;
    for (int e0 = blockIdx.x * blockDim.x + threadIdx.x; e0 < total; e0 += gridDim.x * blockDim.x) {
        int e = e0;
        if (e >= n0 + 3 * n1 + n4 && e < n0 + 3 * n1 + n4 + t0 + 3 * n1 + n4) {
            int r = e - (n0 + 3 * n1 + n4);
            if (r < t0) {  // W'[t][ci][co] = W[co][ci][8 - t], ci < 4
                const int tap = r / 512, ci = (r / 32) % 16, co = r % 32;
                const float v = ci < E_CIN ? M[m.w[0] + (co * E_CIN + ci) * 9 + (8 - tap)] : 0.0f;
                ((bf16 *)(P + p.wt[0]))[r] = (bf16)v;
                continue;
            }
            r -= t0;
            if (r < 3 * n1) {
                const int l = 1 + r / n1, rr = r % n1;
                const int tap = rr / 1024, ci = (rr / 32) % 32, co = rr % 32;
                ((bf16 *)(P + p.wt[l]))[rr] = (bf16)M[m.w[l] + (co * 32 + ci) * 9 + (8 - tap)];
                continue;
            }
            r -= 3 * n1;
            const int tap = r / (32 * E_COUT), ci = (r / E_COUT) % 32, co = r % E_COUT;
            ((bf16 *)(P + p.wt[4]))[r] = (bf16)M[m.w[4] + (co * 32 + ci) * 9 + (8 - tap)];
            continue;
        }
        if (e >= n0 + 3 * n1 + n4) e -= t0 + 3 * n1 + n4;  // past the transposed copies: the biases
        if (e < n0) {
            const int co = e / 64, k = e % 64;
            float v = 0.0f;
            if (k < 9 * E_CIN) v = M[m.w[0] + (co * E_CIN + k % E_CIN) * 9 + k / E_CIN];
            ((bf16 *)(P + p.w[0]))[e] = (bf16)v;
            continue;
        }
        e -= n0;
        if (e < 3 * n1) {
            const int l = 1 + e / n1, r = e % n1;
            const int tap = r / 1024, co = (r / 32) % 32, ci = r % 32;
            ((bf16 *)(P + p.w[l]))[r] = (bf16)M[m.w[l] + (co * 32 + ci) * 9 + tap];
            continue;
        }
        e -= 3 * n1;
        if (e < n4) {
            const int tap = e / (E_COUT * 32), co = (e / 32) % E_COUT, ci = e % 32;
            ((bf16 *)(P + p.w[4]))[e] = (bf16)M[m.w[4] + (co * 32 + ci) * 9 + tap];
            continue;
        }
        e -= n4;
        const int l = e < 128 ? e / 32 : 4, co = e < 128 ? e % 32 : e - 128;
        ((float *)(P + p.b[l]))[co] = M[m.b[l] + co];
    }
}

hipError_t launch_pack_euler(const float *master, void *packed, hipStream_t st)
{
    const int total = 32 * 64 + 3 * 9 * 32 * 32 + 9 * E_COUT * 32 + (9 * 16 * 32 + 3 * 9 * 32 * 32 + 9 * 32 * E_COUT) +
                      4 * 32 + E_COUT;
    hipLaunchKernelGGL(pack_euler_kernel, dim3((total + 255) / 256), dim3(256), 0, st, master, (char *)packed,
                       euler_packed_layout(), euler_master(), total);
    return hipGetLastError();
}

// First layer of the Euler network on 16-pixel-wide, 4R-row tiles: the
// normalised, BF16-rounded input halo ([4][4R + 2][18]) staged in LDS once,
// K = 36 (tap*4 + ci) padded to two 32-wide K blocks, accumulated in K
// order; bias, ReLU, BF16 NHWC out [p][32].
template <int R>
__global__ __launch_bounds__(256) void conv_first_euler_kernel(const float *q, const bf16 *wp, const float *bias,
                                                               bf16 *out, int H, int W, ENorm nrm)
{
    constexpr int HR = 4 * R + 2, HC = HT + 2;
    __shared__ bf16x8 s_w[32 * 64 / 8];
    __shared__ bf16 s_q[E_CIN * HR * HC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, px = lane & 15;
    const int b = blockIdx.z, x0 = blockIdx.x * HT, y0 = blockIdx.y * 4 * R;
    const int hw = H * W;
    const float *qb = q + (size_t)b * E_CIN * hw;
    bf16 *act = out + (size_t)b * hw * 32;
    const bf16x8 *gw = (const bf16x8 *)wp;
    for (int i = tid; i < 32 * 64 / 8; i += 256) s_w[i] = gw[i];
    for (int i = tid; i < E_CIN * HR * HC; i += 256) {
        const int ci = i / (HR * HC), r = i - ci * (HR * HC);
        const int hr = r / HC, hc = r - hr * HC;
        int yy = y0 - 1 + hr;
        yy = yy < 0 ? yy + H : yy % H;
        const int xx = wrap(x0 - 1 + hc, W);
        s_q[i] = (bf16)((qb[(size_t)ci * hw + yy * W + xx] - nrm.mean[ci]) * nrm.inv_std[ci]);
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < R; rr++) {
        const int ry = wave * R + rr, y = y0 + ry;
        bf16x8 bx[2];
#pragma unroll
        for (int kb = 0; kb < 2; kb++)
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int k = 32 * kb + 8 * g + e;
                bf16 v = (bf16)0.0f;
                if (k < 9 * E_CIN) {
                    const int tap = k / E_CIN, ci = k - E_CIN * tap;
                    v = s_q[(ci * HR + ry + tap / 3) * HC + px + tap % 3];
                }
                bx[kb][e] = v;
            }
        if (y >= H) continue;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; kb++)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[(t * 16 + px) * 8 + kb * 4 + g], bx[kb], acc, 0, 0, 0);
            const int co0 = 16 * t + 4 * g;
            bf16x4 o;
#pragma unroll
            for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[i] + bias[co0 + i], 0.0f);
            *(bf16x4 *)(act + ((size_t)y * W + x0 + px) * 32 + co0) = o;
        }
    }
}

hipError_t launch_forward_euler_keep(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                     void *const acts[4], float *z, hipStream_t st)
{
    const EPacked pk = euler_packed_layout();
    const char *P = (const char *)packed;
    if (nx % HT) return hipErrorInvalidValue;
    const int R = halo_rows(B, nx, ny);
    const dim3 fg = halo_grid(B, nx, ny, R), blk(256);
    const bf16 *w0 = (const bf16 *)(P + pk.w[0]);
    const float *b0 = (const float *)(P + pk.b[0]);
    bf16 *a0 = (bf16 *)acts[0];
    if (R == 4) hipLaunchKernelGGL(conv_first_euler_kernel<4>, fg, blk, 0, st, q, w0, b0, a0, ny, nx, nrm);
    else if (R == 2) hipLaunchKernelGGL(conv_first_euler_kernel<2>, fg, blk, 0, st, q, w0, b0, a0, ny, nx, nrm);
    else hipLaunchKernelGGL(conv_first_euler_kernel<1>, fg, blk, 0, st, q, w0, b0, a0, ny, nx, nrm);
    for (int l = 1; l < 4; l++)
        launch_halo<1, 2, 0>((const bf16 *)acts[l - 1], (const bf16 *)(P + pk.w[l]), (const float *)(P + pk.b[l]),
                             nullptr, acts[l], B, nx, ny, st);
    launch_halo<1, 6, 3>((const bf16 *)acts[3], (const bf16 *)(P + pk.w[4]), (const float *)(P + pk.b[4]), nullptr,
                         (void *)z, B, nx, ny, st);
    return hipGetLastError();
}

hipError_t launch_forward_euler(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                void *act0, void *act1, float *z, hipStream_t st)
{
    const EPacked pk = euler_packed_layout();
    const char *P = (const char *)packed;
    if (nx % HT) return hipErrorInvalidValue;
    const int R = halo_rows(B, nx, ny);
    const dim3 fg = halo_grid(B, nx, ny, R), blk(256);
    const bf16 *w0 = (const bf16 *)(P + pk.w[0]);
    const float *b0 = (const float *)(P + pk.b[0]);
    bf16 *a0 = (bf16 *)act0, *a1 = (bf16 *)act1;
    if (R == 4) hipLaunchKernelGGL(conv_first_euler_kernel<4>, fg, blk, 0, st, q, w0, b0, a0, ny, nx, nrm);
    else if (R == 2) hipLaunchKernelGGL(conv_first_euler_kernel<2>, fg, blk, 0, st, q, w0, b0, a0, ny, nx, nrm);
    else hipLaunchKernelGGL(conv_first_euler_kernel<1>, fg, blk, 0, st, q, w0, b0, a0, ny, nx, nrm);
    bf16 *src = a0, *dst = a1;
    for (int l = 1; l < 4; l++) {
        launch_halo<1, 2, 0>(src, (const bf16 *)(P + pk.w[l]), (const float *)(P + pk.b[l]), nullptr, dst, B, nx, ny,
                             st);
        bf16 *t = src;
        src = dst;
        dst = t;
    }
    launch_halo<1, 6, 3>(src, (const bf16 *)(P + pk.w[4]), (const float *)(P + pk.b[4]), nullptr, (void *)z, B, nx,
                         ny, st);
    return hipGetLastError();
}

// ------------------------------------------------------- fused inference
// All five layers for one FT x FT tile of output pixels in one workgroup.
// Layer l's output is computed on the (FT + 2(4 - l))^2 region around the
// tile, so the next layer finds its 3x3 neighbourhood inside the block: the
// input region (FT + 10)^2 is read once with periodic wrap, activations stay
// in LDS (two ping-pong buffers), and all five layers' packed weights are
// staged into LDS together.  Each output pixel accumulates its MFMAs in
// the same order as the layer-by-layer pass (taps 0..8, K slices within a tap), with
// the same bias, ReLU and BF16 rounding, so z is bit-identical to the
// layer-by-layer pass; only the halo pixels are computed more than once.
constexpr int FT = 8;            // output tile side
static_assert(FT == LTILE_CNN, "network pass tile of the work lists");
constexpr int FW_EL = 9 * 5 * 16 * 32;  // largest packed weight block (layer 4), bf16 elements

// Hidden layer NT = 2 co tiles: each wave loads the layer's A fragments
// (9 taps x 2 tiles, 16 bytes per lane each) from LDS into registers once and
// reuses them for all its pixel groups; only B is read per group and tap.
constexpr int FNW = 8;  // waves per workgroup of the fused pass

// LDS layouts of the fused passes, chosen so that the 16 lanes of an MFMA
// operand fragment that share a K block read 16 different 16-byte bank
// groups.  Weights: the packed block's fragment of 64 octets (16 rows x 4 K
// blocks, row-major) is stored K-block-major: octet (row, g) at g * 16 +
// row.  Activations: pixel q's octet g (channels 8g .. 8g + 7) at
// q * AS + g; AS = 5 octets per pixel (an odd stride: 16 consecutive pixels
// fall in 16 different bank groups, and a tap's shift stays a constant
// offset), AS = 4 (unpadded) where LDS has no room for the padding.
__device__ __forceinline__ int wfrag(int f, int row, int g) { return (f * 4 + g) * 16 + row; }
template <int AS> __device__ __forceinline__ int act_slot(int q, int g) { return q * AS + g; }
// bf16 offset of channels co0 .. co0 + 3 (co0 % 4 == 0) of pixel q
template <int AS> __device__ __forceinline__ int act_off(int q, int co0) { return q * AS * 8 + co0; }

// NG pixel groups gi, gi + FNW, ... of a hidden layer with both co tiles:
// 2 NG accumulation chains advanced together.
template <int NG, int AS>
__device__ __forceinline__ void hidden_groups(const bf16x8 *in, int rin, bf16 *out, const bf16x8 (*A)[2],
                                              const float (*bs)[4], int gi, int rout, int npx, int g, int px)
{
    constexpr int NT = 2;
    int p[NG], qb[NG];
#pragma unroll
    for (int k = 0; k < NG; k++) {
        p[k] = (gi + k * FNW) * 16 + px;
        const int pc = p[k] < npx ? p[k] : 0;
        const int py = pc / rout, pxx = pc - py * rout;
        qb[k] = py * rin + pxx;  // the input pixel of tap 0
    }
    floatx4 acc[NG][NT];
#pragma unroll
    for (int k = 0; k < NG; k++)
#pragma unroll
        for (int t = 0; t < NT; t++) acc[k][t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        const int tq = (tap / 3) * rin + tap % 3;
#pragma unroll
        for (int k = 0; k < NG; k++) {
            const bf16x8 bx = in[act_slot<AS>(qb[k] + tq, g)];
#pragma unroll
            for (int t = 0; t < NT; t++)
                acc[k][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[tap][t], bx, acc[k][t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int k = 0; k < NG; k++) {
        if (p[k] < npx) {
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int co0 = 16 * t + 4 * g;
                bf16x4 o;
#pragma unroll
                for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[k][t][i] + bs[t][i], 0.0f);
                *(bf16x4 *)(out + act_off<AS>(p[k], co0)) = o;
            }
        }
    }
}

template <int AS>
__device__ __forceinline__ void fused_hidden(const bf16x8 *in, int rin, bf16 *out, const bf16x8 *w, const float *bias,
                                             int wave, int lane)
{
    constexpr int NT = 2;
    const int g = lane >> 4, px = lane & 15;
    const int rout = rin - 2, npx = rout * rout, ngrp = (npx + 15) >> 4;
    if (wave >= ngrp) return;  // no group for this wave: its weight reads are skipped
    bf16x8 A[9][NT];
#pragma unroll
    for (int tap = 0; tap < 9; tap++)
#pragma unroll
        for (int t = 0; t < NT; t++) A[tap][t] = w[wfrag(tap * NT + t, px, g)];
    float bs[NT][4];
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int i = 0; i < 4; i++) bs[t][i] = bias[16 * t + 4 * g + i];
    // groups gi and gi + FNW of this wave together (wave-uniform test, a
    // real branch: an MFMA does not honour a partial EXEC), their four
    // chains advanced tap by tap; each chain's taps keep their order
    for (int gi = wave; gi < ngrp; gi += 2 * FNW) {
        if (gi + FNW < ngrp) hidden_groups<2, AS>(in, rin, out, A, bs, gi, rout, npx, g, px);
        else hidden_groups<1, AS>(in, rin, out, A, bs, gi, rout, npx, g, px);
    }
}

// The last layer on few pixel groups (NG groups of 16 pixels of the FO x FO
// region, its input region FO + 2 wide in act): wave t < NT takes co tile t
// for every group, so that a wave reads one tile's 9 weight fragments and
// NT waves share the layer; each chain keeps the tap order 0..8.  acc:
// the wave's NG accumulators (zero for waves past NT).
template <int NG, int NT, int FO, int AS>
__device__ __forceinline__ void last_layer_by_tile(const bf16x8 *act, const bf16x8 *w, int wave, int g, int px,
                                                   floatx4 (&acc)[NG])
{
    constexpr int RIN = FO + 2, NPX = FO * FO;
#pragma unroll
    for (int k = 0; k < NG; k++) acc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (wave >= NT) return;  // wave-uniform: a real branch around the MFMAs
    int qb[NG];
#pragma unroll
    for (int k = 0; k < NG; k++) {
        const int p = k * 16 + px, pc = p < NPX ? p : 0;
        const int py = pc / FO, pxx = pc - py * FO;
        qb[k] = py * RIN + pxx;
    }
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        const bf16x8 a = w[wfrag(tap * NT + wave, px, g)];
        const int tq = (tap / 3) * RIN + tap % 3;
#pragma unroll
        for (int k = 0; k < NG; k++)
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[act_slot<AS>(qb[k] + tq, g)], acc[k], 0, 0, 0);
    }
}

// A layer's packed weights (NB blocks of 64 octets) straight from global
// memory into LDS, one global_load_lds_dwordx4 per 1 KB block, blocks
// wave, wave + FNW, ...: lane l of a block writes the block's octet l; with
// PERM that is octet (l & 15, l >> 4) of the packed row-major fragment
// (the K-block-major order wfrag reads), else octet l.  These writes are
// not tracked by the compiler's waits: barrier_after_weights() waits for
// them before any LDS read.
template <int NB, bool PERM = true>
__device__ __forceinline__ void dma_weights(const char *g, bf16x8 *s, int wave, int lane)
{
    for (int b = wave; b < NB; b += FNW) {  // wave-uniform
        const unsigned i = PERM ? ((unsigned)b * 64 | (unsigned)(lane & 15) << 2 | (unsigned)(lane >> 4))
                                : (unsigned)b * 64 + lane;
        __builtin_amdgcn_global_load_lds((const void *)(g + (size_t)i * 16), (void *)(s + b * 64), 16, 0, 0);
    }
}

// All five layers' biases in LDS ([4][32] hidden, then the last layer's
// NL4), so that no layer waits on a global load for them: one float per
// thread, loaded with the weights and stored with them.
template <int NL4, class PK> struct BiasChunk {
    static_assert(4 * 32 + NL4 <= FNW * 64, "one bias per thread");
    float v = 0.0f;
    __device__ __forceinline__ void load(const char *P, const PK &pk)
    {
        const int t = threadIdx.x;
        if (t < 4 * 32 + NL4) {
            const size_t off = t < 32 ? pk.b[0] : t < 64 ? pk.b[1] : t < 96 ? pk.b[2] : t < 128 ? pk.b[3] : pk.b[4];
            v = ((const float *)(P + off))[t < 128 ? (t & 31) : t - 128];
        }
    }
    __device__ __forceinline__ void store(float *s) const
    {
        if (threadIdx.x < 4 * 32 + NL4) s[threadIdx.x] = v;
    }
};

// Plain (MINMOD, HLLE) Heun step of the previous state xprev on the R x R
// region at (ox, oy), recomputed from xprev on the region grown by four
// cells (two per stage): the redo of a step whose learned result was
// inadmissible, on the region one workgroup of the next step reads, so that
// no launch has to finish the redo first.  Each face flux, cell update and
// Heun combine is the plain stage's (learned-stage kernels, MODES 2 and 3)
// arithmetic on the same stencil values.  The TS x TS tile at (x0, y0) writes
// its cells of the result to xk and raises fatal where a plain stage leaves
// one of them inadmissible.  Needs 3 ((R + 8)^2 + (R + 4)^2 + R^2) floats of
// LDS at buf; returns the region, [3][R][R], in buf.
struct PlainRedo {
    const float *xprev;  // the previous step's input [3][H][W]
    const int *flag;     // the previous step's flag slot: redo where it is set
    float *xk;           // the redone state [3][H][W]: this tile's cells written
    const float *dt;
    float rdx, rdy;
    Phys<float> ph;
    int *fatal;
};

// The stage kernels store each face flux to LDS and form the divergence from
// the stored values; a redo that uses its fluxes in registers keeps the
// compiler from fusing a flux's last operation into the divergence (an
// empty asm that may change the values), so it rounds as they do.
template <int N> __device__ __forceinline__ void flux_barrier(float *F)
{
#pragma unroll
    for (int v = 0; v < N; v++) __asm__ volatile("" : "+v"(F[v]));
}

// The four face fluxes of the cell at (r, c) of an LDS field [3][N][N]:
// left, right, bottom, top (the face between cells j and j + 1 of a line
// takes the stencil j - 2 .. j + 3, of which MINMOD reads j - 1 .. j + 2).
template <int N>
__device__ __forceinline__ void plain_cell_fluxes(const float *f, int r, int c, const Phys<float> &ph, float (*F)[3])
{
#pragma unroll
    for (int face = 0; face < 4; face++) {
        const int ax = face >> 1, lo = face & 1;  // axis, and whether the face is on the cell's high side
        float st[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            st[v][0] = 0.0f;
            st[v][5] = 0.0f;
#pragma unroll
            for (int k = 1; k < 5; k++) {
                const int o = k - 3 + lo;
                st[v][k] = ax == 0 ? f[(v * N + r) * N + c + o] : f[(v * N + r + o) * N + c];
            }
        }
        float QL[3], QR[3];
        face_states<1>(st, nullptr, Proj{}, QL, QR);
        if (ax == 0) flux3<fvk::HLLE, 0>(QL, QR, ph, F[face]);
        else flux3<fvk::HLLE, 1>(QL, QR, ph, F[face]);
        flux_barrier<3>(F[face]);
    }
}

// Out of line, its arguments in registers: the common path (no redo) keeps
// the network pass's register budget.
template <int R, int TS>
__device__ __noinline__ float *redo_region(const float *xprev, float *xk, const float *dtp, float rdx, float rdy,
                                           float g, float sqg, float h0, int *fatal, int H, int W, int ox, int oy,
                                           int x0, int y0, float *buf)
{
    constexpr int A = R + 8, S = R + 4, NT = FNW * 64;
    PlainRedo rd;
    rd.xprev = xprev;
    rd.xk = xk;
    rd.dt = dtp;
    rd.rdx = rdx;
    rd.rdy = rdy;
    rd.ph.g = g;
    rd.ph.sqg = sqg;
    rd.ph.gamma = 1.4f;
    rd.ph.h0 = h0;
    rd.fatal = fatal;
    float *sa = buf;              // [3][A][A] xprev from (ox - 4, oy - 4)
    float *ss = sa + 3 * A * A;   // [3][S][S] plain stage 1 from (ox - 2, oy - 2)
    float *sr = ss + 3 * S * S;   // [3][R][R] the redone state from (ox, oy)
    const int tid = threadIdx.x;
    const size_t plane = (size_t)H * W;
    const float dt = rd.dt[0];
    for (int k = tid; k < 3 * A * A; k += NT) {
        const int v = k / (A * A), r = k - v * A * A, ry = r / A, rx = r - ry * A;
        // up to ten cells out from a tile of a grid as small as 8 cells: the full modulo
        sa[k] = rd.xprev[v * plane + (size_t)pwrap(oy - 4 + ry, H) * W + pwrap(ox - 4 + rx, W)];
    }
    __syncthreads();
    bool bad = false;
    // stage 1: S1 = q + dt L(q); cell (j, i) of ss is (j + 2, i + 2) of sa
    for (int k = tid; k < S * S; k += NT) {
        const int j = k / S, i = k - j * S;
        float F[4][3];
        plain_cell_fluxes<A>(sa, j + 2, i + 2, rd.ph, F);
        const int gx = ox - 2 + i - x0, gy = oy - 2 + j - y0;  // tile-relative
        const bool own = gx >= 0 && gx < TS && gy >= 0 && gy < TS;
        float qn[3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            float L = -(F[1][v] - F[0][v]) * rd.rdx - (F[3][v] - F[2][v]) * rd.rdy;
            float o = 1.0f * (sa[(v * A + j + 2) * A + i + 2] + dt * L);
            ss[(v * S + j) * S + i] = o;
            qn[v] = o;
        }
        if (own) bad = bad || !(qn[0] > 0.0f && __builtin_isfinite(qn[0]) && __builtin_isfinite(qn[1]) &&
                                __builtin_isfinite(qn[2]));
    }
    __syncthreads();
    // stage 2: q/2 + (S1 + dt L(S1))/2; cell (j, i) of sr is (j + 2, i + 2) of ss
    for (int k = tid; k < R * R; k += NT) {
        const int j = k / R, i = k - j * R;
        float F[4][3];
        plain_cell_fluxes<S>(ss, j + 2, i + 2, rd.ph, F);
        const int gx = ox + i - x0, gy = oy + j - y0;
        const bool own = gx >= 0 && gx < TS && gy >= 0 && gy < TS;
        float qn[3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            float L = -(F[1][v] - F[0][v]) * rd.rdx - (F[3][v] - F[2][v]) * rd.rdy;
            float o = 0.5f * (ss[(v * S + j + 2) * S + i + 2] + dt * L);
            o = 0.5f * sa[(v * A + j + 4) * A + i + 4] + o;
            sr[(v * R + j) * R + i] = o;
            qn[v] = o;
        }
        if (own) {
#pragma unroll
            for (int v = 0; v < 3; v++) rd.xk[v * plane + (size_t)(y0 + gy) * W + x0 + gx] = qn[v];
            bad = bad || !(qn[0] > 0.0f && __builtin_isfinite(qn[0]) && __builtin_isfinite(qn[1]) &&
                           __builtin_isfinite(qn[2]));
        }
    }
    if (bad) atomicExch(rd.fatal, 1);
    __syncthreads();
    return sr;
}

// ALPHA: instead of z, write the constrained coefficients alpha = base + P z
// of every group of six (same operation order as the learned stage's own
// projection, so alpha is bit-identical to projecting this kernel's z).
// One workgroup's network pass for the FO x FO output region at (x0 - FO +
// FT, y0 - FO + FT): the FT x FT tile (FO = FT), or the tile and its low halo
// row and column (FO = FT + 1).  OUT_Z writes raw z to zb, OUT_ALPHA the
// constrained coefficients alpha = base + P z (same operation order as the
// learned stage's own projection) to zb, OUT_Z_LDS keeps z in LDS
// ([FO*FO][72], returned) and the tile's FP32 stage input with a 3-cell halo
// in qf for a learned stage in the same workgroup, which projects each face's
// coefficients itself (each group of six serves exactly one face).  load_w: stage the
// weights (a workgroup's first tile; its later tiles find them in LDS).
enum { OUT_Z = 0, OUT_ALPHA = 1, OUT_Z_LDS = 2 };
// rd (OUT_Z_LDS only, or NULL): when rd->xprev is set and *rd->flag is not
// zero, the input region is the plain redo of the previous step
// (redo_region) instead of qb.  LO: cells of the output region before the
// tile (FO - FT by default; 1 for the tile and a one-cell ring, FO = FT + 2).
// TS: the tile side (FT; a single solve's kernel on few tiles takes 4, the
// same per-pixel arithmetic on more, smaller workgroups).
template <int FO, int OUT, int LO = FO - FT, int TS = FT>
__device__ __forceinline__ float *fused_tile(const float *qb, const char *P, const Packed &pk, const Norm &nrm, float *zb,
                                             int H, int W, int y0, int x0, const Proj &pr, bool load_w, float *qf,
                                             const PlainRedo *rd = nullptr);

// Workgroups stride over the B x (H/FT) x (W/FT) tiles: a grid of at most the
// workgroups resident at once stages the weights once per workgroup.
template <bool ALPHA>
__global__ __launch_bounds__(FNW * 64) void conv_fused_kernel(const float *q, const char *P, Packed pk, Norm nrm, float *z,
                                                              int B, int H, int W, Proj pr)
{
    const int tx_n = W / FT, ty_n = H / FT, total = B * tx_n * ty_n;
    const size_t hw = (size_t)H * W;
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const bool first = tile == (int)blockIdx.x;
        if (!first) __syncthreads();  // the previous tile's LDS reads are done
        const int b = tile / (tx_n * ty_n);
        const int r = tile - b * tx_n * ty_n;
        fused_tile<FT, ALPHA ? OUT_ALPHA : OUT_Z>(q + (size_t)b * 3 * hw, P, pk, nrm, z + (size_t)b * hw * 72, H, W,
                                                  (r / tx_n) * FT, (r % tx_n) * FT, pr, first, nullptr);
    }
}

// Work-list form: workgroup w finds its solve by binary search over the
// items' first network tile.  STAGE 1 reads q, STAGE 2 reads S1.  ntiles ==
// 0: the tile count is read from the list header (nitems[1]; graph replay).
template <int STAGE>
__global__ __launch_bounds__(FNW * 64) void conv_fused_batch_kernel(const LSolve *__restrict__ tab,
                                                                    const LItem *__restrict__ items,
                                                                    const int *__restrict__ nitems, int ntiles,
                                                                    int one, const char *P, Packed pk, Norm nrm,
                                                                    Proj pr)
{
    const int total = ntiles > 0 ? ntiles : nitems[1];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const bool first = w == (int)blockIdx.x;
        if (!first) __syncthreads();  // the previous tile's LDS reads are done
        LItem it;
        if (one) {
            it = items[0];
        } else {
            const int n = *nitems;
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (items[mid].tb_cnn <= w) lo = mid;
                else hi = mid - 1;
            }
            it = items[lo];
        }
        const LSolve &d = tab[it.solve];
        const int tile = w - it.tb_cnn, tx_n = d.nx / FT;
        const int ty = tile / tx_n, tx = tile - ty * tx_n;
        fused_tile<FT, OUT_ALPHA>(STAGE == 1 ? d.q : d.s1, P, pk, nrm, d.z, d.ny, d.nx, ty * FT, tx * FT, pr, first,
                                  nullptr);
    }
}

template <int FO, int OUT, int LO, int TS>
__device__ __forceinline__ float *fused_tile(const float *qb, const char *P, const Packed &pk, const Norm &nrm, float *zb,
                                             int H, int W, int y0, int x0, const Proj &pr, bool load_w, float *qf,
                                             const PlainRedo *rd)
{
    static_assert((FO == TS && LO == 0) || (OUT == OUT_Z_LDS && ((FO == TS + 1 && LO == 1) || (FO == TS + 2 && LO == 1))),
                  "output region: the tile, the tile and its low halo, or the tile and a one-cell ring");
    static_assert(TS == FT || OUT == OUT_Z_LDS, "other tile sides only for a stage in the same workgroup");
    constexpr int OFF = LO;               // the region starts OFF cells before the tile
    constexpr int FRI_ = FO + 10, FR0_ = FO + 8;
    __shared__ bf16 s_in[3][FRI_ * FRI_];
    // activations, 32 channels = 4 x bf16x8 per pixel: layers 0 and 2 write
    // s_a0, layers 1 and 3 write s_a1
    constexpr int AS = 5;  // activation octets per pixel (act_slot)
    __shared__ bf16x8 s_act[FR0_ * FR0_ * AS + (FR0_ - 2) * (FR0_ - 2) * AS];
    bf16x8 *const s_a0 = s_act;
    bf16x8 *const s_a1 = s_act + FR0_ * FR0_ * AS;
    // all five layers' packed weights, staged together
    constexpr int W0 = 32 * 32 / 8, WH = 9 * 32 * 32 / 8, W4 = FW_EL / 8;
    __shared__ bf16x8 s_wall[W0 + 3 * WH + W4];
    __shared__ float s_bias[4 * 32 + 80];  // layer l < 4 at 32 l, layer 4 at 128

    // the wave index as a scalar: MFMAs under a wave-dependent condition
    // must sit behind a real branch (an MFMA does not honour a partial EXEC)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, px = lane & 15;
    const size_t hw = (size_t)H * W;
    const int ry0 = y0 - OFF - 5, rx0 = x0 - OFF - 5;  // origin of the input region

    // input region, normalised and rounded to BF16 as the first layer reads
    // it, and all five layers' weights: every global load is issued before
    // the first LDS store.  qf (OUT_Z_LDS): the FP32 values of the
    // (TS + 6)^2 cells from (x0 - 3, y0 - 3), kept for the learned stage.
    constexpr int NIN = 3 * FRI_ * FRI_, TIN = (NIN + FNW * 64 - 1) / (FNW * 64);
    // the redo flag's load first: the decision below then waits for it alone,
    // not for the input's loads, and the weights' loads follow at once
    const int rflag = OUT == OUT_Z_LDS && rd && rd->xprev ? *rd->flag : 0;
    float xin[TIN];
#pragma unroll
    for (int k = 0; k < TIN; k++) {
        const int i = threadIdx.x + k * FNW * 64;
        if (i < NIN) {
            const int ci = i / (FRI_ * FRI_), r = i - ci * FRI_ * FRI_;
            const int ry = r / FRI_, rx = r - ry * FRI_;
            const int yy = wrap(ry0 + ry, H), xx = wrap(rx0 + rx, W);
            xin[k] = qb[(size_t)ci * hw + (size_t)yy * W + xx];
        }
    }
    if constexpr (OUT == OUT_Z_LDS) {
        // the redo decision after the loads have been issued (their values
        // are discarded on a redo); the activations' LDS is free until layer
        // 0's first store, which follows the staging barrier below
        if (rflag) {
            static_assert(3 * ((FRI_ + 8) * (FRI_ + 8) + (FRI_ + 4) * (FRI_ + 4) + FRI_ * FRI_) * 4 <= sizeof(s_act),
                          "the redo's three fields fit over the activations");
            const float *sr = redo_region<FRI_, TS>(rd->xprev, rd->xk, rd->dt, rd->rdx, rd->rdy, rd->ph.g, rd->ph.sqg,
                                                rd->ph.h0, rd->fatal, H, W, rx0, ry0, x0, y0, (float *)s_act);
#pragma unroll
            for (int k = 0; k < TIN; k++) {
                const int i = threadIdx.x + k * FNW * 64;
                if (i < NIN) xin[k] = sr[i];
            }
        }
    }
    // all five layers' weights straight into LDS, waited for at the
    // staging barrier (the waves issue no LDS writes for them)
    BiasChunk<80, Packed> cb;
    if (load_w) {
        cb.load(P, pk);
        dma_weights<W0 / 64>(P + pk.w[0], s_wall, wave, lane);
        dma_weights<WH / 64>(P + pk.w[1], s_wall + W0, wave, lane);
        dma_weights<WH / 64>(P + pk.w[2], s_wall + W0 + WH, wave, lane);
        dma_weights<WH / 64>(P + pk.w[3], s_wall + W0 + 2 * WH, wave, lane);
        dma_weights<W4 / 64>(P + pk.w[4], s_wall + W0 + 3 * WH, wave, lane);
    }
#pragma unroll
    for (int k = 0; k < TIN; k++) {
        const int i = threadIdx.x + k * FNW * 64;
        if (i < NIN) {
            const int ci = i / (FRI_ * FRI_), r = i - ci * FRI_ * FRI_;
            s_in[ci][r] = (bf16)((xin[k] - nrm.mean[ci]) * nrm.inv_std[ci]);
            if (OUT == OUT_Z_LDS) {
                // the halo's corner (x0 - 3, y0 - 3) is 2 + OFF cells into the input region
                constexpr int QS = TS + 6, QO = 2 + OFF;
                const int rr = r / FRI_, ry = rr - QO, rx = r - rr * FRI_ - QO;
                if (ry >= 0 && ry < QS && rx >= 0 && rx < QS) qf[(ci * QS + ry) * QS + rx] = xin[k];
            }
        }
    }
    if (load_w) cb.store(s_bias);
    barrier_after_weights();

    // layer 0 on the FR0_ x FR0_ region, 16 pixels per group
    {
        const float *bias = s_bias;
        const bf16x8 A0 = s_wall[wfrag(0, px, g)], A1 = s_wall[wfrag(1, px, g)];
        constexpr int NP0 = FR0_ * FR0_, NG0 = (NP0 + 15) / 16, KG = (NG0 + FNW - 1) / FNW;
        // all KG groups gi = wave + k FNW of this wave at once (a group past
        // the region computes on pixel 0 and stores nothing), so that every
        // operand read is issued before the MFMAs
        bf16x8 bx[KG];
        int pk_[KG];
#pragma unroll
        for (int k = 0; k < KG; k++) {
            const int p = (wave + k * FNW) * 16 + px;
            pk_[k] = p;
            const int pc = p < NP0 ? p : 0;
            const int py = pc / FR0_, pxx = pc - py * FR0_;
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int kk = 8 * g + e;
                bf16 v = (bf16)0.0f;
                if (kk < 27) {
                    const int tap = kk / 3, ci = kk - 3 * tap;
                    v = s_in[ci][(py + tap / 3) * FRI_ + pxx + tap % 3];
                }
                bx[k][e] = v;
            }
        }
#pragma unroll
        for (int k = 0; k < KG; k++) {
            floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, bx[k], acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, bx[k], acc[1], 0, 0, 0);
            const int p = pk_[k];
            if (p < NP0) {
#pragma unroll
                for (int t = 0; t < 2; t++) {
                    const int co0 = 16 * t + 4 * g;
                    bf16x4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[t][i] + bias[co0 + i], 0.0f);
                    *(bf16x4 *)((bf16 *)s_a0 + act_off<AS>(p, co0)) = o;
                }
            }
        }
    }
    // hidden layers 1..3: s_a0 -> s_a1 -> s_a0 -> s_a1
#pragma unroll
    for (int l = 1; l < 4; l++) {
        __syncthreads();  // previous layer's output written
        const int rin = FR0_ - 2 * (l - 1);
        const bf16x8 *in = (l & 1) ? s_a0 : s_a1;
        bf16 *out = (bf16 *)((l & 1) ? s_a1 : s_a0);
        fused_hidden<AS>(in, rin, out, s_wall + W0 + (l - 1) * WH, s_bias + 32 * l, wave, lane);
    }
    __syncthreads();
    // layer 4: s_a1 (FO + 2)^2 -> z on the FO x FO region: NG pixel groups x
    // 5 co tiles of accumulation chains of 9 taps
    const bf16x8 *s_w = s_wall + W0 + 3 * WH;
    // [FO*FO][72] over the activations (modes that stage z in LDS; the
    // weights stay for the workgroup's next tile): it covers s_a0 and the
    // start of s_a1, which layer 4 reads before the barrier that precedes its
    // first store
    float *s_z = (float *)s_act;
    static_assert(FO * FO * 72 * 4 <= sizeof(s_act), "coefficient region fits over the activations");
    constexpr bool ALPHA = OUT != OUT_Z;  // z staged in LDS
    constexpr int NG4 = (FO * FO + 15) / 16;
    if constexpr (NG4 <= 3) {
        floatx4 acc[NG4];
        last_layer_by_tile<NG4, 5, FO, AS>(s_a1, s_w, wave, g, px, acc);
        if (ALPHA) __syncthreads();  // every wave past its layer-4 reads of s_a1 before it holds z
        const float *bias = s_bias + 128;
        const int co0 = 16 * wave + 4 * g;
        if (wave < 5 && co0 < 72) {
#pragma unroll
            for (int k = 0; k < NG4; k++) {
                const int p = k * 16 + px;
                if (p < FO * FO) {
                    floatx4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = acc[k][i] + bias[co0 + i];
                    if (ALPHA) {
                        *(floatx4 *)(s_z + p * 72 + co0) = o;
                    } else {
                        const int py = p / FO, pxx = p - py * FO;
                        *(floatx4 *)(zb + ((size_t)(y0 + py) * W + x0 + pxx) * 72 + co0) = o;
                    }
                }
            }
        }
    } else {
        // pixel groups wave, wave + FNW, ... with all NT co tiles, the
        // activation fragment read once per tap for NT MFMAs; each co tile's
        // chain keeps the tap order 0..8
        constexpr int NT = 5, RIN = FO + 2, NPX = FO * FO, NG = (NPX + 15) / 16, GPW = (NG + FNW - 1) / FNW;
        const float *bias = s_bias + 128;
        floatx4 acc[GPW][NT];
#pragma unroll
        for (int k = 0; k < GPW; k++)
#pragma unroll
            for (int t = 0; t < NT; t++) acc[k][t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < GPW; k++) {
            const int gi = wave + k * FNW, p = gi * 16 + px;
            if (gi < NG) {  // wave-uniform, a real branch: an MFMA does not honour a partial EXEC
                const int pc = p < NPX ? p : 0;
                const int py = pc / FO, pxx = pc - py * FO;
                const int qb = py * RIN + pxx;
#pragma unroll
                for (int tap = 0; tap < 9; tap++) {
                    const bf16x8 bx = s_a1[act_slot<AS>(qb + (tap / 3) * RIN + tap % 3, g)];
#pragma unroll
                    for (int t = 0; t < NT; t++)
                        acc[k][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[wfrag(tap * NT + t, px, g)], bx,
                                                                            acc[k][t], 0, 0, 0);
                }
            }
        }
        if (ALPHA) __syncthreads();  // every wave past its layer-4 reads of s_a1 before it holds z
#pragma unroll
        for (int k = 0; k < GPW; k++) {
            const int gi = wave + k * FNW, p = gi * 16 + px;
            if (gi < NG && p < NPX) {
                const int py = p / FO, pxx = p - py * FO;
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const int co0 = 16 * t + 4 * g;
                    if (co0 < 72) {
                        floatx4 o;
#pragma unroll
                        for (int i = 0; i < 4; i++) o[i] = acc[k][t][i] + bias[co0 + i];
                        if (ALPHA) *(floatx4 *)(s_z + p * 72 + co0) = o;
                        else *(floatx4 *)(zb + ((size_t)(y0 + py) * W + x0 + pxx) * 72 + co0) = o;
                    }
                }
            }
        }
    }
    if (ALPHA) __syncthreads();
    if (OUT == OUT_ALPHA) {
        // FO^2 pixels x 12 groups of six, (axis*2 + side)*3 + var: alpha
        // replaces z in place
        for (int task = threadIdx.x; task < FO * FO * 12; task += FNW * 64) {
            const int p = task / 12, grp = task - p * 12;
            alpha_group(s_z + p * 72 + grp * 6, (grp / 3) & 1, pr);
        }
        __syncthreads();
        // each tile row's 8 x 72 values, contiguous in the output, leave as
        // 16-byte stores
        constexpr int RV = TS * 72 / 4;  // float4 per tile row
        for (int i = threadIdx.x; i < TS * RV; i += FNW * 64) {
            const int row = i / RV, c = i - row * RV;
            ((float4 *)(zb + ((size_t)(y0 + row) * W + x0) * 72))[c] = ((const float4 *)(s_z + row * TS * 72))[c];
        }
    }
    return s_z;
}

// ------------------------------------------- Euler network, one launch
// All five layers of the Euler network (4 -> 32 -> 32 -> 32 -> 32 -> 96) for
// one output region per workgroup pass, as fused_tile does for the planar
// network: the normalised BF16 input region (FO + 10)^2 of the four
// variables and every layer's weights staged in LDS, the activations kept in
// two LDS buffers, layer l computed on the (FO + 2(4 - l))^2 region.  Per
// output the MFMAs run in the layer-by-layer pass's order (layer 0: K blocks
// 0, 1; other layers: taps 0..8), with the same bias, ReLU and BF16 rounding,
// so z is bit-identical to launch_forward_euler's.
constexpr int EW0 = 32 * 64 / 8, EWH = 9 * 32 * 32 / 8, EW4 = 9 * 6 * 16 * 32 / 8;  // packed octets per layer

// Plain (MINMOD, FLUX) Heun step of one Euler solve's previous state xprev
// on the R x R region at (ox, oy), recomputed from xprev on the region grown
// by four cells, as redo_region does for shallow water: the redo of a flagged
// step on the region one workgroup of the next step reads.  Each face's
// states (MINMOD with the admissibility fallback), flux and each cell's
// update are the learned Euler stage kernel's plain arithmetic (MODES 2 and
// 3).  The TS x TS tile at (x0, y0) writes its cells of the result to xk and
// raises *fatal where a plain stage leaves one of them inadmissible.  Needs
// 4 ((R + 8)^2 + (R + 4)^2 + R^2) floats of LDS at buf; returns the region,
// [4][R][R], in buf.  Out of line, its arguments in registers.
template <int N, int FLUX>
__device__ __forceinline__ void euler_cell_fluxes(const float *f, int r, int c, float gamma, float (*F)[4])
{
#pragma unroll
    for (int face = 0; face < 4; face++) {
        const int ax = face >> 1, hi = face & 1;  // axis, and whether the face is on the cell's high side
        float st[4][6];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            st[v][0] = 0.0f;
            st[v][5] = 0.0f;
#pragma unroll
            for (int k = 1; k < 5; k++) {
                const int o = k - 3 + hi;
                st[v][k] = ax == 0 ? f[(v * N + r) * N + c + o] : f[(v * N + r + o) * N + c];
            }
        }
        float QL[4], QR[4];
        eln::face_states<false>(st, nullptr, Proj{}, gamma, QL, QR);
        if (ax == 0) eln::flux4<FLUX, 0>(QL, QR, gamma, F[face]);
        else eln::flux4<FLUX, 1>(QL, QR, gamma, F[face]);
        flux_barrier<4>(F[face]);
    }
}

template <int R, int FLUX, int TS>
__device__ __noinline__ float *euler_redo_region(const float *xprev, float *xk, float dt, float rdx, float rdy,
                                                 float gamma, int *fatal, int H, int W, int ox, int oy, int x0, int y0,
                                                 float *buf)
{
    constexpr int A = R + 8, S = R + 4, NT = FNW * 64;
    float *sa = buf;              // [4][A][A] xprev from (ox - 4, oy - 4)
    float *ss = sa + 4 * A * A;   // [4][S][S] plain stage 1 from (ox - 2, oy - 2)
    float *sr = ss + 4 * S * S;   // [4][R][R] the redone state from (ox, oy)
    const int tid = threadIdx.x;
    const size_t plane = (size_t)H * W;
    for (int k = tid; k < 4 * A * A; k += NT) {
        const int v = k / (A * A), r = k - v * A * A, ry = r / A, rx = r - ry * A;
        // up to ten cells out from a tile of a grid as small as 16 cells: the full modulo
        sa[k] = xprev[v * plane + (size_t)pwrap(oy - 4 + ry, H) * W + pwrap(ox - 4 + rx, W)];
    }
    __syncthreads();
    bool bad = false;
    // stage 1: S1 = q + dt L(q); cell (j, i) of ss is (j + 2, i + 2) of sa
    for (int k = tid; k < S * S; k += NT) {
        const int j = k / S, i = k - j * S;
        float F[4][4];
        euler_cell_fluxes<A, FLUX>(sa, j + 2, i + 2, gamma, F);
        const int gx = ox - 2 + i - x0, gy = oy - 2 + j - y0;  // tile-relative
        float qn[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const float L = -(F[1][v] - F[0][v]) * rdx - (F[3][v] - F[2][v]) * rdy;
            float o = 1.0f * (sa[(v * A + j + 2) * A + i + 2] + dt * L);
            ss[(v * S + j) * S + i] = o;
            qn[v] = o;
        }
        if (gx >= 0 && gx < TS && gy >= 0 && gy < TS) bad = bad || !eln::admissible(qn, gamma);
    }
    __syncthreads();
    // stage 2: q/2 + (S1 + dt L(S1))/2; cell (j, i) of sr is (j + 2, i + 2) of ss
    for (int k = tid; k < R * R; k += NT) {
        const int j = k / R, i = k - j * R;
        float F[4][4];
        euler_cell_fluxes<S, FLUX>(ss, j + 2, i + 2, gamma, F);
        const int gx = ox + i - x0, gy = oy + j - y0;
        float qn[4];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const float L = -(F[1][v] - F[0][v]) * rdx - (F[3][v] - F[2][v]) * rdy;
            float o = 0.5f * (ss[(v * S + j + 2) * S + i + 2] + dt * L);
            o = 0.5f * sa[(v * A + j + 4) * A + i + 4] + o;
            sr[(v * R + j) * R + i] = o;
            qn[v] = o;
        }
        if (gx >= 0 && gx < TS && gy >= 0 && gy < TS) {
#pragma unroll
            for (int v = 0; v < 4; v++) xk[v * plane + (size_t)(y0 + gy) * W + x0 + gx] = qn[v];
            bad = bad || !eln::admissible(qn, gamma);
        }
    }
    if (bad) atomicExch(fatal, 1);
    __syncthreads();
    return sr;
}

// The output region is the TS x TS tile at (x0, y0) (FO = TS: z written to
// zb, [H][W][96]) or the tile and its low halo row and column (FO = TS + 1,
// ZLDS: z kept in LDS as [FO*FO][96] from (x0 - 1, y0 - 1) and returned, and
// the FP32 stage input with a three-cell halo in qf, [4][TS+6][TS+6] from
// (x0 - 3, y0 - 3)).  load_w: stage the weights (the workgroup's first tile).
// redo (ZLDS): the input region is the plain redo of the previous step from
// redo_from (euler_redo_region, the tile's cells written to qb) instead of qb.
// TS: the tile side (FT, or 4 for a stage in the same workgroup on few tiles).
template <int FO, bool ZLDS, int FLUX = 0, int TS = FT>
__device__ __forceinline__ float *fused_tile_euler(const float *qb, const char *P, const EPacked &pk,
                                                   const ENorm &nrm, float *zb, int H, int W, int y0, int x0,
                                                   bool load_w, float *qf, const float *redo_from = nullptr,
                                                   const eln::StageArgs *ra = nullptr, int *fatal = nullptr)
{
    static_assert(FO == TS || (FO == TS + 1 && ZLDS), "output region: the tile, or the tile and its low halo");
    static_assert(TS == FT || ZLDS, "other tile sides only for a stage in the same workgroup");
    constexpr int OFF = FO - TS, FRI_ = FO + 10, FR0_ = FO + 8;
    __shared__ bf16 s_in[E_CIN][FRI_ * FRI_];
    // activation octets per pixel (act_slot): the padded layout, except on
    // the largest region with the stage's buffers, where it would not fit
    constexpr int AS = (ZLDS && FO == FT + 1) ? 4 : 5;
    __shared__ bf16x8 s_act[FR0_ * FR0_ * AS + (FR0_ - 2) * (FR0_ - 2) * AS];
    __shared__ bf16x8 s_wall[EW0 + 3 * EWH + EW4];
    __shared__ float s_bias[4 * 32 + E_COUT];  // layer l < 4 at 32 l, layer 4 at 128
    bf16x8 *const s_a0 = s_act;
    bf16x8 *const s_a1 = s_act + FR0_ * FR0_ * AS;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, px = lane & 15;
    const size_t hw = (size_t)H * W;
    const int ry0 = y0 - OFF - 5, rx0 = x0 - OFF - 5;
    // every global load (input region, weights) before the first LDS store
    constexpr int NIN = E_CIN * FRI_ * FRI_, TIN = (NIN + FNW * 64 - 1) / (FNW * 64);
    float xin[TIN];
#pragma unroll
    for (int k = 0; k < TIN; k++) {
        const int i = threadIdx.x + k * FNW * 64;
        if (i < NIN) {
            const int ci = i / (FRI_ * FRI_), r = i - ci * FRI_ * FRI_;
            const int ry = r / FRI_, rx = r - ry * FRI_;
            xin[k] = qb[(size_t)ci * hw + (size_t)wrap(ry0 + ry, H) * W + wrap(rx0 + rx, W)];
        }
    }
    if constexpr (ZLDS) {
        // the redo decision after the loads have been issued (their values
        // are discarded); the activations' LDS is free until layer 0's first
        // store, which follows the staging barrier below
        if (redo_from) {
            static_assert(4 * ((FRI_ + 8) * (FRI_ + 8) + (FRI_ + 4) * (FRI_ + 4) + FRI_ * FRI_) * 4 <= sizeof(s_act),
                          "the redo's three fields fit over the activations");
            const float *sr = euler_redo_region<FRI_, FLUX, TS>(redo_from, (float *)qb, ra->dt, ra->rdx, ra->rdy,
                                                            ra->gamma, fatal, H, W, rx0, ry0, x0, y0,
                                                            (float *)s_act);
#pragma unroll
            for (int k = 0; k < TIN; k++) {
                const int i = threadIdx.x + k * FNW * 64;
                if (i < NIN) xin[k] = sr[i];
            }
        }
    }
    // all five layers' weights straight into LDS (layer 0's in the packed
    // order: it reads its two K blocks so), waited for at the staging barrier
    BiasChunk<E_COUT, EPacked> cb;
    if (load_w) {
        cb.load(P, pk);
        dma_weights<EW0 / 64, false>(P + pk.w[0], s_wall, wave, lane);
        dma_weights<EWH / 64>(P + pk.w[1], s_wall + EW0, wave, lane);
        dma_weights<EWH / 64>(P + pk.w[2], s_wall + EW0 + EWH, wave, lane);
        dma_weights<EWH / 64>(P + pk.w[3], s_wall + EW0 + 2 * EWH, wave, lane);
        dma_weights<EW4 / 64>(P + pk.w[4], s_wall + EW0 + 3 * EWH, wave, lane);
    }
#pragma unroll
    for (int k = 0; k < TIN; k++) {
        const int i = threadIdx.x + k * FNW * 64;
        if (i < NIN) {
            const int ci = i / (FRI_ * FRI_), r = i - ci * FRI_ * FRI_;
            s_in[ci][r] = (bf16)((xin[k] - nrm.mean[ci]) * nrm.inv_std[ci]);
            if (ZLDS) {
                // the halo's corner (x0 - 3, y0 - 3) is 2 + OFF cells into the input region
                constexpr int QS = TS + 6, QO = 2 + OFF;
                const int rr = r / FRI_, ry = rr - QO, rx = r - rr * FRI_ - QO;
                if (ry >= 0 && ry < QS && rx >= 0 && rx < QS) qf[(ci * QS + ry) * QS + rx] = xin[k];
            }
        }
    }
    if (load_w) cb.store(s_bias);
    barrier_after_weights();
    // layer 0 on the FR0_ x FR0_ region: K = 36 (tap*4 + ci) in two blocks
    {
        const float *bias = s_bias;
        constexpr int NP0 = FR0_ * FR0_, NG0 = (NP0 + 15) / 16;
        for (int gi = wave; gi < NG0; gi += FNW) {
            const int p = gi * 16 + px;
            const int pc = p < NP0 ? p : 0;
            const int py = pc / FR0_, pxx = pc - py * FR0_;
            bf16x8 bx[2];
#pragma unroll
            for (int kb = 0; kb < 2; kb++)
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int kk = 32 * kb + 8 * g + e;
                    bf16 v = (bf16)0.0f;
                    if (kk < 9 * E_CIN) {
                        const int tap = kk / E_CIN, ci = kk - E_CIN * tap;
                        v = s_in[ci][(py + tap / 3) * FRI_ + pxx + tap % 3];
                    }
                    bx[kb][e] = v;
                }
#pragma unroll
            for (int t = 0; t < 2; t++) {
                floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 2; kb++)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_wall[(t * 16 + px) * 8 + kb * 4 + g], bx[kb], acc,
                                                                  0, 0, 0);
                if (p < NP0) {
                    const int co0 = 16 * t + 4 * g;
                    bf16x4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[i] + bias[co0 + i], 0.0f);
                    *(bf16x4 *)((bf16 *)s_a0 + act_off<AS>(p, co0)) = o;
                }
            }
        }
    }
    // hidden layers 1..3: s_a0 -> s_a1 -> s_a0 -> s_a1
#pragma unroll
    for (int l = 1; l < 4; l++) {
        __syncthreads();
        const int rin = FR0_ - 2 * (l - 1);
        const bf16x8 *in = (l & 1) ? s_a0 : s_a1;
        bf16 *out = (bf16 *)((l & 1) ? s_a1 : s_a0);
        fused_hidden<AS>(in, rin, out, s_wall + EW0 + (l - 1) * EWH, s_bias + 32 * l, wave, lane);
    }
    __syncthreads();
    // layer 4: s_a1 (FO + 2)^2 -> z on the FO x FO region, pixel groups wave,
    // wave + FNW, ... with all six co tiles, each chain in tap order.  ZLDS:
    // z over the activations ([FO*FO][96] covers s_a0 and the start of s_a1),
    // stored after every wave's layer-4 reads
    float *s_z = (float *)s_act;
    static_assert(!ZLDS || FO * FO * E_COUT * 4 <= sizeof(s_act), "coefficient region fits over the activations");
    constexpr int NG4 = (FO * FO + 15) / 16;
    if constexpr (NG4 <= 3) {
        // few pixel groups: one co tile per wave (last_layer_by_tile)
        floatx4 acc[NG4];
        last_layer_by_tile<NG4, 6, FO, AS>(s_a1, s_wall + EW0 + 3 * EWH, wave, g, px, acc);
        if (ZLDS) __syncthreads();
        const float *bias = s_bias + 128;
        const int co0 = 16 * wave + 4 * g;
        if (wave < 6) {
#pragma unroll
            for (int k = 0; k < NG4; k++) {
                const int p = k * 16 + px;
                if (p < FO * FO) {
                    floatx4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = acc[k][i] + bias[co0 + i];
                    if (ZLDS) {
                        *(floatx4 *)(s_z + p * E_COUT + co0) = o;
                    } else {
                        const int py = p / FO, pxx = p - py * FO;
                        *(floatx4 *)(zb + ((size_t)(y0 + py) * W + x0 + pxx) * E_COUT + co0) = o;
                    }
                }
            }
        }
    } else {
        constexpr int NT = 6, RIN = FO + 2, NPX = FO * FO, NG = (NPX + 15) / 16, GPW = (NG + FNW - 1) / FNW;
        const bf16x8 *s_w = s_wall + EW0 + 3 * EWH;
        const float *bias = s_bias + 128;
        floatx4 acc[GPW][NT];
#pragma unroll
        for (int k = 0; k < GPW; k++) {
#pragma unroll
            for (int t = 0; t < NT; t++) acc[k][t] = floatx4{0.f, 0.f, 0.f, 0.f};
            const int gi = wave + k * FNW, p = gi * 16 + px;
            if (gi < NG) {  // wave-uniform, a real branch: an MFMA does not honour a partial EXEC
                const int pc = p < NPX ? p : 0;
                const int py = pc / FO, pxx = pc - py * FO;
                const int qb = py * RIN + pxx;
#pragma unroll
                for (int tap = 0; tap < 9; tap++) {
                    const bf16x8 bx = s_a1[act_slot<AS>(qb + (tap / 3) * RIN + tap % 3, g)];
#pragma unroll
                    for (int t = 0; t < NT; t++)
                        acc[k][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[wfrag(tap * NT + t, px, g)], bx,
                                                                            acc[k][t], 0, 0, 0);
                }
            }
        }
        if (ZLDS) __syncthreads();
#pragma unroll
        for (int k = 0; k < GPW; k++) {
            const int gi = wave + k * FNW, p = gi * 16 + px;
            if (gi < NG && p < NPX) {
                const int py = p / FO, pxx = p - py * FO;
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const int co0 = 16 * t + 4 * g;
                    floatx4 o;
#pragma unroll
                    for (int i = 0; i < 4; i++) o[i] = acc[k][t][i] + bias[co0 + i];
                    if (ZLDS) *(floatx4 *)(s_z + p * E_COUT + co0) = o;
                    else *(floatx4 *)(zb + ((size_t)(y0 + py) * W + x0 + pxx) * E_COUT + co0) = o;
                }
            }
        }
    }
    if (ZLDS) __syncthreads();
    return s_z;
}

// Workgroups stride over the B x (H/FT) x (W/FT) tiles, staging the weights
// once.
__global__ __launch_bounds__(FNW * 64) void conv_fused_euler_kernel(const float *q, const char *P, EPacked pk,
                                                                    ENorm nrm, float *z, int B, int H, int W)
{
    const size_t hw = (size_t)H * W;
    const int tx_n = W / FT, ty_n = H / FT, total = B * tx_n * ty_n;
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const bool load_w = tile == (int)blockIdx.x;
        if (!load_w) __syncthreads();  // the previous tile's LDS reads are done
        const int b = tile / (tx_n * ty_n);
        const int rt = tile - b * tx_n * ty_n;
        fused_tile_euler<FT, false>(q + (size_t)b * E_CIN * hw, P, pk, nrm, z + (size_t)b * hw * E_COUT, H, W,
                                    (rt / tx_n) * FT, (rt % tx_n) * FT, load_w, nullptr);
    }
}

// Network pass and learned Euler stage (the learned Euler stage kernel's
// MODE 0 arithmetic) of one stage for B solves, one FT x FT tile per
// workgroup pass: the coefficients of the tile and its low halo stay in LDS,
// each face projects its owner's 48, forms both states with the per-side
// admissibility fallback and takes the Euler flux; one x face, one y face and
// one cell per thread.  Frozen solves are skipped.  Flags and fallback counts
// as the stage kernel's.
template <int FLUX, int TS = FT>
__global__ __launch_bounds__(FNW * 64) void conv_learned_euler_kernel(eln::StageArgs a, const char *P, EPacked pk,
                                                                      ENorm nrm, const float *xprev)
{
    constexpr int TX = TS, TY = TS, QS = TS + 6, FO = TS + 1;
    constexpr int NFX = TY * (TX + 1), NFY = (TY + 1) * TX, YB = 128;  // y faces start at thread YB
    static_assert(NFX <= YB && YB + NFY <= FNW * 64 && TX * TY <= FNW * 64, "one face or cell per thread");
    __shared__ float s_qf[4 * QS * QS];
    __shared__ float s_fx[4][TY][TX + 1];
    __shared__ float s_fy[4][TY + 1][TX];
    __shared__ int s_cnt, s_bad;
    const int nx = a.nx, ny = a.ny, tid = threadIdx.x;
    const size_t plane = (size_t)nx * ny;
    const int tx_n = nx / TS, ty_n = ny / TS, total = a.B * tx_n * ty_n;
    bool staged = false;  // this workgroup's weights are in LDS
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int b = tile / (tx_n * ty_n);
        // stage 1 with xprev: a solve whose previous step is flagged is redone
        // on this workgroup's region first (no writer of that slot in stage
        // 1).  A frozen solve's tiles run the pass but write nothing (live
        // false), so that neither flag is waited for before the input's
        // loads are issued (an early exit makes the compiler wait for them)
        const int fz = a.fatal[b];
        const int rf = a.flagbit == 1 && xprev ? a.flags[2 * b + (a.parity ^ 1)] : 0;
        if (staged) __syncthreads();  // the previous tile's LDS reads are done
        const int rt = tile - b * tx_n * ty_n;
        const int y0 = (rt / tx_n) * TS, x0 = (rt % tx_n) * TS;
        const bool live = fz == 0, redo = rf != 0 && live;
        // stage 2 (a0 != 0): the cell's q^n loaded now, its latency behind the network pass
        float q0v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (a.a0 != 0.0f && tid < TX * TY) {
            const int cy = tid / TX, cx = tid - cy * TX;
            const size_t idx = (size_t)b * 4 * plane + (size_t)(y0 + cy) * nx + x0 + cx;
#pragma unroll
            for (int v = 0; v < 4; v++) q0v[v] = a.q0[idx + v * plane];
        }
        float *s_z = fused_tile_euler<FO, true, FLUX, TS>(
            a.qs + (size_t)b * 4 * plane, P, pk, nrm, nullptr, ny, nx, y0, x0, !staged, s_qf,
            redo ? xprev + (size_t)b * 4 * plane : nullptr, &a, a.fatal + b);
        staged = true;
        if (redo && rt == 0 && tid == 0) a.redone[b] += 1;
        int *flag = a.flags + 2 * b + a.parity;
        // stage 2 of a solve whose stage 1 failed is evaluated (its result is
        // discarded by the redo) but its fallback sides are not counted
        const bool count = !(a.flagbit == 2 && (*flag & 1));
        if (tid == 0) {
            s_cnt = 0;
            s_bad = 0;
        }
        // every pixel's sixteen groups of six projected in place by all the
        // workgroup's threads, alpha = base + P z (the faces then read alpha)
        for (int task = tid; task < FO * FO * 16; task += FNW * 64) {
            const int p = task >> 4, grp = task & 15;
            alpha_group(s_z + p * E_COUT + grp * 6, (grp >> 2) & 1, a.pr);
        }
        __syncthreads();
        int nfb = 0;
        if (tid < NFX) {
            // x face: owner cell (x0 - 1 + xi, y0 + xj), pixel (xi, xj + 1) of the coefficient region
            const int xj = tid / (TX + 1), xi = tid - xj * (TX + 1);
            float st[4][6];
#pragma unroll
            for (int v = 0; v < 4; v++)
#pragma unroll
                for (int k = 0; k < 6; k++) st[v][k] = s_qf[(v * QS + xj + 3) * QS + xi + k];
            float QL[4], QR[4], F[4];
            const int c = eln::face_states<true, true>(st, s_z + ((xj + 1) * FO + xi) * E_COUT, a.pr, a.gamma, QL,
                                                       QR);
            if (xi < TX) nfb += c;  // counted once: as a cell's low face
            eln::flux4<FLUX, 0>(QL, QR, a.gamma, F);
#pragma unroll
            for (int v = 0; v < 4; v++) s_fx[v][xj][xi] = F[v];
        }
        if (tid >= YB && tid < YB + NFY) {
            // y face: owner cell (x0 + yi, y0 - 1 + yj), pixel (yi + 1, yj)
            const int f = tid - YB, yj = f / TX, yi = f - yj * TX;
            float st[4][6];
#pragma unroll
            for (int v = 0; v < 4; v++)
#pragma unroll
                for (int k = 0; k < 6; k++) st[v][k] = s_qf[(v * QS + yj + k) * QS + yi + 3];
            float QL[4], QR[4], F[4];
            const int c = eln::face_states<true, true>(st, s_z + (yj * FO + yi + 1) * E_COUT + 48, a.pr, a.gamma,
                                                       QL, QR);
            if (yj < TY) nfb += c;
            eln::flux4<FLUX, 1>(QL, QR, a.gamma, F);
#pragma unroll
            for (int v = 0; v < 4; v++) s_fy[v][yj][yi] = F[v];
        }
        __syncthreads();
        bool bad = false;
        if (live && tid < TX * TY) {
            const int cy = tid / TX, cx = tid - cy * TX;
            const size_t idx = (size_t)b * 4 * plane + (size_t)(y0 + cy) * nx + x0 + cx;
            float qn[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const float L = -(s_fx[v][cy][cx + 1] - s_fx[v][cy][cx]) * a.rdx -
                                (s_fy[v][cy + 1][cx] - s_fy[v][cy][cx]) * a.rdy;
                float o = a.a1 * (s_qf[(v * QS + cy + 3) * QS + cx + 3] + a.dt * L);
                if (a.a0 != 0.0f) o = a.a0 * q0v[v] + o;
                a.out[idx + v * plane] = o;
                qn[v] = o;
            }
            bad = !eln::admissible(qn, a.gamma);
        }
        if (live && count && nfb) atomicAdd(&s_cnt, nfb);
        if (bad) s_bad = 1;
        __syncthreads();
        if (live && tid == 0) {
            if (s_cnt) atomicAdd(&a.nfb[b], (unsigned long long)s_cnt);
            if (s_bad) atomicOr(flag, a.flagbit);
            // stage 2: every reader of the previous step's slot has finished
            // (its stage 2 and this step's stage 1)
            if (a.flagbit == 2 && rt == 0) a.flags[2 * b + (a.parity ^ 1)] = 0;
        }
    }
}

int fused_euler_grid()
{
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int cus = 0, m = 0;
        int m1 = 0, m2 = 0, m3 = 0, m4 = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, conv_fused_euler_kernel, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&m1, conv_learned_euler_kernel<fvk::HLLE>, FNW * 64, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&m2, conv_learned_euler_kernel<fvk::RUSANOV>, FNW * 64, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&m3, conv_learned_euler_kernel<fvk::HLLE, 4>, FNW * 64, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&m4, conv_learned_euler_kernel<fvk::RUSANOV, 4>, FNW * 64, 0) !=
                hipSuccess)
            return 256;
        m = m < m1 ? m : m1;
        m = m < m2 ? m : m2;
        m = m < m3 ? m : m3;
        m = m < m4 ? m : m4;
        cache[dev] = (m > 0 ? m : 1) * (cus > 0 ? cus : 256);
    }
    return cache[dev];
}

hipError_t launch_forward_euler_fused(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                      float *z, hipStream_t st)
{
    if (nx % FT || ny % FT) return hipErrorInvalidValue;
    const int tiles = B * (nx / FT) * (ny / FT);
    const int cap = fused_euler_grid();
    hipLaunchKernelGGL(conv_fused_euler_kernel, dim3((unsigned)(tiles < cap ? tiles : cap)), dim3(FNW * 64), 0, st,
                       q, (const char *)packed, euler_packed_layout(), nrm, z, B, ny, nx);
    return hipGetLastError();
}

template <int TS>
static void launch_learned_euler_ts(int flux, int g, const char *Pc, const ENorm &nrm, const eln::StageArgs &a,
                                    hipStream_t st, const float *xprev)
{
    if (flux == fvk::RUSANOV)
        hipLaunchKernelGGL((conv_learned_euler_kernel<fvk::RUSANOV, TS>), dim3(g), dim3(FNW * 64), 0, st, a, Pc,
                           euler_packed_layout(), nrm, xprev);
    else
        hipLaunchKernelGGL((conv_learned_euler_kernel<fvk::HLLE, TS>), dim3(g), dim3(FNW * 64), 0, st, a, Pc,
                           euler_packed_layout(), nrm, xprev);
}

hipError_t launch_learned_euler(int flux, const void *packed, const ENorm &nrm, const eln::StageArgs &a, hipStream_t st,
                                const float *xprev)
{
    if (a.nx % FT || a.ny % FT || a.B < 1 || (a.flagbit != 1 && a.flagbit != 2) || (a.flagbit == 2 && xprev))
        return hipErrorInvalidValue;
    const int cap = fused_euler_grid();
    // 4 x 4 tiles while they all get a resident workgroup (more, shorter
    // workgroups on small batches of small grids), else 8 x 8
    const int ts = (size_t)a.B * (a.nx / 4) * (a.ny / 4) <= (size_t)cap ? 4 : FT;
    const int tiles = a.B * (a.nx / ts) * (a.ny / ts), g = tiles < cap ? tiles : cap;
    if (ts == 4) launch_learned_euler_ts<4>(flux, g, (const char *)packed, nrm, a, st, xprev);
    else launch_learned_euler_ts<FT>(flux, g, (const char *)packed, nrm, a, st, xprev);
    return hipGetLastError();
}

// ---------------------------------------- network pass + learned stage
// The learned stage (learned-stage kernels, MODE 0, HLLE) on the FT x FT tile
// at (x0, y0), in the workgroup that has just computed z on the tile and its
// low halo (s_z, [(FT+1)^2][72] from (x0 - 1, y0 - 1)) and kept the stage
// input with a 3-cell halo (qf, [3][FT+6][FT+6] from (x0 - 3, y0 - 3)): one x
// face, one y face and one cell per thread, the face and cell arithmetic of
// the learned-stage kernels; each face projects its owner's coefficients
// (alpha = base + P z, the network pass's operation order).  STAGE 1: S1 = q + dt L(q); STAGE 2: S2 = q/2 +
// (S1 + dt L(S1))/2.  Stage flags and fallback counts as there.
// DIR: the direct face-state scheme (face_states_direct): s_z holds the raw
// output on the tile and a one-cell ring ([(FT+2)^2][72] from (x0 - 1,
// y0 - 1)); each face takes its owner's high-side and its neighbour's
// low-side states (sig = 1 / inv_std of the network input).
// dt: the solve's step (*d.dt, read by the caller before the network pass);
// q0v (STAGE 2, or NULL): the cell's q^n values, loaded by the caller.
template <int STAGE, bool BL = false, bool DIR = false, int TS = FT>
__device__ __forceinline__ void learned_epilogue(const LSolve &d, const LItem &it, float *s_z, const float *qf,
                                                 const Proj &pr, const int x0, const int y0, const float dt,
                                                 const float *sig = nullptr, const float *q0v = nullptr)
{
    constexpr int TX = TS, TY = TS, QS = TS + 6, FO = DIR ? TS + 2 : TS + 1;
    constexpr int NFX = TY * (TX + 1), NFY = (TY + 1) * TX, YB = 128;  // y faces start at thread YB
    static_assert(NFX <= YB && YB + NFY <= FNW * 64 && TX * TY <= FNW * 64, "one face or cell per thread");
    constexpr float a0 = STAGE == 1 ? 0.0f : 0.5f, a1 = STAGE == 1 ? 1.0f : 0.5f;
    __shared__ float s_fx[3][TY][TX + 1];
    __shared__ float s_fy[3][TY + 1][TX];
    __shared__ int s_cnt;
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int nx = d.nx;
    const size_t plane = (size_t)nx * d.ny;
    int *bad = d.flags + it.parity;
    Phys<float> ph;
    ph.g = d.g;
    ph.sqg = d.sqg;
    ph.gamma = 1.4f;
    ph.h0 = d.h0;
    // stage 2 of a solve whose stage 1 failed is evaluated (its result is
    // discarded by the redo) but its fallback faces are not counted
    const bool count = !(STAGE == 2 && (*bad & 1));
    if (tid == 0) {
        s_cnt = 0;
        s_bad = 0;
    }
    if constexpr (!DIR) {
        // every pixel's twelve groups of six projected in place by all the
        // workgroup's threads, alpha = base + P z (the faces then read alpha)
        for (int task = tid; task < FO * FO * 12; task += FNW * 64) {
            const int p = task / 12, grp = task - p * 12;
            alpha_group(s_z + p * 72 + grp * 6, (grp / 3) & 1, pr);
        }
        __syncthreads();
    }
    int nfb = 0;
    if (tid < NFX) {
        // x face: owner cell (x0 - 1 + xi, y0 + xj)
        const int xj = tid / (TX + 1), xi = tid - xj * (TX + 1);
        float st[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = qf[(v * QS + xj + 3) * QS + xi + k];
        float QL[3], QR[3], F[3];
        const int c = DIR ? face_states_direct(st, s_z + ((xj + 1) * FO + xi) * 72 + 3,
                                               s_z + ((xj + 1) * FO + xi + 1) * 72, sig, QL, QR)
                          : face_states<0, true>(st, s_z + ((xj + 1) * FO + xi) * 72, pr, QL, QR);
        if (xi < TX) nfb += c;  // each face counted once: as the left face of a cell of this tile
        flux3<fvk::HLLE, 0>(QL, QR, ph, F);
        if (BL) blend_flux<fvk::HLLE, 0>(st, ph, F);
#pragma unroll
        for (int v = 0; v < 3; v++) s_fx[v][xj][xi] = F[v];
    }
    if (tid >= YB && tid < YB + NFY) {
        // y face: owner cell (x0 + yi, y0 - 1 + yj)
        const int f = tid - YB, yj = f / TX, yi = f - yj * TX;
        float st[3][6];
#pragma unroll
        for (int v = 0; v < 3; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) st[v][k] = qf[(v * QS + yj + k) * QS + yi + 3];
        float QL[3], QR[3], F[3];
        const int c = DIR ? face_states_direct(st, s_z + (yj * FO + yi + 1) * 72 + 9,
                                               s_z + ((yj + 1) * FO + yi + 1) * 72 + 6, sig, QL, QR)
                          : face_states<0, true>(st, s_z + (yj * FO + yi + 1) * 72 + 36, pr, QL, QR);
        if (yj < TY) nfb += c;
        flux3<fvk::HLLE, 1>(QL, QR, ph, F);
        if (BL) blend_flux<fvk::HLLE, 1>(st, ph, F);
#pragma unroll
        for (int v = 0; v < 3; v++) s_fy[v][yj][yi] = F[v];
    }
    __syncthreads();
    bool bc = false;
    if (tid < TX * TY) {
        const int cy = tid / TX, cx = tid - cy * TX;
        const size_t idx = (size_t)(y0 + cy) * nx + x0 + cx;
        const float *q0 = d.q;
        float *out = STAGE == 1 ? d.s1 : d.s2;
        float qn[3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            float L = -(s_fx[v][cy][cx + 1] - s_fx[v][cy][cx]) * d.rdx - (s_fy[v][cy + 1][cx] - s_fy[v][cy][cx]) * d.rdy;
            float o = a1 * (qf[(v * QS + cy + 3) * QS + cx + 3] + dt * L);
            if (a0 != 0.0f) o = a0 * (q0v ? q0v[v] : q0[idx + v * plane]) + o;
            out[idx + v * plane] = o;
            qn[v] = o;
        }
        const bool ok = qn[0] > 0.0f && __builtin_isfinite(qn[0]) && __builtin_isfinite(qn[1]) && __builtin_isfinite(qn[2]);
        bc = !ok;
    }
    if (count && nfb) atomicAdd(&s_cnt, nfb);
    if (bc) s_bad = 1;
    __syncthreads();
    if (tid == 0) {
        if (s_cnt) atomicAdd(d.nfb, (unsigned long long)s_cnt);
        if (s_bad) atomicOr(bad, STAGE);
    }
}

// Network pass and learned stage of one step's stage for the listed solves:
// workgroups stride over the lists' network tiles (FT x FT); each computes
// z on its tile and low halo and runs the learned stage on the tile, so the
// coefficients never leave LDS.  ntiles == 0: the tile count is read from the list
// header (nitems[1]; graph replay).  BL: the flux-limiter blend of the face
// fluxes (blend_flux).
template <int STAGE, bool BL = false>
__global__ __launch_bounds__(FNW * 64) void conv_learned_batch_kernel(const LSolve *__restrict__ tab,
                                                                      const LItem *__restrict__ items,
                                                                      const int *__restrict__ nitems, int ntiles,
                                                                      int one, const char *P, Packed pk, Norm nrm,
                                                                      Proj pr)
{
    constexpr int QS = FT + 6;
    __shared__ float s_qf[3 * QS * QS];
    const int total = ntiles > 0 ? ntiles : nitems[1];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const bool first = w == (int)blockIdx.x;
        if (!first) __syncthreads();  // the previous tile's LDS reads are done
        LItem it;
        if (one) {
            it = items[0];
        } else {
            const int n = *nitems;
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (items[mid].tb_cnn <= w) lo = mid;
                else hi = mid - 1;
            }
            it = items[lo];
        }
        const LSolve &d = tab[it.solve];
        const int tile = w - it.tb_cnn, tx_n = d.nx / FT;
        const int ty = tile / tx_n, tx = tile - ty * tx_n;
        const float dt = d.dt[0];  // its latency behind the network pass
        float *s_z = fused_tile<FT + 1, OUT_Z_LDS>(STAGE == 1 ? d.q : d.s1, P, pk, nrm, nullptr, d.ny, d.nx, ty * FT,
                                                   tx * FT, pr, first, s_qf);
        learned_epilogue<STAGE, BL>(d, it, s_z, s_qf, pr, tx * FT, ty * FT, dt);
    }
}

// One solve's learned stage in a launch of its own (network pass and learned
// stage per FT x FT tile, as conv_learned_batch_kernel; DIR: the direct
// face-state scheme on the network's raw output for the tile and a one-cell
// ring, the stage of learned_tile<0, HLLE, false, true>), the solve passed by
// value: d.q is the step's input, d.s2 the step's output (the other buffer of
// a pair, so the input survives for a redo).  Stage 1 with xprev != NULL:
// when the previous step's flag slot is set, every workgroup first redoes
// that step from xprev on the region it reads (redo_region, the result's
// tile written to d.q) and workgroup 0 counts the redo.  Stage 2's workgroup 0
// clears the previous step's slot (every reader of it has finished: the
// previous step's stage 2 and this step's stage 1) and advances the time.
template <int STAGE, bool BL = false, bool DIR = false, int TS = FT>
__global__ __launch_bounds__(FNW * 64) void conv_learned_one_kernel(LSolve d, int parity, const float *xprev,
                                                                    const char *P, Packed pk, Norm nrm, Proj pr)
{
    constexpr int QS = TS + 6;
    __shared__ float s_qf[3 * QS * QS];
    const int tx_n = d.nx / TS, total = tx_n * (d.ny / TS);
    const LItem it{0, 0, 0, parity, 0};
    float sig[3];  // DIR: the direct states' de-normalisation, 1 / inv_std (correctly rounded, as the host's)
#pragma unroll
    for (int v = 0; v < 3; v++) sig[v] = DIR ? 1.0f / nrm.inv_std[v] : 0.0f;
    PlainRedo rd;
    rd.xprev = STAGE == 1 ? xprev : nullptr;
    rd.flag = d.flags + (parity ^ 1);
    {
        rd.xk = d.q;
        rd.dt = d.dt;
        rd.rdx = d.rdx;
        rd.rdy = d.rdy;
        rd.ph.g = d.g;
        rd.ph.sqg = d.sqg;
        rd.ph.gamma = 1.4f;
        rd.ph.h0 = d.h0;
        rd.fatal = d.fatal;
    }
    const float dt0 = d.dt[0];  // read now, its latency behind the network pass
    // the grid never exceeds the tile count: every workgroup has a first
    // tile, whose loads need not wait for the loop test
    int w = blockIdx.x;
    do {
        const bool first = w == (int)blockIdx.x;
        if (!first) __syncthreads();  // the previous tile's LDS reads are done
        const int ty = w / tx_n, tx = w - ty * tx_n;
        // stage 2 on small tiles (register room): the cell's q^n loaded now,
        // its latency behind the network pass
        constexpr bool PRE = STAGE == 2 && TS == 4 && !DIR;
        float q0v[3] = {0.0f, 0.0f, 0.0f};
        if (PRE && threadIdx.x < TS * TS) {
            const int cy = threadIdx.x / TS, cx = threadIdx.x - cy * TS;
            const size_t idx = (size_t)(ty * TS + cy) * d.nx + tx * TS + cx, plane = (size_t)d.nx * d.ny;
#pragma unroll
            for (int v = 0; v < 3; v++) q0v[v] = d.q[idx + v * plane];
        }
        float *s_z = fused_tile<DIR ? TS + 2 : TS + 1, OUT_Z_LDS, 1, TS>(
            STAGE == 1 ? d.q : d.s1, P, pk, nrm, nullptr, d.ny, d.nx, ty * TS, tx * TS, pr, first, s_qf, &rd);
        learned_epilogue<STAGE, BL, DIR, TS>(d, it, s_z, s_qf, pr, tx * TS, ty * TS, dt0, sig, PRE ? q0v : nullptr);
        w += gridDim.x;
    } while (w < total);
    // no writer of the previous step's slot in stage 1
    if (STAGE == 1 && xprev && blockIdx.x == 0 && threadIdx.x == 0 && d.flags[parity ^ 1]) *d.redone += 1;
    if (STAGE == 2 && blockIdx.x == 0 && threadIdx.x == 0) {
        d.flags[parity ^ 1] = 0;
        if (d.t) {
            *d.t += (double)d.dt[0];
            *d.steps += 1;
        }
    }
}

int fused_max_grid()
{
    // resident workgroups of the tiled pass (one per CU: its LDS), per device
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int cus = 0, a = 0, b = 0, c = 0, e = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, conv_fused_kernel<true>, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, conv_fused_kernel<false>, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, conv_learned_batch_kernel<1>, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&e, conv_learned_batch_kernel<2>, FNW * 64, 0) != hipSuccess)
            return 256;
        int f = 0, h = 0, i = 0, j = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&f, conv_fused_batch_kernel<1>, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&h, conv_fused_batch_kernel<2>, FNW * 64, 0) != hipSuccess)
            return 256;
        // the blended forms (a second numerical flux per face) are launched
        // with the same cap
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&i, conv_learned_batch_kernel<1, true>, FNW * 64, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&j, conv_learned_batch_kernel<2, true>, FNW * 64, 0) !=
                hipSuccess)
            return 256;
        int k1 = 0, k2 = 0, k3 = 0, k4 = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k1, conv_learned_one_kernel<1>, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&k2, conv_learned_one_kernel<2>, FNW * 64, 0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&k3, conv_learned_one_kernel<1, true>, FNW * 64, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&k4, conv_learned_one_kernel<2, true>, FNW * 64, 0) !=
                hipSuccess)
            return 256;
        int k5 = 0, k6 = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k5, conv_learned_one_kernel<1, false, true>, FNW * 64, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&k6, conv_learned_one_kernel<2, false, true>, FNW * 64, 0) !=
                hipSuccess)
            return 256;
        k4 = k4 < k5 ? k4 : k5;
        k4 = k4 < k6 ? k4 : k6;
        // the single solve's 4 x 4 network tiles (launched with the same cap)
        int t[6] = {0, 0, 0, 0, 0, 0};
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&t[0], conv_learned_one_kernel<1, false, false, 4>, FNW * 64,
                                                         0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&t[1], conv_learned_one_kernel<2, false, false, 4>, FNW * 64,
                                                         0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&t[2], conv_learned_one_kernel<1, true, false, 4>, FNW * 64,
                                                         0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&t[3], conv_learned_one_kernel<2, true, false, 4>, FNW * 64,
                                                         0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&t[4], conv_learned_one_kernel<1, false, true, 4>, FNW * 64,
                                                         0) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&t[5], conv_learned_one_kernel<2, false, true, 4>, FNW * 64,
                                                         0) != hipSuccess)
            return 256;
        for (int i = 0; i < 6; i++) k4 = k4 < t[i] ? k4 : t[i];
        int m = a < b ? a : b;
        m = m < k1 ? m : k1;
        m = m < k2 ? m : k2;
        m = m < k3 ? m : k3;
        m = m < k4 ? m : k4;
        m = m < c ? m : c;
        m = m < e ? m : e;
        m = m < f ? m : f;
        m = m < h ? m : h;
        m = m < i ? m : i;
        m = m < j ? m : j;
        cache[dev] = (m > 0 ? m : 1) * (cus > 0 ? cus : 256);
    }
    return cache[dev];
}

hipError_t launch_forward_batch(int stage, const void *packed, const Norm &nrm, const Proj &pr, const LSolve *tab,
                                const LItem *items, const int *nitems, int ntiles, hipStream_t st, int one)
{
    if (ntiles <= 0) return hipSuccess;
    const Packed pk = packed_layout();
    const int cap = fused_max_grid(), g = ntiles < cap ? ntiles : cap;
    if (stage == 1)
        hipLaunchKernelGGL(conv_fused_batch_kernel<1>, dim3(g), dim3(FNW * 64), 0, st, tab, items, nitems, ntiles,
                           one, (const char *)packed, pk, nrm, pr);
    else
        hipLaunchKernelGGL(conv_fused_batch_kernel<2>, dim3(g), dim3(FNW * 64), 0, st, tab, items, nitems, ntiles,
                           one, (const char *)packed, pk, nrm, pr);
    return hipGetLastError();
}

hipError_t launch_forward_batch_list(int stage, const void *packed, const Norm &nrm, const Proj &pr,
                                     const LSolve *tab, const LItem *items, const int *list, int wgs,
                                     hipStream_t st)
{
    if (wgs <= 0) return hipErrorInvalidValue;
    const Packed pk = packed_layout();
    if (stage == 1)
        hipLaunchKernelGGL(conv_fused_batch_kernel<1>, dim3(wgs), dim3(FNW * 64), 0, st, tab, items, list, 0, 0,
                           (const char *)packed, pk, nrm, pr);
    else
        hipLaunchKernelGGL(conv_fused_batch_kernel<2>, dim3(wgs), dim3(FNW * 64), 0, st, tab, items, list, 0, 0,
                           (const char *)packed, pk, nrm, pr);
    return hipGetLastError();
}

hipError_t launch_conv_learned(int stage, const void *packed, const Norm &nrm, const Proj &pr, const LSolve *tab,
                               const LItem *items, const int *nitems, int ntiles, hipStream_t st, int one, int blend)
{
    if (ntiles <= 0) return hipSuccess;
    const Packed pk = packed_layout();
    const int cap = fused_max_grid(), g = ntiles < cap ? ntiles : cap;
    if (blend) {
        if (stage == 1)
            hipLaunchKernelGGL((conv_learned_batch_kernel<1, true>), dim3(g), dim3(FNW * 64), 0, st, tab, items, nitems,
                               ntiles, one, (const char *)packed, pk, nrm, pr);
        else
            hipLaunchKernelGGL((conv_learned_batch_kernel<2, true>), dim3(g), dim3(FNW * 64), 0, st, tab, items, nitems,
                               ntiles, one, (const char *)packed, pk, nrm, pr);
        return hipGetLastError();
    }
    if (stage == 1)
        hipLaunchKernelGGL(conv_learned_batch_kernel<1>, dim3(g), dim3(FNW * 64), 0, st, tab, items, nitems, ntiles,
                           one, (const char *)packed, pk, nrm, pr);
    else
        hipLaunchKernelGGL(conv_learned_batch_kernel<2>, dim3(g), dim3(FNW * 64), 0, st, tab, items, nitems, ntiles,
                           one, (const char *)packed, pk, nrm, pr);
    return hipGetLastError();
}

hipError_t launch_conv_learned_list(int stage, const void *packed, const Norm &nrm, const Proj &pr,
                                    const LSolve *tab, const LItem *items, const int *list, int wgs, hipStream_t st)
{
    if (wgs <= 0) return hipErrorInvalidValue;
    const Packed pk = packed_layout();
    if (stage == 1)
        hipLaunchKernelGGL(conv_learned_batch_kernel<1>, dim3(wgs), dim3(FNW * 64), 0, st, tab, items, list, 0, 0,
                           (const char *)packed, pk, nrm, pr);
    else
        hipLaunchKernelGGL(conv_learned_batch_kernel<2>, dim3(wgs), dim3(FNW * 64), 0, st, tab, items, list, 0, 0,
                           (const char *)packed, pk, nrm, pr);
    return hipGetLastError();
}

// One solve's kernels for tile side TS, grid g.
template <int TS>
static void launch_one_ts(int stage, int blend, int direct, int g, const char *Pc, const Packed &pk, const Norm &nrm,
                          const Proj &pr, const LSolve &d, int parity, const float *xprev, hipStream_t st)
{
    if (direct) {
        if (stage == 1)
            hipLaunchKernelGGL((conv_learned_one_kernel<1, false, true, TS>), dim3(g), dim3(FNW * 64), 0, st, d,
                               parity, xprev, Pc, pk, nrm, pr);
        else
            hipLaunchKernelGGL((conv_learned_one_kernel<2, false, true, TS>), dim3(g), dim3(FNW * 64), 0, st, d,
                               parity, xprev, Pc, pk, nrm, pr);
    } else if (blend) {
        if (stage == 1)
            hipLaunchKernelGGL((conv_learned_one_kernel<1, true, false, TS>), dim3(g), dim3(FNW * 64), 0, st, d,
                               parity, xprev, Pc, pk, nrm, pr);
        else
            hipLaunchKernelGGL((conv_learned_one_kernel<2, true, false, TS>), dim3(g), dim3(FNW * 64), 0, st, d,
                               parity, xprev, Pc, pk, nrm, pr);
    } else if (stage == 1) {
        hipLaunchKernelGGL((conv_learned_one_kernel<1, false, false, TS>), dim3(g), dim3(FNW * 64), 0, st, d, parity,
                           xprev, Pc, pk, nrm, pr);
    } else {
        hipLaunchKernelGGL((conv_learned_one_kernel<2, false, false, TS>), dim3(g), dim3(FNW * 64), 0, st, d, parity,
                           xprev, Pc, pk, nrm, pr);
    }
}

int learned_one_tile(int nx, int ny)
{
    if (nx % FT || ny % FT) return 0;
    // 4 x 4 tiles while they all get a resident workgroup: four times the
    // workgroups on small grids, each with about half the network work of
    // an 8 x 8 tile (the halo recompute grows, the latency falls)
    return (nx / 4) * (ny / 4) <= fused_max_grid() ? 4 : FT;
}

hipError_t launch_conv_learned_one(int stage, const void *packed, const Norm &nrm, const Proj &pr, const LSolve &d,
                                   int parity, const float *xprev, hipStream_t st, int blend, int direct)
{
    if (d.nx % FT || d.ny % FT || (parity & ~1) || (stage != 1 && stage != 2) || (stage == 2 && xprev) ||
        (blend && direct))
        return hipErrorInvalidValue;
    const Packed pk = packed_layout();
    const int ts = learned_one_tile(d.nx, d.ny);
    const int tiles = (d.nx / ts) * (d.ny / ts), cap = fused_max_grid(), g = tiles < cap ? tiles : cap;
    const char *Pc = (const char *)packed;
    if (ts == 4) launch_one_ts<4>(stage, blend, direct, g, Pc, pk, nrm, pr, d, parity, xprev, st);
    else launch_one_ts<FT>(stage, blend, direct, g, Pc, pk, nrm, pr, d, parity, xprev, st);
    return hipGetLastError();
}

hipError_t launch_forward_fused(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny, float *z,
                                hipStream_t st, const Proj *alpha)
{
    if (nx % FT || ny % FT) return hipErrorInvalidValue;
    const int tiles = B * (nx / FT) * (ny / FT), cap = fused_max_grid();
    const dim3 g(tiles < cap ? tiles : cap);
    if (alpha)
        hipLaunchKernelGGL(conv_fused_kernel<true>, g, dim3(FNW * 64), 0, st, q, (const char *)packed,
                           packed_layout(), nrm, z, B, ny, nx, *alpha);
    else
        hipLaunchKernelGGL(conv_fused_kernel<false>, g, dim3(FNW * 64), 0, st, q, (const char *)packed,
                           packed_layout(), nrm, z, B, ny, nx, Proj{});
    return hipGetLastError();
}

}  // namespace cnn

// ================================================================ backward
namespace cnn {

// Network input as the forward rounds it: x0 = bf16((q - mean) * inv_std),
// NHWC with 16 channels (3 used) for the layer-0 weight gradient.
template <int C, typename NormT>
__global__ void x0_kernel(const float *q, bf16 *x0, int B, int H, int W, NormT nrm)
{
    const long hw = (long)H * W, npix = (long)B * hw;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < npix * 16; i += (long)gridDim.x * blockDim.x) {
        long p = i / 16;
        int c = (int)(i - p * 16);
        long b = p / hw, r = p - b * hw;
        float v = c < C ? (q[(b * C + c) * hw + r] - nrm.mean[c]) * nrm.inv_std[c] : 0.0f;
        x0[i] = (bf16)v;
    }
}

// Input gradient of the first layer: dx0[p] = sum_t Wt[t] G[p + d_t] with the
// transposed, tap-flipped weights (16 output rows, 3 used), one 16-pixel
// group per wave; adds dq[c] += dx0[c] * inv_std[c] into the FP32 planar
// state gradient.
template <int C, typename NormT>
__global__ __launch_bounds__(256) void conv_dgrad_input_kernel(const bf16 *G, const bf16 *wt, float *dq, int B, int H,
                                                               int W, NormT nrm)
{
    constexpr int WEL = 9 * 16 * 32;
    __shared__ bf16x8 s_w[WEL / 8];
    const bf16x8 *gw = (const bf16x8 *)wt;
    for (int i = threadIdx.x; i < WEL / 8; i += 256) s_w[i] = gw[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, px = lane & 15;
    const long npix = (long)B * H * W;
    const long p0 = ((long)blockIdx.x * 4 + wave) * 16;
    if (p0 >= npix) return;
    const long p = p0 + px;
    const int hw = H * W;
    const int b = (int)(p / hw);
    const int rem = (int)(p - (long)b * hw);
    const int y = rem / W, x = rem - y * W;
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
    const bf16 *gb = G + (size_t)b * hw * 32;
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        int yy = wrap(y + tap / 3 - 1, H), xx = wrap(x + tap % 3 - 1, W);
        const bf16x8 bx = *(const bf16x8 *)(gb + (size_t)(yy * W + xx) * 32 + 8 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[(tap * 16 + px) * 4 + g], bx, acc, 0, 0, 0);
    }
    if (g == 0) {
#pragma unroll
        for (int c = 0; c < C; c++) dq[((size_t)b * C + c) * hw + rem] += acc[c] * nrm.inv_std[c];
    }
}

// Weight and bias gradient of a convolution over one 16 x 16 tile of pixels
// of one solve per workgroup:
//   dW[t][co][ci] += sum_p G[p][co] In[p + d_t][ci],  db[co] += sum_p G[p][co].
// MFMA with K = the tile's pixels, two tile rows (32 pixels) per step.  The
// workgroup stages G transposed ([co][256 pixels]) and the input's 18-row
// halo transposed three times, shifted by dx = -1, 0, +1 ([dx][ci][18 rows]
// [16 columns]), so that for every tap the operand fragment (eight pixels of
// one row, one channel) is one aligned 16-byte LDS read and every input pixel
// is loaded once per tile instead of once per tap.  A staging job loads eight
// (G) or ten (input: the union of the three shifts) consecutive pixels' eight
// channels and transposes them in registers.  Rows past ny contribute nothing
// (their G is staged as zero).  The bias is one more MFMA per co tile against
// a fragment whose column 0 is all ones.  Each workgroup writes its partial
// sums; a fixed-order reduction adds the partials of all workgroups.
template <int CO_T, int CI>
struct WgradShape {
    static constexpr int NCO = CO_T * 16;
    static constexpr int JI = (HT + 2) * 2 * (CI / 8);   // input jobs: halo row, column octet, channel octet
    static constexpr int JG = HT * 2 * (NCO / 8);        // G jobs: tile row, column octet, channel octet
    static constexpr int SLOTS = (JI + JG + 255) / 256;
    static constexpr int GLD = HT * HT + 8;              // G^T row stride (BF16)
    static constexpr int ILD = (HT + 2) * HT + 8;        // input^T stride per (shift, channel) (BF16)
    static constexpr int PER = 9 * NCO * CI + NCO;       // partial floats per workgroup
};

template <int CG, int CO_T, int CI>
__global__ __launch_bounds__(256) void wgrad_kernel(const bf16 *G, const bf16 *In, int H, int W, float *partial)
{
    using S = WgradShape<CO_T, CI>;
    constexpr int CI_T = CI / 16, NCO = S::NCO, JI = S::JI, JG = S::JG, SLOTS = S::SLOTS;
    constexpr int GLD = S::GLD, ILD = S::ILD;
    constexpr int NTILE = CO_T * CI_T;
    constexpr int TPW = (NTILE + 3) / 4;
    __shared__ bf16x8 sG[NCO * GLD / 8];
    __shared__ bf16x8 sI[3 * CI * ILD / 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int x0 = blockIdx.x * HT, y0 = blockIdx.y * HT, b = blockIdx.z;
    const size_t hw = (size_t)H * W;

    // staging: loads first, then the transposes and LDS writes
    bf16x8 v[SLOTS][10];
#pragma unroll
    for (int s = 0; s < SLOTS; s++) {
        const int j = tid + 256 * s;
        if (j < JI) {
            const int c8 = j % (CI / 8), q = (j / (CI / 8)) & 1, h = j / (2 * (CI / 8));
            int yy = y0 - 1 + h;
            yy = yy < 0 ? yy + H : yy % H;
            const bf16 *row = In + ((size_t)b * hw + (size_t)yy * W) * CI + c8 * 8;
            const int xs = x0 + 8 * q - 1;  // first of the ten columns
#pragma unroll
            for (int i = 0; i < 10; i++) v[s][i] = *(const bf16x8 *)(row + (size_t)wrap(xs + i, W) * CI);
        } else if (j < JI + JG) {
            const int jj = j - JI;
            const int c8 = jj % (NCO / 8), q = (jj / (NCO / 8)) & 1, r = jj / (2 * (NCO / 8));
            if (y0 + r < H) {
                const bf16 *src = G + ((size_t)b * hw + (size_t)(y0 + r) * W + x0 + 8 * q) * CG + c8 * 8;
#pragma unroll
                for (int i = 0; i < 8; i++) v[s][i] = *(const bf16x8 *)(src + (size_t)i * CG);
            } else {
#pragma unroll
                for (int i = 0; i < 8; i++)
#pragma unroll
                    for (int e = 0; e < 8; e++) v[s][i][e] = (bf16)0.0f;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < SLOTS; s++) {
        const int j = tid + 256 * s;
        if (j < JI) {
            const int c8 = j % (CI / 8), q = (j / (CI / 8)) & 1, h = j / (2 * (CI / 8));
#pragma unroll
            for (int d = 0; d < 3; d++)
#pragma unroll
                for (int c = 0; c < 8; c++) {
                    bf16x8 w;
#pragma unroll
                    for (int i = 0; i < 8; i++) w[i] = v[s][i + d][c];
                    sI[((d * CI + c8 * 8 + c) * ILD + h * HT + 8 * q) / 8] = w;
                }
        } else if (j < JI + JG) {
            const int jj = j - JI;
            const int c8 = jj % (NCO / 8), q = (jj / (NCO / 8)) & 1, r = jj / (2 * (NCO / 8));
#pragma unroll
            for (int c = 0; c < 8; c++) {
                bf16x8 w;
#pragma unroll
                for (int i = 0; i < 8; i++) w[i] = v[s][i][c];
                sG[((c8 * 8 + c) * GLD + r * HT + 8 * q) / 8] = w;
            }
        }
    }
    __syncthreads();

    floatx4 acc[TPW][9], accb[TPW];
#pragma unroll
    for (int j = 0; j < TPW; j++) {
        accb[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; t++) acc[j][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; e++) ones[e] = (bf16)(r16 == 0 ? 1.0f : 0.0f);
    // lane (r16, g) of step ks: tile row 2 ks + (g >> 1), columns 8 (g & 1) .. +7
#pragma unroll
    for (int j = 0; j < TPW; j++) {
        const int id = wave + 4 * j;
        if (id < NTILE) {
            const int cot = id / CI_T, cit = id - cot * CI_T;
            for (int ks = 0; ks < HT / 2; ks++) {
                const int r = 2 * ks + (g >> 1), cq = 8 * (g & 1);
                const bf16x8 af = sG[((cot * 16 + r16) * GLD + r * HT + cq) / 8];
                bf16x8 bf[9];
#pragma unroll
                for (int t = 0; t < 9; t++)
                    bf[t] = sI[(((t % 3) * CI + cit * 16 + r16) * ILD + (r + t / 3) * HT + cq) / 8];
#pragma unroll
                for (int t = 0; t < 9; t++)
                    acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[t], acc[j][t], 0, 0, 0);
                if (cit == 0) accb[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, ones, accb[j], 0, 0, 0);
            }
        }
    }
    // partial layout: [9][NCO][CI] then [NCO] bias
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float *pp = partial + (size_t)blk * S::PER;
#pragma unroll
    for (int j = 0; j < TPW; j++) {
        const int id = wave + 4 * j;
        if (id < NTILE) {
            const int cot = id / CI_T, cit = id - cot * CI_T;
#pragma unroll
            for (int t = 0; t < 9; t++)
#pragma unroll
                for (int i = 0; i < 4; i++)
                    pp[((size_t)t * NCO + cot * 16 + 4 * g + i) * CI + cit * 16 + r16] = acc[j][t][i];
            if (cit == 0 && r16 == 0) {
#pragma unroll
                for (int i = 0; i < 4; i++) pp[9 * NCO * CI + cot * 16 + 4 * g + i] = accb[j][i];
            }
        }
    }
}

// grads[W_l, b_l] += sum over blocks of the partials.  A workgroup owns 64
// consecutive entries; its wave w sums the partials of blocks w, w + 16,
// w + 32, ... in that order and wave 0 adds the sixteen wave sums in wave
// order: the order is fixed, independent of scheduling.
constexpr int RED_WAVES = 16;
__global__ __launch_bounds__(RED_WAVES * 64) void wgrad_reduce_kernel(const float *partial, int nblocks, int NCO,
                                                                      int CI, int co_real, int ci_real, int woff,
                                                                      int boff, float *grads)
{
    __shared__ float red[RED_WAVES][64];
    const int per = 9 * NCO * CI + NCO;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (e < per) {
#pragma unroll 4
        for (int k = wave; k < nblocks; k += RED_WAVES) s += partial[(size_t)k * per + e];
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave != 0 || e >= per) return;
    float t = 0.0f;
#pragma unroll
    for (int w = 0; w < RED_WAVES; w++) t += red[w][lane];
    int co, ci = 0, tap = 0;
    const bool isb = e >= 9 * NCO * CI;
    if (isb) {
        co = e - 9 * NCO * CI;
    } else {
        tap = e / (NCO * CI);
        int r = e - tap * NCO * CI;
        co = r / CI;
        ci = r - co * CI;
    }
    if (co >= co_real || ci >= ci_real) return;
    if (isb) grads[boff + co] += t;
    else grads[woff + (co * ci_real + ci) * 9 + tap] += t;
}

static dim3 wgrad_grid(int B, int nx, int ny) { return dim3((unsigned)(nx / HT), (unsigned)((ny + HT - 1) / HT), (unsigned)B); }

size_t backward_scratch_bytes(int B, int nx, int ny)
{
    long npix = (long)B * nx * ny;
    const dim3 wg = wgrad_grid(B, nx, ny);
    size_t part = (size_t)wg.x * wg.y * wg.z * WgradShape<5, 32>::PER * 4;
    return 2 * al256(npix * 32 * 2) + al256(npix * 16 * 2) + al256(part);
}

template <int CG, int CO_T, int CI>
static void wgrad(const bf16 *G, const bf16 *In, int B, int H, int W, float *partial, int co_real, int ci_real,
                  int woff, int boff, float *grads, hipStream_t st)
{
    const dim3 wg = wgrad_grid(B, W, H);
    const int nblocks = (int)(wg.x * wg.y * wg.z);
    hipLaunchKernelGGL((wgrad_kernel<CG, CO_T, CI>), wg, dim3(256), 0, st, G, In, H, W, partial);
    const int per = WgradShape<CO_T, CI>::PER;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((per + 63) / 64), dim3(RED_WAVES * 64), 0, st, (const float *)partial,
                       nblocks, CO_T * 16, CI, co_real, ci_real, woff, boff, grads);
}

hipError_t launch_backward(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny,
                           void *const acts[4], const void *dzv, float *dq, float *grads, void *scratch,
                           hipStream_t st)
{
    const Packed pk = packed_layout();
    const MasterLayout ml = master_layout();
    const char *P = (const char *)packed;
    const long npix = (long)B * nx * ny;
    // the halo-tile kernels take 16-pixel-wide tiles
    if (nx % HT) return hipErrorInvalidValue;
    const bf16 *dz = (const bf16 *)dzv;
    char *sc = (char *)scratch;
    bf16 *dA = (bf16 *)sc;
    sc += al256(npix * 32 * 2);
    bf16 *dB = (bf16 *)sc;
    sc += al256(npix * 32 * 2);
    bf16 *x0 = (bf16 *)sc;
    sc += al256(npix * 16 * 2);
    float *partial = (float *)sc;
    const bf16 *a[4] = {(const bf16 *)acts[0], (const bf16 *)acts[1], (const bf16 *)acts[2], (const bf16 *)acts[3]};
    unsigned eg = (unsigned)((npix * 16 + 255) / 256);
    if (eg > 8192) eg = 8192;
    dim3 cg((unsigned)((npix + 63) / 64)), blk(256);

    // layer 4: 32 -> 72
    wgrad<96, 5, 32>(dz, a[3], B, ny, nx, partial, 72, 32, ml.w[4], ml.b[4], grads, st);
    launch_halo<3, 2, 2>(dz, (const bf16 *)(P + pk.wt[4]), nullptr, a[3], (void *)dA, B, nx, ny, st);
    // layers 3, 2, 1: 32 -> 32
    bf16 *cur = dA, *nxt = dB;
    for (int l = 3; l >= 1; l--) {
        wgrad<32, 2, 32>(cur, a[l - 1], B, ny, nx, partial, 32, 32, ml.w[l], ml.b[l], grads, st);
        launch_halo<1, 2, 2>(cur, (const bf16 *)(P + pk.wt[l]), nullptr, a[l - 1], (void *)nxt, B, nx, ny, st);
        bf16 *t = cur;
        cur = nxt;
        nxt = t;
    }
    // layer 0: 3 -> 32 (input rebuilt as the forward rounds it)
    hipLaunchKernelGGL((x0_kernel<3, Norm>), dim3(eg), blk, 0, st, q, x0, B, ny, nx, nrm);
    wgrad<32, 2, 16>(cur, x0, B, ny, nx, partial, 32, 3, ml.w[0], ml.b[0], grads, st);
    hipLaunchKernelGGL((conv_dgrad_input_kernel<3, Norm>), cg, blk, 0, st, (const bf16 *)cur,
                       (const bf16 *)(P + pk.wt[0]), dq, B, ny, nx, nrm);
    return hipGetLastError();
}

size_t backward_scratch_bytes_euler(int B, int nx, int ny)
{
    long npix = (long)B * nx * ny;
    const dim3 wg = wgrad_grid(B, nx, ny);
    size_t part = (size_t)wg.x * wg.y * wg.z * WgradShape<6, 32>::PER * 4;
    return 2 * al256(npix * 32 * 2) + al256(npix * 16 * 2) + al256(part);
}

// The planar network's backward on the Euler network's shapes: layer 4
// 32 -> 96 (six co tiles, dz read as three 32-channel K blocks), layer 0
// 4 -> 32.
hipError_t launch_backward_euler(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                 void *const acts[4], const void *dzv, float *dq, float *grads, void *scratch,
                                 hipStream_t st)
{
    const EPacked pk = euler_packed_layout();
    const EMaster ml = euler_master();
    const char *P = (const char *)packed;
    const long npix = (long)B * nx * ny;
    if (nx % HT) return hipErrorInvalidValue;
    const bf16 *dz = (const bf16 *)dzv;
    char *sc = (char *)scratch;
    bf16 *dA = (bf16 *)sc;
    sc += al256(npix * 32 * 2);
    bf16 *dB = (bf16 *)sc;
    sc += al256(npix * 32 * 2);
    bf16 *x0 = (bf16 *)sc;
    sc += al256(npix * 16 * 2);
    float *partial = (float *)sc;
    const bf16 *a[4] = {(const bf16 *)acts[0], (const bf16 *)acts[1], (const bf16 *)acts[2], (const bf16 *)acts[3]};
    unsigned eg = (unsigned)((npix * 16 + 255) / 256);
    if (eg > 8192) eg = 8192;
    dim3 cg((unsigned)((npix + 63) / 64)), blk(256);

    wgrad<E_COUT, 6, 32>(dz, a[3], B, ny, nx, partial, E_COUT, 32, ml.w[4], ml.b[4], grads, st);
    launch_halo<3, 2, 2>(dz, (const bf16 *)(P + pk.wt[4]), nullptr, a[3], (void *)dA, B, nx, ny, st);
    bf16 *cur = dA, *nxt = dB;
    for (int l = 3; l >= 1; l--) {
        wgrad<32, 2, 32>(cur, a[l - 1], B, ny, nx, partial, 32, 32, ml.w[l], ml.b[l], grads, st);
        launch_halo<1, 2, 2>(cur, (const bf16 *)(P + pk.wt[l]), nullptr, a[l - 1], (void *)nxt, B, nx, ny, st);
        bf16 *t = cur;
        cur = nxt;
        nxt = t;
    }
    hipLaunchKernelGGL((x0_kernel<E_CIN, ENorm>), dim3(eg), blk, 0, st, q, x0, B, ny, nx, nrm);
    wgrad<32, 2, 16>(cur, x0, B, ny, nx, partial, 32, E_CIN, ml.w[0], ml.b[0], grads, st);
    hipLaunchKernelGGL((conv_dgrad_input_kernel<E_CIN, ENorm>), cg, blk, 0, st, (const bf16 *)cur,
                       (const bf16 *)(P + pk.wt[0]), dq, B, ny, nx, nrm);
    return hipGetLastError();
}

}  // namespace cnn
