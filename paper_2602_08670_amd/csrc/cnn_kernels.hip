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

// MODE 0: first layer, input = states (FP32 planar) normalised and rounded
//         to BF16 on the fly, K = 27 (tap*3 + ci) padded to 32;
// MODE 1: hidden layer, NHWC BF16 in and out (bias, ReLU, round to BF16);
// MODE 2: last layer, 72 FP32 outputs (bias only).
template <int MODE>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const void *in, const bf16 *wp, const float *bias, void *out,
                                                       int B, int H, int W, Norm nrm)
{
    constexpr int NT = MODE == 2 ? 5 : 2;
    constexpr int WEL = MODE == 0 ? 32 * 32 : 9 * NT * 16 * 32;
    __shared__ bf16x8 s_w[WEL / 8];
    const bf16x8 *gw = (const bf16x8 *)wp;
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

    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};

    if (MODE == 0) {
        const float *q = (const float *)in + (size_t)b * 3 * hw;
        bf16x8 bx;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            int k = 8 * g + e;
            float v = 0.0f;
            if (k < 27) {
                int tap = k / 3, ci = k - 3 * tap;
                int yy = wrap(y + tap / 3 - 1, H), xx = wrap(x + tap % 3 - 1, W);
                v = (q[(size_t)ci * hw + yy * W + xx] - nrm.mean[ci]) * nrm.inv_std[ci];
            }
            bx[e] = (bf16)v;
        }
#pragma unroll
        for (int t = 0; t < NT; t++)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[(t * 16 + px) * 4 + g], bx, acc[t], 0, 0, 0);
    } else {
        const bf16 *act = (const bf16 *)in + (size_t)b * hw * 32;
#pragma unroll
        for (int tap = 0; tap < 9; tap++) {
            int yy = wrap(y + tap / 3 - 1, H), xx = wrap(x + tap % 3 - 1, W);
            bf16x8 bx = *(const bf16x8 *)(act + (size_t)(yy * W + xx) * 32 + 8 * g);
#pragma unroll
            for (int t = 0; t < NT; t++)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[((tap * NT + t) * 16 + px) * 4 + g], bx, acc[t],
                                                                 0, 0, 0);
        }
    }

#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int co0 = 16 * t + 4 * g;
        if (MODE < 2) {
            bf16x4 o;
#pragma unroll
            for (int i = 0; i < 4; i++) o[i] = (bf16)__builtin_fmaxf(acc[t][i] + bias[co0 + i], 0.0f);
            *(bf16x4 *)((bf16 *)out + (size_t)p * 32 + co0) = o;
        } else if (co0 < 72) {
            floatx4 o;
#pragma unroll
            for (int i = 0; i < 4; i++) o[i] = acc[t][i] + bias[co0 + i];
            *(floatx4 *)((float *)out + (size_t)p * 72 + co0) = o;
        }
    }
}

hipError_t launch_forward(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny,
                          void *const acts[4], float *z, hipStream_t st)
{
    const Packed pk = packed_layout();
    const char *P = (const char *)packed;
    const long npix = (long)B * nx * ny;
    dim3 grid((unsigned)((npix + 63) / 64)), blk(256);
    hipLaunchKernelGGL(conv_fwd_kernel<0>, grid, blk, 0, st, (const void *)q, (const bf16 *)(P + pk.w[0]),
                       (const float *)(P + pk.b[0]), acts[0], B, ny, nx, nrm);
    for (int l = 1; l < 4; l++)
        hipLaunchKernelGGL(conv_fwd_kernel<1>, grid, blk, 0, st, (const void *)acts[l - 1], (const bf16 *)(P + pk.w[l]),
                           (const float *)(P + pk.b[l]), acts[l], B, ny, nx, nrm);
    hipLaunchKernelGGL(conv_fwd_kernel<2>, grid, blk, 0, st, (const void *)acts[3], (const bf16 *)(P + pk.w[4]),
                       (const float *)(P + pk.b[4]), (void *)z, B, ny, nx, nrm);
    return hipGetLastError();
}

}  // namespace cnn
