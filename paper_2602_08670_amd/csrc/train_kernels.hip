// Training helpers: the unrolled loss of eq 2.28 with its gradient, and Adam.
#include "cnn_internal.hpp"

namespace cnn {

__global__ __launch_bounds__(256) void loss_kernel(const float *pred, const float *tgt, const float *scale3, int B,
                                                   int plane, float *G, double *partials, int nvar)
{
    __shared__ double s[256];
    const size_t n = (size_t)B * nvar * plane;
    const double inv_n = 1.0 / (double)n;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        int v = (int)((i / plane) % nvar);
        float sv = scale3[v];
        float d = pred[i] - tgt[i];
        double r = (double)d / sv;
        acc += r * r * inv_n;
        G[i] += (float)(2.0 * (double)d / ((double)sv * sv) * inv_n);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// loss_acc += sum of the block partials: thread i adds partials i, i + 256,
// ... in order, then a fixed tree over the 256 thread sums.
__global__ __launch_bounds__(256) void loss_final_kernel(const double *partials, int nblocks, double *loss_acc)
{
    __shared__ double s[256];
    double t = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) t += partials[b];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss_acc += s[0];
}

hipError_t launch_loss(const float *pred, const float *tgt, const float *scale3, int B, int nx, int ny, float *G,
                       double *partials, int max_blocks, double *loss_acc, hipStream_t st, int nvar)
{
    size_t n = (size_t)B * nvar * nx * ny;
    int blocks = (int)((n + 255) / 256);
    if (blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, st, pred, tgt, scale3, B, nx * ny, G, partials, nvar);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, (const double *)partials, blocks, loss_acc);
    return hipGetLastError();
}

__global__ void scale_kernel(float *out, const float *in, float a, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = a * in[i];
}

hipError_t launch_scale(float *out, const float *in, float a, size_t n, hipStream_t st)
{
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(scale_kernel, dim3(blocks), dim3(256), 0, st, out, in, a, n);
    return hipGetLastError();
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / bc1) / (sqrt(v / bc2) + eps), bc_k = 1 - b_k^t.
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float gi = g[i];
        float mi = b1 * m[i] + (1.0f - b1) * gi;
        float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (__builtin_sqrtf(vi / bc2) + eps);
    }
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t st)
{
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

__global__ void flags_or_kernel(const int *flags, int B, int *any)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B && flags[b]) atomicOr(any, 1);
}

hipError_t launch_flags_or(const int *flags, int B, int *any, hipStream_t st)
{
    hipLaunchKernelGGL(flags_or_kernel, dim3((B + 255) / 256), dim3(256), 0, st, flags, B, any);
    return hipGetLastError();
}

}  // namespace cnn

namespace cnn {

// Exact cell-average coarsening: coarse(I, J) = mean of the f x f fine block,
// accumulated in double precision in a fixed order.
__global__ void coarsen_kernel(const float *fine, int nvar, int nx, int ny, int f, float *coarse)
{
    const int cx = nx / f, cy = ny / f;
    const size_t n = (size_t)nvar * cx * cy;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        int v = (int)(i / ((size_t)cx * cy));
        int r = (int)(i - (size_t)v * cx * cy);
        int J = r / cx, I = r - J * cx;
        const float *src = fine + (size_t)v * nx * ny + (size_t)J * f * nx + (size_t)I * f;
        double acc = 0.0;
        for (int a = 0; a < f; a++)
            for (int b = 0; b < f; b++) acc += (double)src[(size_t)a * nx + b];
        coarse[i] = (float)(acc / ((double)f * f));
    }
}

hipError_t launch_coarsen(const float *fine, int nvar, int nx, int ny, int f, float *coarse, hipStream_t st)
{
    size_t n = (size_t)nvar * (nx / f) * (ny / f);
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(coarsen_kernel, dim3(blocks), dim3(256), 0, st, fine, nvar, nx, ny, f, coarse);
    return hipGetLastError();
}

}  // namespace cnn
