// Internal interface of the stencil-coefficient network and the learned step.
//
// Network (thesis section 2.5.3, fourth approach): five 3x3 convolutions
// 3 -> 32 -> 32 -> 32 -> 32 -> 72 with ReLU between layers and periodic
// padding; BF16 weights and activations, FP32 accumulation on MFMA.
//
// Master parameters (FP32, owned by the caller), layer by layer:
//   W_l[co][ci][ky][kx] then b_l[co]; 49 448 floats in total.
// Packed layout used by the kernels (BF16 weights, FP32 biases):
//   layer 0  : [32 co][32 k]          k = tap*3 + ci (k >= 27 zero)
//   layer 1-3: [9 tap][32 co][32 ci]
//   layer 4  : [9 tap][80 co][32 ci]  (co >= 72 zero)
//   tap = ky*3 + kx reads the input at (y + ky - 1, x + kx - 1).
// Transposed, tap-flipped copies drive the input-gradient convolutions:
//   layer l > 0: [9 tap][CI_PAD co'][CO_PAD ci'] with W'[t][ci][co] = W[co][ci][8-t]
// Activations: NHWC, [solve][y][x][32] BF16.  Raw coefficients z:
//   [solve][y][x][72] FP32, channel ((axis*2 + side)*3 + var)*6 + k.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cnn {

constexpr int CIN = 3, CH = 32, COUT = 72, COUT_PAD = 80, NL = 5;
constexpr int NPARAM = (32 * 3 * 9 + 32) + 3 * (32 * 32 * 9 + 32) + (72 * 32 * 9 + 72);
static_assert(NPARAM == 49448, "parameter count");

// Offsets (in floats) of W_l and b_l inside the master parameter vector.
struct MasterLayout {
    int w[NL], b[NL];
};
MasterLayout master_layout();

struct Packed {
    // byte offsets inside the packed buffer
    size_t w[NL];      // forward weights (bf16)
    size_t wt[NL];     // transposed/flipped weights for input gradients (bf16), layers 1..4
    size_t b[NL];      // biases (fp32)
    size_t bytes;
};
Packed packed_layout();

struct Norm {
    float mean[3], inv_std[3];
};

// Constraint data for the learned reconstruction: alpha = base + P z per
// group of six coefficients (side 0 = left state, side 1 = right state).
struct Proj {
    float P[36];     // row-major 6x6
    float base[12];  // [side][k]
};

// Pack FP32 master parameters into the kernel layouts.
hipError_t launch_pack(const float *master, void *packed, hipStream_t st);

// Forward of B solves of size ny x nx (nx % 16 == 0, ny*nx % 64 == 0).
//   q    : [B][3][ny][nx] FP32 states;
//   acts : 4 activation buffers [B][ny][nx][32] BF16 (outputs of layers 0..3);
//          acts[k] may alias acts[k-2] when activations are not kept;
//   z    : [B][ny][nx][72] FP32.
hipError_t launch_forward(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny,
                          void *const acts[4], float *z, hipStream_t st);

}  // namespace cnn
