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

// Device descriptor of one learned solve (periodic nx x ny shallow water,
// flat bed, fixed Delta t) for the work-list kernels.
struct LSolve {
    float *q, *s1, *s2;      // state and stage buffers [3][n][n]
    float *z;                // constrained coefficients [n][n][72] of the separate network pass
    const float *dt;         // fixed step (device)
    int *flags;              // two per-step flag slots
    unsigned long long *nfb, *redone;
    int *fatal;              // the plain redo failed: the solve is frozen
    double *t;               // simulated time and step count
    long long *steps;
    int nx, ny;
    float rdx, rdy, g, sqg, h0;  // 1/dx, 1/dy, gravity, sqrt(g), pressure reference depth
    float pad;
};
// One solve of a step's list: its first workgroup in the network-pass and in
// the stage launches (prefix sums over the list), and which flag slot the
// step uses.
struct LItem {
    int solve, tb_cnn, tb_st, parity;
    int tb_h;  // first 16 x 16 tile in the layer-by-layer network pass's numbering
};
constexpr int LTILE_CNN = 8;            // network pass tile side
constexpr int LTILE_X = 32, LTILE_Y = 4;  // stage tile
inline int ltiles_cnn(int nx, int ny) { return (nx / LTILE_CNN) * (ny / LTILE_CNN); }
inline int ltiles_st(int nx, int ny) { return ((nx + LTILE_X - 1) / LTILE_X) * ((ny + LTILE_Y - 1) / LTILE_Y); }

// Work-list launches over the listed solves (one != 0: exactly one solve,
// tab[items[0].solve]).  Network pass: stage 1 reads q, stage 2 reads S1,
// both write alpha to z; its workgroups (at most fused_max_grid()) stride
// over the network tiles.  Learned stage: MODE 0 with stage 1 or 2 (reads
// alpha from z), MODE 2, 3 (as learned_stage), HLLE, over the stage tiles.
hipError_t launch_forward_batch(int stage, const void *packed, const Norm &nrm, const Proj &pr, const LSolve *tab,
                                const LItem *items, const int *nitems, int ntiles, hipStream_t st, int one = 0);
hipError_t launch_learned_batch(int mode, int stage, const LSolve *tab, const LItem *items, const int *nitems,
                                int ntiles, const Proj &pr, hipStream_t st, int one = 0);
// The forms recorded in graphs: wgs workgroups (set before each replay: the
// list's stage tiles, and for the network pass at most fused_max_grid()),
// the tile counts read from the list header list = {items, network tiles,
// stage tiles, 0}.
hipError_t launch_forward_batch_list(int stage, const void *packed, const Norm &nrm, const Proj &pr,
                                     const LSolve *tab, const LItem *items, const int *list, int wgs,
                                     hipStream_t st);
hipError_t launch_learned_batch_list(int mode, int stage, const LSolve *tab, const LItem *items, const int *list,
                                     int wgs, const Proj &pr, hipStream_t st);
// One layer (0..4) of the layer-by-layer network pass of the listed solves
// (nx, ny multiples of 16) on 16 x 16 tiles, wgs workgroups (the list
// header's fourth entry, 16 x 16 tiles): layer 0 reads q (stage 1) or S1
// (stage 2) into act0, layers 1..3 go act0 -> act1 -> act0 -> act1, layer 4
// writes alpha to each solve's z.  act0 and act1 hold [pixels][32] BF16,
// solve d's pixels at offset tb_h * 256.  The same alpha as
// launch_forward_batch_list.
hipError_t launch_layer_list(int layer, int stage, const void *packed, const Norm &nrm, const Proj &pr,
                             const LSolve *tab, const LItem *items, const int *list, int wgs, void *act0, void *act1,
                             hipStream_t st);
// Workgroups of the tiled network pass resident at once on the current
// device: its launches use at most this many, each striding over tiles and
// staging the weights once.
int fused_max_grid();
// Network pass and learned stage (MODE 0) of one stage in one launch over the
// listed solves' network tiles (the coefficients stay in LDS; nx, ny
// multiples of LTILE_CNN): stage 1 writes S1 from q, stage 2 writes S2 from
// S1 and q; the same results as the network pass followed by learned_stage
// MODE 0.  The list form is the one recorded in graphs (wgs set before each
// replay to at most fused_max_grid(), the network tile count read from the
// list header).  blend: the flux-limiter blend of the face fluxes (blend_flux).
hipError_t launch_conv_learned(int stage, const void *packed, const Norm &nrm, const Proj &pr, const LSolve *tab,
                               const LItem *items, const int *nitems, int ntiles, hipStream_t st, int one = 0,
                               int blend = 0);
hipError_t launch_conv_learned_list(int stage, const void *packed, const Norm &nrm, const Proj &pr,
                                    const LSolve *tab, const LItem *items, const int *list, int wgs, hipStream_t st);
// One solve's stage (HLLE) in one launch, the solve passed by value: stage 1
// reads d.q and writes d.s1, stage 2 reads d.s1 and d.q and writes d.s2 (the
// step's output, kept apart from its input); flags in slot d.flags[parity].
// Stage 1 with xprev (the previous step's input): when the previous step's
// slot d.flags[parity ^ 1] is set, the previous step is first redone with the
// plain scheme from xprev into d.q (counted in d.redone; an inadmissible
// plain result sets d.fatal).  Stage 2 clears the previous step's slot and
// advances d.t and d.steps.
// direct: the direct face-state scheme (raw output, face_states_direct) instead of the
// learned coefficients; blend: the flux-limiter blend of the learned fluxes.
hipError_t launch_conv_learned_one(int stage, const void *packed, const Norm &nrm, const Proj &pr, const LSolve &d,
                                   int parity, const float *xprev, hipStream_t st, int blend = 0, int direct = 0);

// The same forward in one launch, without keeping activations: every
// workgroup runs all five layers on an 8x8 tile of pixels (nx % 8 == 0,
// ny % 8 == 0); z is bit-identical to launch_forward's.  With alpha != NULL
// the output is the constrained coefficients base + P z per group of six
// instead of z.
hipError_t launch_forward_fused(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny, float *z,
                                hipStream_t st, const Proj *alpha = nullptr);

struct LearnedArgs;

// Launch wrappers of the learned stage (learned_kernels.hip).
struct StageBatch {
    const float *qs, *q0;
    float *out;
    const float *z;          // raw coefficients, or (alpha != 0) constrained ones, [B][ny][nx][72]
    int alpha;
    int B, nx, ny;
    float rdx, rdy, g, h0;
    float a0, a1;
    const float *dt;
    int *bad;                // per-solve flag bits: 1 = stage 1 failed, 2 = stage 2 failed
    int flagbit;             // bit this stage sets; stage 2 (flagbit 2) skips counting when bit 1 is set
    unsigned long long *nfb;
    int *fatal;
    Proj pr;
    // modes 2 and 3 (the end of a step in two launches instead of four):
    const float *commit_src;     // mode 2: S2, copied to commit_dst for admissible solves (NULL: no copy)
    float *commit_dst;
    int *bad_next;               // mode 3: the next step's flags, cleared
    unsigned long long *redone;  // mode 3: per solve, +1 when the step was redone (or NULL)
    double *t;                   // mode 3: solve 0's time and step count advance (or NULL)
    long long *steps;
    int direct;                  // mode 0: the direct face-state scheme (z raw, channels 0..11)
    float sig[3];                // direct: 1 / inv_std of the network's input normalisation
    int blend;                   // mode 0: flux-limiter blend of the learned fluxes (z raw)
};
// mode 0: learned stage with fallback (sets bad bits);
// mode 1: plain MINMOD stage, only for solves with bad != 0;
// mode 2: solves with bad == 0 commit S2 -> q, the others run the plain
//         first stage (redo);
// mode 3: plain second stage for solves with bad != 0, and the step's
//         bookkeeping (redone count, next flags cleared, time).
hipError_t learned_stage(int mode, int flux, const StageBatch &sb, hipStream_t st);
hipError_t launch_commit(float *q, const float *s2, const int *bad, size_t per_solve, int B, hipStream_t st);
hipError_t launch_finish(int *bad, unsigned long long *redone, int *record, int B, const float *dt, double *t,
                         long long *steps, hipStream_t st);

// Training helpers (train_kernels.hip).
// loss_acc += sum((pred - tgt)/s_v)^2 / N over the batch (N = B*3*ny*nx,
// FP64 fixed-order reduction) and G += 2 (pred - tgt) / (s_v^2 N).
hipError_t launch_loss(const float *pred, const float *tgt, const float *scale3, int B, int nx, int ny, float *G,
                       double *partials, int max_blocks, double *loss_acc, hipStream_t st, int nvar = 3);
hipError_t launch_scale(float *out, const float *in, float a, size_t n, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t st);
hipError_t launch_flags_or(const int *flags, int B, int *any, hipStream_t st);
hipError_t launch_coarsen(const float *fine, int nvar, int nx, int ny, int f, float *coarse, hipStream_t st);

// Reverse pass of one learned stage (adjoint_kernels.hip): writes
// gqs = (accumulate ? gqs : 0) + a1*gout + (FV part of the adjoint), and dz,
// the adjoint of the raw coefficients z of this stage rounded to BF16 in the
// network backward's layout.
struct AdjStage {
    const float *qs, *z, *gout;
    float a1, dt;
    int B, nx, ny;
    float rdx, rdy, g, h0;
    Proj pr;
    const int *plain;  // per solve: the step ran the plain scheme (or NULL)
    float *contrib;    // scratch [2][B][ny][nx][ADJ_REC]
    void *dz;          // [B][ny][nx][DZ_CH] BF16: channels 0..71 written, the rest left as they are (zero)
    float *gqs;
    int accumulate;
    int direct;        // the direct face-state scheme (dz channels 0..11 written, the rest left zero)
    float sig[3];      // direct: 1 / inv_std of the network's input normalisation
    int blend;         // the flux-limiter blend of the learned face fluxes
};
hipError_t launch_adjoint(int flux, const AdjStage &s, hipStream_t st);
// Floats per face in the adjoint's contribution scratch: 18 used, padded so
// that a record is whole 16-byte vectors.
constexpr int ADJ_REC = 20;
// Channels per pixel of dz: the 72 coefficients padded to three 32-channel K
// blocks of the layer-4 input-gradient convolution.
constexpr int DZ_CH = 96;

// Backward of the network for B solves: adds d loss / d theta into grads
// (master layout, FP32) and d loss / d q into dq ([B][3][ny][nx], FP32),
// given dz = d loss / d z (BF16 [p][DZ_CH], channels >= 72 zero) and the
// activations saved by the forward.
size_t backward_scratch_bytes(int B, int nx, int ny);
hipError_t launch_backward(const void *packed, const Norm &nrm, const float *q, int B, int nx, int ny,
                           void *const acts[4], const void *dz, float *dq, float *grads, void *scratch,
                           hipStream_t st);

// ------------------------------------------------------------------------
// Network of the learned Euler step (the same stack on the four conserved
// variables): 4 -> 32 -> 32 -> 32 -> 32 -> 96, z channel
// ((axis*2 + side)*4 + var)*6 + k.  Master layout as the planar network's
// (W_l[co][ci][ky][kx] then b_l, layer by layer; 56 672 floats).  Packed:
//   layer 0  : [32 co][64 k]          k = tap*4 + ci (k >= 36 zero)
//   layer 1-3: [9 tap][32 co][32 ci]  (as the planar network)
//   layer 4  : [9 tap][96 co][32 ci]
//   biases FP32 (32, 32, 32, 32, 96);
// and the transposed, tap-flipped copies of the input-gradient
// convolutions: layer 0 [9][16 ci (4 used)][32 co], layers 1-3
// [9][32 ci][32 co], layer 4 [9][32 ci][96 co].
constexpr int E_CIN = 4, E_COUT = 96;
constexpr int E_NPARAM = (32 * 4 * 9 + 32) + 3 * (32 * 32 * 9 + 32) + (96 * 32 * 9 + 96);
static_assert(E_NPARAM == 56672, "Euler network parameter count");
struct EPacked {
    size_t w[NL], wt[NL], b[NL], bytes;
};
EPacked euler_packed_layout();
struct ENorm {
    float mean[4], inv_std[4];
};
hipError_t launch_pack_euler(const float *master, void *packed, hipStream_t st);
// Forward of B solves [B][4][ny][nx] (nx % 16 == 0): act0, act1 are two
// activation buffers [B][ny][nx][32] BF16 (ping-pong), z [B][ny][nx][96] FP32.
hipError_t launch_forward_euler(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                void *act0, void *act1, float *z, hipStream_t st);
// The same forward in one launch (nx % 8 == 0, ny % 8 == 0): every
// workgroup runs all five layers on 8 x 8 tiles in LDS; z is bit-identical.
hipError_t launch_forward_euler_fused(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                      float *z, hipStream_t st);
// The same forward keeping every layer's activation (acts[0..3], each
// [B][ny][nx][32] BF16) for the backward.
hipError_t launch_forward_euler_keep(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                     void *const acts[4], float *z, hipStream_t st);
// Backward of the Euler network: grads (master layout) += d loss / d theta,
// dq ([B][4][ny][nx]) += d loss / d q, given dz (BF16 [p][96]) and the
// activations of launch_forward_euler_keep.
size_t backward_scratch_bytes_euler(int B, int nx, int ny);
hipError_t launch_backward_euler(const void *packed, const ENorm &nrm, const float *q, int B, int nx, int ny,
                                 void *const acts[4], const void *dz, float *dq, float *grads, void *scratch,
                                 hipStream_t st);

// Projector onto the null space of the moment conditions of the given order
// (exactness for cell averages of polynomials of degree <= order) and Fromm's
// base stencils.
Proj make_projection(int order);

}  // namespace cnn
