// Internal interface of the learned Euler step (euler_learned_kernels.hip,
// euler_learned_api.cpp).  States [B][4][ny][nx] FP32, periodic; raw
// network coefficients [B][ny][nx][96] FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "cnn_internal.hpp"

namespace eln {

struct StageArgs {
    const float *qs, *q0;  // stage input; q0 for the a0 term
    float *out;
    const float *z;        // MODE 0: raw coefficients
    int B, nx, ny;
    float rdx, rdy, gamma, dt, a0, a1;
    int *flags;            // [B][2]: flag bits of the step (1: stage 1 failed, 2: stage 2 failed)
    int parity;            // the step's slot
    int flagbit;           // MODE 0: the bit this stage sets
    unsigned long long *nfb, *redone;
    int *fatal;            // [B]: the plain redo failed, the solve is frozen
    cnn::Proj pr;
    const float *commit_src;  // MODE 2: S2 (NULL: the result is in place, nothing to copy)
    float *commit_dst;        // MODE 2: q
    int *record;              // MODE 3 (or NULL): per solve, 1 when this step was redone (training)
};

hipError_t stage(int mode, int flux, const StageArgs &a, hipStream_t st);

// Reverse pass of one learned stage (training): gqs = (accumulate ? gqs :
// 0) + a1 gout + the finite-volume part of the adjoint, and dz, the
// adjoint of the stage's raw coefficients as BF16 [B][ny][nx][96].
constexpr int ADJ_REC = 24;  // floats per face in the contribution scratch (4 variables x 6 cells)
struct AdjArgs {
    const float *qs;    // stage input [B][4][ny][nx]
    const float *z;     // raw coefficients of the stage [B][ny][nx][96]
    const float *gout;  // adjoint of the stage output
    float wscale;       // a1 dt
    int B, nx, ny;
    float rdx, rdy, gamma;
    cnn::Proj pr;
    const int *plain;   // per solve: the step ran the plain scheme (or NULL)
    float *contrib;     // [2][B][ny][nx][ADJ_REC]
    __bf16 *dz;         // [B][ny][nx][96]
};
hipError_t adjoint(int flux, const AdjArgs &a, float *gqs, float a1, int accumulate, hipStream_t st);

}  // namespace eln

namespace cnn {
// The network pass and the learned stage (MODE 0 of eln::stage, the same
// arithmetic) of one stage in one launch, for grids of whole 8 x 8 tiles:
// a.qs is the stage input and the network's, the coefficients stay in LDS
// (a.z unused); a.flagbit is the stage (1 or 2).
// xprev (stage 1, or NULL): the previous step's input; a solve whose
// previous step is flagged (a.flags[2b + (a.parity ^ 1)]) is first redone
// with the plain scheme from xprev, on the region each workgroup reads, into
// a.qs (counted in a.redone; an inadmissible plain result freezes the solve).
// Stage 2 clears the previous step's slot of each solve it steps.
hipError_t launch_learned_euler(int flux, const void *packed, const ENorm &nrm, const eln::StageArgs &a,
                                hipStream_t st, const float *xprev = nullptr);
// Workgroups of the one-launch Euler network pass resident at once.
int fused_euler_grid();
}  // namespace cnn
