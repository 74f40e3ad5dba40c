// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace fvk {

// Device control block of one solve (lives in the caller's workspace).
struct Ctl {
    double t;             // simulated time
    long long step;       // completed steps
    int bad;              // a step produced an inadmissible cell
    int pad0;
    unsigned long long pad1[5];
};
static_assert(sizeof(Ctl) == 64, "control block layout");

// CFL rate slots.  Slot k holds RATE_SUB sub-slots, each the bits of a
// non-negative double reduced with atomicMax on the bit pattern (monotone for
// x >= 0).  Workgroups spread their atomics over the sub-slots, which sit
// RATE_STRIDE bytes apart so concurrent atomics land on different memory
// channels; readers load one sub-slot per lane and take a wave max.
constexpr int RATE_SUB = 64;
constexpr int RATE_STRIDE = 256;
constexpr size_t RATE_BYTES = 3 * RATE_SUB * RATE_STRIDE;
__host__ __device__ inline unsigned long long *rate_slot(unsigned long long *base, int k, int s)
{
    return base + ((size_t)(k * RATE_SUB + s) * RATE_STRIDE) / sizeof(unsigned long long);
}
constexpr size_t CTL_BYTES = 256;

struct StageDesc {
    int prec;   // 0 float, 1 double
    int eqn;    // 0 SWE, 1 Euler
    int bathy;  // bed present
    int flux;
    int recon;
    int nx, ny, bc_x, bc_y;
    double rdx, rdy, g, gamma;
    double h0;  // SWE reference depth of the pressure term (mean initial depth)
    double cfl, dt_fixed;
};

// One RK stage: out = a0*q0 + a1*(qs + dt*L(qs)); q0 is read only at the
// updated cell, so out may alias q0.  On the last stage the CFL rate of out
// is reduced into ctl->rate[rate_out] (rate_out >= 0), rate_clear is zeroed,
// admissibility is checked and time/step advance.
hipError_t launch_stage(const StageDesc &d, const void *qs, const void *q0, void *out, const void *bed,
                        double a0, double a1, Ctl *ctl, unsigned long long *rates, int rate_in, int rate_out,
                        int rate_clear, int last, hipStream_t st);

// Batched FP32 Heun stages over many solves (serving).  BatchSolve is one
// solve's device descriptor; WorkItem one solve of a step's list: where its
// workgroups start in the launch and its CFL slots at that step.
struct BatchSolve {
    void *q, *s1;
    const void *bed;
    void *ctl, *rates;
    int nx, ny, bc_x, bc_y;
    double rdx, rdy, g, sqg, gamma, h0, cfl, dt_fixed;
};
struct WorkItem {
    int solve;
    int tile_begin;  // index of the solve's first workgroup in the launch (prefix sum of tiles)
    int tiles_x;     // tiles per row of the solve; tile = workgroup - tile_begin, row-major
    unsigned char ri, ro, rc, pad;
};
#ifndef FV_TILE_Y
#define FV_TILE_Y 32
#endif
constexpr int TILE_X = 64, TILE_Y = FV_TILE_Y;  // FP32 tile of the stage kernels
// One workgroup per tile: grid = the list's tiles.  one != 0 declares that
// the list holds exactly one solve, solves[0].
hipError_t launch_batch_stage(int eqn, int bathy, int stage, const BatchSolve *solves, const WorkItem *items,
                              const int *nitems, int grid, hipStream_t st, int one = 0);
// One solve, descriptor and list entry by value (it.tile_begin == 0): the
// launches of a single solve.
hipError_t launch_batch_stage_one(int eqn, int bathy, int stage, const BatchSolve &d, const WorkItem &it, int grid,
                                  hipStream_t st);
// The form recorded in graphs: wgs workgroups (a multiple of 8, set to
// xcd_grid(tiles) before each replay), the tile count read from the list
// header list = {items, tiles}.
hipError_t launch_batch_stage_list(int eqn, int bathy, int stage, const BatchSolve *solves, const WorkItem *items,
                                   const int *list, int wgs, hipStream_t st);
// Grid of a tiled launch: the tiles padded to a multiple of the 8 XCDs.
__host__ __device__ inline int xcd_grid(int ntiles) { return (ntiles + 7) & ~7; }


// Reduce the CFL rate of q into ctl->rate[slot] and flag inadmissible cells.
hipError_t launch_rate(const StageDesc &d, const void *q, Ctl *ctl, unsigned long long *rates, int slot,
                       hipStream_t st);

// Deterministic double-precision totals (nvar sums + energy) into out_dev.
hipError_t launch_totals(const StageDesc &d, const void *q, double *partials, int max_blocks, double *out_dev,
                         hipStream_t st);

// Face fluxes of q (flat bottom): fx [nv][ny][nx+1], fy [nv][ny+1][nx].
hipError_t launch_face_fluxes(const StageDesc &d, const void *q, void *fx, void *fy, hipStream_t st);

constexpr int TOTALS_MAX_BLOCKS = 1024;

// Reset a solve's control block and CFL rate slots on the device (a kernel:
// nothing host-side, no memset node).
hipError_t launch_reset(Ctl *ctl, unsigned long long *rates, hipStream_t st);
// Copy a solve's simulated time, completed steps and inadmissible flag into
// the caller's device record {double t; int64 steps; int32 bad; int32 pad}.
hipError_t launch_report(const Ctl *ctl, void *info, hipStream_t st);

}  // namespace fvk
