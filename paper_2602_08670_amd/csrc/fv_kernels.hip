// Finite-volume stage kernels for gfx950 (MI355X).
//
// One workgroup of TY/2 wave64 (two tile rows per wave) owns a TX x TY tile of cells.
//  1. The tile plus a two-cell halo of every variable (and eta = h + b with a
//     bed) is staged into LDS with coalesced row loads; ghost cells are
//     synthesised during the load (periodic wrap or wall mirror with the
//     normal momentum negated).
//  2. Every x face and y face of the tile is evaluated exactly once
//     (reconstruction, hydrostatic step, numerical flux), by the lane of its
//     high-side cell, and stays in registers: a cell's high x face comes from
//     the next lane by a DPP shift, its high y face from the lane's next row
//     (faces at a wave's edge go through LDS).
//  3. Each cell forms the flux divergence (eq 2.9 / eq 2.23), adds the bed
//     source, combines the Runge-Kutta stage (eq 2.19 / eq 2.20) and writes
//     its new value.  On the last stage the CFL rate of the new state is
//     reduced over the wave with DPP, then one atomicMax per wave into a
//     device sub-slot read by the next step, so Delta t never travels
//     through the host.
#include "fv_device.hpp"
#include "fv_internal.hpp"

namespace fvk {

__device__ __forceinline__ int map_index(int i, int n, int bc, bool &flip)
{
    if (i >= 0 && i < n) return i;
    if (bc == 0) return ((i % n) + n) % n;
    flip = true;
    int m = i < 0 ? -1 - i : 2 * n - 1 - i;
    return m < 0 ? 0 : (m >= n ? n - 1 : m);  // cells past the ghost layer are never used
}

template <typename T> struct Tile;
template <> struct Tile<float> { static constexpr int X = TILE_X, Y = TILE_Y; };
static_assert(TILE_X == 64, "a tile row is one wave64");
template <> struct Tile<double> { static constexpr int X = 64, Y = 8; };

template <typename T> struct StageArgs {
    const T *qs;
    const T *q0;
    T *out;
    const T *bed;
    int nx, ny, bc_x, bc_y;
    T rdx, rdy;
    Phys<T> ph;
    T a0, a1;
    double cfl, dt_fixed;
    Ctl *ctl;
    unsigned long long *rates;
    int rate_in, rate_out, rate_clear, last;
};

// Global-memory view of a pointer.  The batched kernels read their array
// pointers from a device descriptor, where the compiler cannot see that they
// address global memory; it would then emit flat accesses, which may alias
// LDS and so are ordered behind every LDS store.
template <typename T> using gmem = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ const gmem<T> *gload(const T *p) { return (const gmem<T> *)p; }
template <typename T> __device__ __forceinline__ gmem<T> *gstore(T *p) { return (gmem<T> *)p; }
// base[i] for a wave-uniform base and a byte offset that fits in 32 bits:
// the address is then an SGPR pair plus a 32-bit VGPR offset, with no 64-bit
// arithmetic per element.
// The base goes through readfirstlane so that the compiler keeps it in
// SGPRs instead of folding a uniform offset into every lane's address.
template <typename T> __device__ __forceinline__ T *sbase(T *p)
{
    const unsigned long long u = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (T *)(((unsigned long long)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T ld_off(const T *base, unsigned i)
{
    return *(const gmem<T> *)((const char *)sbase(base) + i * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ gmem<T> *st_off(T *base, unsigned i)
{
    return (gmem<T> *)((char *)sbase(base) + i * (unsigned)sizeof(T));
}

template <typename T> __device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = tmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void push_rate(unsigned long long *rates, int k, double m, int block_linear)
{
    atomicMax(rate_slot(rates, k, block_linear & (RATE_SUB - 1)), (unsigned long long)__double_as_longlong(m));
}

// Max over a wave of non-negative values, in every lane.  Non-negative
// floats order like their bit patterns, so the float path reduces unsigned
// integers with DPP row shifts (lane 15 of each 16-lane row ends with its
// row's max) and combines the four rows with lane reads.
template <int CTRL> __device__ __forceinline__ unsigned dpp_u(unsigned x)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, false);  // lanes with no source read 0
}
__device__ __forceinline__ float wave_max_nonneg(float v)
{
    unsigned x = __float_as_uint(v);
    x = max(x, dpp_u<0x111>(x));  // row_shr:1
    x = max(x, dpp_u<0x112>(x));  // row_shr:2
    x = max(x, dpp_u<0x114>(x));  // row_shr:4
    x = max(x, dpp_u<0x118>(x));  // row_shr:8
    const unsigned a = max((unsigned)__builtin_amdgcn_readlane((int)x, 15), (unsigned)__builtin_amdgcn_readlane((int)x, 31));
    const unsigned b = max((unsigned)__builtin_amdgcn_readlane((int)x, 47), (unsigned)__builtin_amdgcn_readlane((int)x, 63));
    return __uint_as_float(max(a, b));
}
// The same for non-negative doubles, as 64-bit patterns in two halves (no
// lane-index arithmetic, so nothing stays live across a workgroup's tiles).
template <int CTRL> __device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x)
{
    return (unsigned long long)dpp_u<CTRL>((unsigned)(x >> 32)) << 32 | dpp_u<CTRL>((unsigned)x);
}
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int l)
{
    return (unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l) << 32 |
           (unsigned)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
__device__ __forceinline__ double wave_max_nonneg(double v)
{
    unsigned long long x = (unsigned long long)__double_as_longlong(v);
    x = umax64(x, dpp_u64<0x111>(x));
    x = umax64(x, dpp_u64<0x112>(x));
    x = umax64(x, dpp_u64<0x114>(x));
    x = umax64(x, dpp_u64<0x118>(x));
    const unsigned long long a = umax64(readlane_u64(x, 15), readlane_u64(x, 31));
    const unsigned long long b = umax64(readlane_u64(x, 47), readlane_u64(x, 63));
    return __longlong_as_double((long long)umax64(a, b));
}

// Largest CFL rate stored in slot k (max over its sub-slots, all >= 0),
// wave-uniform.
static_assert(RATE_SUB == 64, "one sub-slot per lane");
__device__ __forceinline__ double read_rate(unsigned long long *rates, int k, int lane)
{
    return wave_max_nonneg(__longlong_as_double(*gload(rate_slot(rates, k, lane))));
}

// Block-wide max of v (threads 0..255) -> returned in thread 0.
template <typename T> __device__ __forceinline__ T block_max256(T v, T *red)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T m = red[0];
#pragma unroll
    for (int w = 1; w < 4; w++) m = tmax(m, red[w]);
    return m;
}

// Lane l receives v from lane l + 1 of its wave (DPP wave shift); lane 63
// receives `edge`.  Every lane of the wave must be active.
__device__ __forceinline__ float from_right(float v, float edge)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_right(double v, double edge)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long e = (unsigned long long)__double_as_longlong(edge);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)e, (int)(unsigned)b, 0x130, 0xf, 0xf, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(e >> 32), (int)(unsigned)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// LDS of one stage tile: the halo tile of every variable (and eta), the
// faces handed between waves, and the step's Delta t.
template <typename T, int EQN, bool BATHY, int TX, int TY> struct StageLds {
    static constexpr int RPW = 2;             // tile rows per wave
    static constexpr int NW = TY / RPW;       // waves per workgroup
    static constexpr int NTH = 64 * NW;       // threads per workgroup
    static_assert(TY % RPW == 0 && NW >= 2 && NW <= 16, "whole rows per wave, 2..16 waves");
    static constexpr int NV = EQN == SWE ? 3 : 4;
    static constexpr int NL = NV + (BATHY ? 1 : 0);  // LDS planes: variables (+ eta)
    static constexpr int NT = FaceSide<T, EQN, BATHY>::N;
    static constexpr int HX = TX + 4, HY = TY + 4;
    static constexpr int NIT = (HY * HX + NTH - 1) / NTH;  // halo elements per thread
    // rows past HY pad each plane to NIT * NTH elements: the last pass of the
    // halo staging then stores unconditionally (its extra lanes write padding),
    // so every halo load is issued before the first store
    static constexpr int HYP = (NIT * NTH + HX - 1) / HX;
    T q[NL][HYP][HX];
    T edge[NT][TY];         // right face of column TX-1, handed to that cell
    T low[NW - 1][NT][TX];  // low y face of wave w+1's first row, handed to wave w
    double dt;
};

// Halo values of one inner tile held in registers between the issue of their
// loads and their store to LDS.
template <typename T, int EQN, bool BATHY, int TX, int TY> struct HaloRegs {
    using L = StageLds<T, EQN, BATHY, TX, TY>;
    T val[L::NIT][L::NL];
};

// A tile whose two-cell halo lies inside the grid (all but the border tiles)
// loads without ghost synthesis.
template <int TX, int TY> __device__ __forceinline__ bool inner_tile(int x0, int y0, int nx, int ny)
{
    return x0 >= 2 && y0 >= 2 && x0 + TX + 2 <= nx && y0 + TY + 2 <= ny;
}

// Issue every halo load of an inner tile (no LDS access, no wait).  The last
// pass re-reads the tile's first halo element on lanes past the end.
template <typename T, int EQN, bool BATHY, int TX, int TY>
__device__ __forceinline__ void halo_issue(const StageArgs<T> &a, const int x0, const int y0, const int tid,
                                           HaloRegs<T, EQN, BATHY, TX, TY> &r)
{
    using L = StageLds<T, EQN, BATHY, TX, TY>;
    const int nx = a.nx;
    const size_t plane = (size_t)nx * a.ny;
    const size_t hb = (size_t)y0 * nx + x0 - 2 * (size_t)nx - 2;
#pragma unroll
    for (int it = 0; it < L::NIT; it++) {
        const int e = tid + it * L::NTH;
        const int ec = e < L::HY * L::HX ? e : 0;
        const int ly = ec / L::HX, lx = ec - ly * L::HX;
        const unsigned off = (unsigned)(ly * nx + lx);
#pragma unroll
        for (int v = 0; v < L::NV; v++) r.val[it][v] = ld_off(a.qs + v * plane + hb, off);
        if constexpr (BATHY) r.val[it][L::NV] = ld_off(a.bed + hb, off);
    }
}

template <typename T, int EQN, bool BATHY, int TX, int TY>
__device__ __forceinline__ void halo_commit(const HaloRegs<T, EQN, BATHY, TX, TY> &r,
                                            StageLds<T, EQN, BATHY, TX, TY> &sh, const int tid)
{
    using L = StageLds<T, EQN, BATHY, TX, TY>;
#pragma unroll
    for (int it = 0; it < L::NIT; it++) {
        const int e = tid + it * L::NTH;
        const int ly = e / L::HX, lx = e - ly * L::HX;
#pragma unroll
        for (int v = 0; v < L::NV; v++) sh.q[v][ly][lx] = r.val[it][v];
        if constexpr (BATHY) sh.q[L::NV][ly][lx] = r.val[it][0] + r.val[it][L::NV];
    }
}

// Border tiles: ghost cells synthesised during the load (periodic wrap or
// wall mirror with the normal momentum negated).
template <typename T, int EQN, bool BATHY, int TX, int TY>
__device__ __forceinline__ void halo_border(const StageArgs<T> &a, const int x0, const int y0, const int tid,
                                            StageLds<T, EQN, BATHY, TX, TY> &sh)
{
    using L = StageLds<T, EQN, BATHY, TX, TY>;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    for (int k = tid; k < L::HY * L::HX; k += L::NTH) {
        int ly = k / L::HX, lx = k - ly * L::HX;
        bool fx = false, fy = false;
        int ix = map_index(x0 - 2 + lx, nx, a.bc_x, fx);
        int iy = map_index(y0 - 2 + ly, ny, a.bc_y, fy);
        size_t idx = (size_t)iy * nx + ix;
        T val[L::NV];
#pragma unroll
        for (int v = 0; v < L::NV; v++) val[v] = gload(a.qs)[v * plane + idx];
        const T b = BATHY ? gload(a.bed)[idx] : T(0);
#pragma unroll
        for (int v = 0; v < L::NV; v++) sh.q[v][ly][lx] = ((v == 1 && fx) || (v == 2 && fy)) ? -val[v] : val[v];
        if constexpr (BATHY) sh.q[L::NV][ly][lx] = val[0] + b;
    }
}

// Delta t of the step = CFL / (max over the previous step's rate sub-slots),
// read by wave 1 into LDS.
template <typename T, int EQN, bool BATHY, int TX, int TY>
__device__ __forceinline__ void stage_dt(const StageArgs<T> &a, const int tid, StageLds<T, EQN, BATHY, TX, TY> &sh)
{
    if ((tid >> 6) == 1) {
        const int lane = tid & 63;
        const double d = a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl / read_rate(a.rates, a.rate_in, lane);
        if (lane == 0) sh.dt = d;
    }
}

// One RK stage on the TX x TY tile at (x0, y0) whose halo, faces and Delta t
// are staged in `sh` (after a barrier).  `tile_linear` is the tile's index
// within its solve; the tile with index 0 does the per-step bookkeeping of
// the solve.  Shared by every stage kernel, so a solve computes bit-identical
// results in all of them.
//
// Work split: lane = column, wave w owns tile rows [2w, 2w+1].  Each
// lane evaluates the low x face and the low y face of each of its cells, so
// face results stay in registers: the high x face arrives from lane + 1 by a
// DPP shift, the high y face from the same lane's next row.  Faces with no
// owner inside the wave are the tile's right column (one lane per row, wave
// 0, through LDS), the tile's top row (last wave) and the low face of each
// wave's first row, which the wave below reads through LDS.
// tid: threadIdx.x (a workgroup looping over tiles passes it opaquely, so
// that per-lane index arithmetic is redone per tile instead of being held in
// registers across the loop).
template <typename T, int EQN, bool BATHY, int FLUX, int RECON, int TX, int TY>
__device__ __forceinline__ void stage_compute(const StageArgs<T> &a, const int x0, const int y0,
                                              const int tile_linear, const int tid,
                                              StageLds<T, EQN, BATHY, TX, TY> &sh)
{
    static_assert(TX == 64, "a tile row is one wave64");
    using LD = StageLds<T, EQN, BATHY, TX, TY>;
    constexpr int NW = LD::NW, RPW = LD::RPW;
    constexpr int NV = LD::NV, NL = LD::NL, NT = LD::NT;
    auto &s_q = sh.q;
    auto &s_edge = sh.edge;
    auto &s_low = sh.low;

    // An earlier step failed: the state is frozen.  The flag is checked only
    // where something would be written, so its load is off the critical path.
    const bool frozen = gload(a.ctl)->bad != 0;
    const int lane = tid & 63, wave = tid >> 6;
    const int r0 = wave * RPW;
    const int nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)nx * ny;
    const size_t tbase = (size_t)y0 * nx + x0;
    const T dt = (T)sh.dt;
    // stage weight times Delta t over the cell width, per axis
    const T cxs = a.a1 * dt * a.rdx, cys = a.a1 * dt * a.rdy;

    // 2. faces with no owner lane: the tile's right column and top row
    if (wave == 0 && lane < TY) {
        T st[NL][4];
#pragma unroll
        for (int v = 0; v < NL; v++)
#pragma unroll
            for (int k = 0; k < 4; k++) st[v][k] = s_q[v][lane + 2][TX + k];
        T tl[NT], tr[NT];
        face_eval<T, EQN, BATHY, FLUX, RECON, 0>(st, a.ph, tl, tr);
#pragma unroll
        for (int k = 0; k < NT; k++) s_edge[k][lane] = tl[k];
    }
    T top[NT];  // low-side values of the y face above this wave's last row
    if (wave == NW - 1) {
        T st[NL][4];
#pragma unroll
        for (int v = 0; v < NL; v++)
#pragma unroll
            for (int k = 0; k < 4; k++) st[v][k] = s_q[v][TY + k][lane + 2];
        T tr[NT];
        face_eval<T, EQN, BATHY, FLUX, RECON, 1>(st, a.ph, top, tr);
    }

    // 3. y faces: the low face of every own row, evaluated from the last row
    //    down so that each row's y divergence can be formed at once
    T Ly[RPW][NV];
    T lowR[NT];  // high-side values of the low face of the wave's first row
#pragma unroll
    for (int j = RPW - 1; j >= 0; j--) {
        const int cy = r0 + j;
        T st[NL][4];
#pragma unroll
        for (int v = 0; v < NL; v++)
#pragma unroll
            for (int k = 0; k < 4; k++) st[v][k] = s_q[v][cy + k][lane + 2];
        T tl[NT], tr[NT];
        face_eval<T, EQN, BATHY, FLUX, RECON, 1>(st, a.ph, tl, tr);
        if (j == RPW - 1) {
            if (wave == NW - 1) {
#pragma unroll
                for (int v = 0; v < NV; v++) Ly[j][v] = tr[v] - top[v];
                if constexpr (BATHY) Ly[j][2] += bed_term(tr[NV], tr[NV + 1], top[NV], top[NV + 1], a.ph.g);
            } else {
#pragma unroll
                for (int k = 0; k < NT; k++) lowR[k] = tr[k];  // finished after the exchange
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; v++) Ly[j][v] = tr[v] - top[v];
            if constexpr (BATHY) Ly[j][2] += bed_term(tr[NV], tr[NV + 1], top[NV], top[NV + 1], a.ph.g);
        }
        if (j == 0 && wave > 0) {
#pragma unroll
            for (int k = 0; k < NT; k++) s_low[wave - 1][k][lane] = tl[k];
        }
#pragma unroll
        for (int k = 0; k < NT; k++) top[k] = tl[k];
    }
    __syncthreads();
    if (wave < NW - 1) {
        T up[NT];
#pragma unroll
        for (int k = 0; k < NT; k++) up[k] = s_low[wave][k][lane];
#pragma unroll
        for (int v = 0; v < NV; v++) Ly[RPW - 1][v] = lowR[v] - up[v];
        if constexpr (BATHY) Ly[RPW - 1][2] += bed_term(lowR[NV], lowR[NV + 1], up[NV], up[NV + 1], a.ph.g);
    }

    // q0 is needed only in the final combine: issued here, its latency hides
    // behind the x faces, and it holds no registers during the y faces
    T q0r[RPW][NV];
    if (a.a0 != T(0)) {
#pragma unroll
        for (int j = 0; j < RPW; j++) {
            const int cy = r0 + j;
            const bool in = x0 + lane < nx && y0 + cy < ny;
            const unsigned off = in ? (unsigned)(cy * nx + lane) : 0u;
#pragma unroll
            for (int v = 0; v < NV; v++) q0r[j][v] = ld_off(a.q0 + v * plane + tbase, off);
        }
    }

    // 4. x faces, divergence, bed source, RK combine
    T lmax = T(0);
    bool bad = false;
#pragma unroll
    for (int j = 0; j < RPW; j++) {
        const int cy = r0 + j;
        T st[NL][4];
#pragma unroll
        for (int v = 0; v < NL; v++)
#pragma unroll
            for (int k = 0; k < 4; k++) st[v][k] = s_q[v][cy + 2][lane + k];
        T tl[NT], tr[NT], rt[NT];
        face_eval<T, EQN, BATHY, FLUX, RECON, 0>(st, a.ph, tl, tr);
#pragma unroll
        for (int k = 0; k < NT; k++) rt[k] = from_right(tl[k], s_edge[k][cy]);
        T Lv[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) Lv[v] = tr[v] - rt[v];
        if constexpr (BATHY) Lv[1] += bed_term(tr[NV], tr[NV + 1], rt[NV], rt[NV + 1], a.ph.g);
        const bool in = x0 + lane < nx && y0 + cy < ny && !frozen;
        if (in) {
            const unsigned off = (unsigned)(cy * nx + lane);
            T qn[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                // out = a0 q0 + a1 (q + dt L), L = (x flux difference) / dx + (y flux difference) / dy;
                // the increment is summed first, so the result is rounded
                // twice at its own magnitude (once per added state)
                const T inc = cxs * Lv[v] + cys * Ly[j][v];
                T o = a.a1 * st[v][2] + inc;
                if (a.a0 != T(0)) o = a.a0 * q0r[j][v] + o;
                __builtin_nontemporal_store(o, st_off(a.out + v * plane + tbase, off));
                qn[v] = o;
            }
            if (a.last) {
                T r;
                if (cell_rate_ok<T, EQN>(qn, a.ph, a.rdx, a.rdy, r)) lmax = tmax(lmax, r);
                else bad = true;
            }
        }
    }
    if (!a.last || frozen) return;
    if (bad) atomicExch(&a.ctl->bad, 1);
    if (a.rate_out >= 0) {
        // one atomic per wave: no block-wide reduction, no further barrier
        const T m = wave_max_nonneg(lmax);
        if (lane == 0) push_rate(a.rates, a.rate_out, (double)m, tile_linear * NW + wave);
    }
    if (tile_linear == 0) {
        if (tid == 0) {
            a.ctl->t += sh.dt;
            a.ctl->step += 1;
        }
        if (a.rate_clear >= 0 && tid < RATE_SUB) *rate_slot(a.rates, a.rate_clear, tid) = 0ull;
    }
}

// One RK stage on one tile, loaded and computed by the calling workgroup.
template <typename T, int EQN, bool BATHY, int FLUX, int RECON, int TX, int TY>
__device__ __forceinline__ void stage_tile(const StageArgs<T> &a, const int x0, const int y0, const int tile_linear,
                                           const int tid)
{
    __shared__ StageLds<T, EQN, BATHY, TX, TY> sh;
    if (inner_tile<TX, TY>(x0, y0, a.nx, a.ny)) {
        // every halo load is issued before the first LDS store and before
        // the Delta t read, whose reduction would otherwise hold them back
        HaloRegs<T, EQN, BATHY, TX, TY> r;
        halo_issue(a, x0, y0, tid, r);
        stage_dt(a, tid, sh);
        halo_commit(r, sh, tid);
    } else {
        stage_dt(a, tid, sh);
        halo_border(a, x0, y0, tid, sh);
    }
    __syncthreads();
    stage_compute<T, EQN, BATHY, FLUX, RECON, TX, TY>(a, x0, y0, tile_linear, tid, sh);
}

// Workgroups are handed to the eight XCDs in turn (workgroup w runs on XCD
// w mod 8).  For a grid that is a multiple of 8, give XCD k the contiguous
// k-th eighth of the tiles, so that neighbouring tiles, which re-read each
// other's halo rows, share one L2.
__device__ __forceinline__ int xcd_tile(int w, int grid)
{
    return (grid & 7) ? w : (w & 7) * (grid >> 3) + (w >> 3);
}

template <typename T, int EQN, bool BATHY, int FLUX, int RECON, int TX, int TY>
__global__ __launch_bounds__((StageLds<T, EQN, BATHY, TX, TY>::NTH)) void stage_kernel(StageArgs<T> a, int tiles_x,
                                                                                   int ntiles)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    stage_tile<T, EQN, BATHY, FLUX, RECON, TX, TY>(a, tx * TX, ty * TY, tile, threadIdx.x);
}

// Batched stage over many solves: the step's list holds one item per solve
// (sorted by tile_begin); tile w of the launch belongs to the solve whose tile
// range contains it (binary search).  STAGE 1: S1 = q + dt L(q); STAGE 2:
// q = q/2 + (S1 + dt L(S1))/2 (Heun).
struct TileRef {
    int x0, y0, tile;
};

template <typename T, int STAGE>
__device__ __forceinline__ TileRef batch_fill(const BatchSolve &d, const WorkItem &it, const int w, StageArgs<T> &a);

template <typename T, int STAGE>
__device__ __forceinline__ TileRef batch_resolve(const BatchSolve *__restrict__ solves,
                                                 const WorkItem *__restrict__ items, const int *__restrict__ nitems,
                                                 const int w, const int one, StageArgs<T> &a)
{
    // one != 0: the list is known to hold one solve, solves[0] (a single
    // solve stepping through this kernel); its descriptor and list entry are
    // then fetched together instead of one after the other
    WorkItem it;
    const BatchSolve *dp;
    if (one) {
        it = items[0];
        dp = solves;
    } else {
        const int n = *nitems;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (items[mid].tile_begin <= w) lo = mid;
            else hi = mid - 1;
        }
        it = items[lo];
        dp = solves + it.solve;
    }
    return batch_fill<T, STAGE>(*dp, it, w, a);
}

// The stage arguments of workgroup w, whose solve is d with list entry it.
template <typename T, int STAGE>
__device__ __forceinline__ TileRef batch_fill(const BatchSolve &d, const WorkItem &it, const int w, StageArgs<T> &a)
{
    constexpr int TX = Tile<T>::X, TY = Tile<T>::Y;
    const int tile = w - it.tile_begin;
    a.qs = (const T *)(STAGE == 1 ? d.q : d.s1);
    a.q0 = (const T *)d.q;
    a.out = (T *)(STAGE == 1 ? d.s1 : d.q);
    a.bed = (const T *)d.bed;
    a.nx = d.nx;
    a.ny = d.ny;
    a.bc_x = d.bc_x;
    a.bc_y = d.bc_y;
    a.rdx = (T)d.rdx;
    a.rdy = (T)d.rdy;
    a.ph.g = (T)d.g;
    a.ph.sqg = (T)d.sqg;
    a.ph.gamma = (T)d.gamma;
    a.ph.h0 = (T)d.h0;
    a.a0 = STAGE == 1 ? T(0) : T(0.5);
    a.a1 = STAGE == 1 ? T(1) : T(0.5);
    a.cfl = d.cfl;
    a.dt_fixed = d.dt_fixed;
    a.ctl = (Ctl *)d.ctl;
    a.rates = (unsigned long long *)d.rates;
    a.rate_in = it.ri;
    a.rate_out = STAGE == 1 ? -1 : it.ro;
    a.rate_clear = STAGE == 1 ? -1 : it.rc;
    a.last = STAGE == 2;
    const int ty = tile / it.tiles_x, tx = tile - ty * it.tiles_x;
    return TileRef{tx * TX, ty * TY, tile};
}

// One workgroup per tile.  ntiles > 0: the list holds ntiles tiles.
// ntiles == 0: the tile count is read from the list header (nitems[1]), so
// that a launch recorded in a graph serves whatever list is uploaded before
// each replay.  The grid is xcd_grid(tiles).  Eight waves per SIMD (at most
// 64 VGPRs): every tile of a 1024^2 grid is then resident at once.
template <typename T, int EQN, bool BATHY, int STAGE>
__global__ __launch_bounds__((StageLds<T, EQN, BATHY, Tile<T>::X, Tile<T>::Y>::NTH), 8) void batch_stage_kernel(
    const BatchSolve *__restrict__ solves, const WorkItem *__restrict__ items, const int *__restrict__ nitems,
    int ntiles, int one)
{
    constexpr int TX = Tile<T>::X, TY = Tile<T>::Y;
    const int total = ntiles > 0 ? ntiles : nitems[1];
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= total) return;
    StageArgs<T> a;
    const TileRef t = batch_resolve<T, STAGE>(solves, items, nitems, w, one, a);
    stage_tile<T, EQN, BATHY, HLLE, MINMOD, TX, TY>(a, t.x0, t.y0, t.tile, threadIdx.x);
}

// One solve, its descriptor and list entry passed by value: the halo loads
// wait for nothing but the arguments.  The same stage arguments, hence the
// same results, as the list form.
template <typename T, int EQN, bool BATHY, int STAGE>
__global__ __launch_bounds__((StageLds<T, EQN, BATHY, Tile<T>::X, Tile<T>::Y>::NTH), 8) void batch_stage_one_kernel(
    BatchSolve d, WorkItem it, int ntiles)
{
    constexpr int TX = Tile<T>::X, TY = Tile<T>::Y;
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= ntiles) return;
    StageArgs<T> a;
    const TileRef t = batch_fill<T, STAGE>(d, it, w, a);
    stage_tile<T, EQN, BATHY, HLLE, MINMOD, TX, TY>(a, t.x0, t.y0, t.tile, threadIdx.x);
}

// ------------------------------------------------------------ CFL rate of q
template <typename T, int EQN>
__global__ __launch_bounds__(256) void rate_kernel(const T *q, int n, T rdx, T rdy, Phys<T> ph, Ctl *ctl,
                                                   unsigned long long *rates, int slot)
{
    __shared__ T s_red[4];
    constexpr int NV = EQN == SWE ? 3 : 4;
    T lmax = T(0);
    bool bad = false;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        T s[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) s[v] = q[(size_t)v * n + k];
        T r;
        if (cell_rate_ok<T, EQN>(s, ph, rdx, rdy, r)) lmax = tmax(lmax, r);
        else bad = true;
    }
    if (bad) atomicExch(&ctl->bad, 1);
    T m = block_max256(lmax, s_red);
    if (threadIdx.x == 0) push_rate(rates, slot, (double)m, blockIdx.x);
}

// ----------------------------------------------------------------- totals
// Block b sums a fixed set of cells in a fixed order, then a fixed-order tree;
// a single block then adds the block partials in index order.
template <typename T, int EQN>
__global__ __launch_bounds__(256) void totals_partial_kernel(const T *q, int n, double dA, double g, double *partials)
{
    constexpr int NV = EQN == SWE ? 3 : 4;
    __shared__ double s[NV + 1][256];
    double acc[NV + 1];
#pragma unroll
    for (int v = 0; v <= NV; v++) acc[v] = 0.0;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        double c[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) c[v] = (double)q[(size_t)v * n + k];
#pragma unroll
        for (int v = 0; v < NV; v++) acc[v] += c[v] * dA;
        double kin = 0.5 * (c[1] * c[1] + c[2] * c[2]) / c[0];
        acc[NV] += (EQN == SWE ? 0.5 * g * c[0] * c[0] + kin : kin) * dA;
    }
#pragma unroll
    for (int v = 0; v <= NV; v++) s[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int v = 0; v <= NV; v++) s[v][threadIdx.x] += s[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int v = 0; v <= NV; v++) partials[blockIdx.x * (NV + 1) + v] = s[v][0];
}

// One workgroup per output: thread t adds partials t, t+256, ... in order,
// then a fixed-order tree over the 256 threads.
__global__ __launch_bounds__(256) void totals_final_kernel(const double *partials, int nblocks, int nout, double *out)
{
    __shared__ double s[256];
    const int o = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) acc += partials[b * nout + o];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[o] = s[0];
}

// ------------------------------------------------------- solve reset/report
__global__ __launch_bounds__(256) void reset_kernel(Ctl *ctl, unsigned long long *rates)
{
    const int t = threadIdx.x;
    for (int k = t; k < (int)(RATE_BYTES / sizeof(unsigned long long)); k += 256) rates[k] = 0ull;
    if (t < (int)(sizeof(Ctl) / sizeof(unsigned long long))) ((unsigned long long *)ctl)[t] = 0ull;
}

struct RunInfo {
    double t;
    long long steps;
    int bad;
    int pad;
};

__global__ void report_kernel(const Ctl *ctl, RunInfo *info)
{
    if (threadIdx.x == 0) {
        info->t = ctl->t;
        info->steps = ctl->step;
        info->bad = ctl->bad;
        info->pad = 0;
    }
}

hipError_t launch_reset(Ctl *ctl, unsigned long long *rates, hipStream_t st)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(256), 0, st, ctl, rates);
    return hipGetLastError();
}

hipError_t launch_report(const Ctl *ctl, void *info, hipStream_t st)
{
    hipLaunchKernelGGL(report_kernel, dim3(1), dim3(64), 0, st, ctl, (RunInfo *)info);
    return hipGetLastError();
}

// --------------------------------------------------------------- face export
template <typename T, int EQN, int FLUX, int RECON>
__global__ void face_kernel(const T *q, int nx, int ny, int bc_x, int bc_y, Phys<T> ph, T *fx, T *fy)
{
    constexpr int NV = EQN == SWE ? 3 : 4;
    const size_t plane = (size_t)nx * ny;
    const int nfx = (nx + 1) * ny, nfy = nx * (ny + 1);
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfx + nfy) return;
    int axis = f < nfx ? 0 : 1;
    int i, j;
    if (axis == 0) {
        j = f / (nx + 1);
        i = f - j * (nx + 1) - 1;  // face between cells i and i+1
    } else {
        int g = f - nfx;
        j = g / nx - 1;            // face between rows j and j+1
        i = g - (j + 1) * nx;
    }
    T st[NV][4];
    for (int k = 0; k < 4; k++) {
        int ci = axis == 0 ? i - 1 + k : i, cj = axis == 0 ? j : j - 1 + k;
        bool flx = false, fly = false;
        int ix = map_index(ci, nx, bc_x, flx), iy = map_index(cj, ny, bc_y, fly);
        for (int v = 0; v < NV; v++) {
            T val = q[v * plane + (size_t)iy * nx + ix];
            if ((v == 1 && flx) || (v == 2 && fly)) val = -val;
            st[v][k] = val;
        }
    }
    T Fl[NV], frn;
    if (axis == 0) {
        face_flux<T, EQN, false, FLUX, RECON, 0>(st, ph, Fl, frn);
        for (int v = 0; v < NV; v++) fx[(size_t)v * nfx + (size_t)j * (nx + 1) + i + 1] = Fl[v];
    } else {
        face_flux<T, EQN, false, FLUX, RECON, 1>(st, ph, Fl, frn);
        for (int v = 0; v < NV; v++) fy[(size_t)v * nfy + (size_t)(j + 1) * nx + i] = Fl[v];
    }
}

// ----------------------------------------------------------------- dispatch

template <typename T, int EQN, bool BATHY, int FLUX, int RECON>
static hipError_t stage_t(const StageDesc &d, const void *qs, const void *q0, void *out, const void *bed, double a0,
                          double a1, Ctl *ctl, unsigned long long *rates, int ri, int ro, int rc, int last,
                          hipStream_t st)
{
    StageArgs<T> a;
    a.qs = (const T *)qs;
    a.q0 = (const T *)q0;
    a.out = (T *)out;
    a.bed = (const T *)bed;
    a.nx = d.nx;
    a.ny = d.ny;
    a.bc_x = d.bc_x;
    a.bc_y = d.bc_y;
    a.rdx = (T)d.rdx;
    a.rdy = (T)d.rdy;
    a.ph.g = (T)d.g;
    a.ph.sqg = (T)__builtin_sqrt(d.g);
    a.ph.gamma = (T)d.gamma;
    a.ph.h0 = (T)d.h0;
    a.a0 = (T)a0;
    a.a1 = (T)a1;
    a.cfl = d.cfl;
    a.dt_fixed = d.dt_fixed;
    a.ctl = ctl;
    a.rates = rates;
    a.rate_in = ri;
    a.rate_out = ro;
    a.rate_clear = rc;
    a.last = last;
    constexpr int TX = Tile<T>::X, TY = Tile<T>::Y;
    const int tiles_x = (d.nx + TX - 1) / TX, ntiles = tiles_x * ((d.ny + TY - 1) / TY);
    constexpr int NTH = StageLds<T, EQN, BATHY, TX, TY>::NTH;
    hipLaunchKernelGGL((stage_kernel<T, EQN, BATHY, FLUX, RECON, TX, TY>), dim3(xcd_grid(ntiles)), dim3(NTH), 0, st, a,
                       tiles_x, ntiles);
    return hipGetLastError();
}

template <typename T, int EQN, bool BATHY, int FLUX>
static hipError_t stage_r(const StageDesc &d, const void *qs, const void *q0, void *out, const void *bed, double a0,
                          double a1, Ctl *ctl, unsigned long long *rates, int ri, int ro, int rc, int last,
                          hipStream_t st)
{
    if (d.recon == FIRST)
        return stage_t<T, EQN, BATHY, FLUX, FIRST>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
    return stage_t<T, EQN, BATHY, FLUX, MINMOD>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
}

template <typename T, int EQN, bool BATHY>
static hipError_t stage_f(const StageDesc &d, const void *qs, const void *q0, void *out, const void *bed, double a0,
                          double a1, Ctl *ctl, unsigned long long *rates, int ri, int ro, int rc, int last,
                          hipStream_t st)
{
    switch (d.flux) {
    case RUSANOV: return stage_r<T, EQN, BATHY, RUSANOV>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
    case ROE: return stage_r<T, EQN, BATHY, ROE>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
    default: return stage_r<T, EQN, BATHY, HLLE>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
    }
}

template <typename T>
static hipError_t stage_p(const StageDesc &d, const void *qs, const void *q0, void *out, const void *bed, double a0,
                          double a1, Ctl *ctl, unsigned long long *rates, int ri, int ro, int rc, int last,
                          hipStream_t st)
{
    if (d.eqn == EULER) return stage_f<T, EULER, false>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
    if (d.bathy) return stage_f<T, SWE, true>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
    return stage_f<T, SWE, false>(d, qs, q0, out, bed, a0, a1, ctl, rates, ri, ro, rc, last, st);
}

hipError_t launch_stage(const StageDesc &d, const void *qs, const void *q0, void *out, const void *bed, double a0,
                        double a1, Ctl *ctl, unsigned long long *rates, int rate_in, int rate_out, int rate_clear,
                        int last, hipStream_t st)
{
    if (d.prec == 1)
        return stage_p<double>(d, qs, q0, out, bed, a0, a1, ctl, rates, rate_in, rate_out, rate_clear, last, st);
    return stage_p<float>(d, qs, q0, out, bed, a0, a1, ctl, rates, rate_in, rate_out, rate_clear, last, st);
}

template <typename T>
static hipError_t rate_t(const StageDesc &d, const void *q, Ctl *ctl, unsigned long long *rates, int slot,
                         hipStream_t st)
{
    int n = d.nx * d.ny;
    int blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    Phys<T> ph{(T)d.g, (T)__builtin_sqrt(d.g), (T)d.gamma, T(0)};
    if (d.eqn == EULER)
        hipLaunchKernelGGL((rate_kernel<T, EULER>), dim3(blocks), dim3(256), 0, st, (const T *)q, n, (T)d.rdx,
                           (T)d.rdy, ph, ctl, rates, slot);
    else
        hipLaunchKernelGGL((rate_kernel<T, SWE>), dim3(blocks), dim3(256), 0, st, (const T *)q, n, (T)d.rdx,
                           (T)d.rdy, ph, ctl, rates, slot);
    return hipGetLastError();
}

template <int STAGE>
static void batch_stage_go(int eqn, int bathy, dim3 g, const BatchSolve *solves, const WorkItem *items,
                           const int *nitems, int ntiles, int one, hipStream_t st)
{
    constexpr int TX = Tile<float>::X, TY = Tile<float>::Y;
    if (eqn == EULER)
        hipLaunchKernelGGL((batch_stage_kernel<float, EULER, false, STAGE>), g,
                           dim3(StageLds<float, EULER, false, TX, TY>::NTH), 0, st, solves, items, nitems, ntiles, one);
    else if (bathy)
        hipLaunchKernelGGL((batch_stage_kernel<float, SWE, true, STAGE>), g,
                           dim3(StageLds<float, SWE, true, TX, TY>::NTH), 0, st, solves, items, nitems, ntiles, one);
    else
        hipLaunchKernelGGL((batch_stage_kernel<float, SWE, false, STAGE>), g,
                           dim3(StageLds<float, SWE, false, TX, TY>::NTH), 0, st, solves, items, nitems, ntiles, one);
}

hipError_t launch_batch_stage(int eqn, int bathy, int stage, const BatchSolve *solves, const WorkItem *items,
                              const int *nitems, int grid, hipStream_t st, int one)
{
    if (grid <= 0) return hipSuccess;
    const dim3 g(xcd_grid(grid));
    if (stage == 1) batch_stage_go<1>(eqn, bathy, g, solves, items, nitems, grid, one, st);
    else batch_stage_go<2>(eqn, bathy, g, solves, items, nitems, grid, one, st);
    return hipGetLastError();
}

template <int STAGE>
static void batch_stage_one_go(int eqn, int bathy, dim3 g, const BatchSolve &d, const WorkItem &it, int ntiles,
                               hipStream_t st)
{
    constexpr int TX = Tile<float>::X, TY = Tile<float>::Y;
    if (eqn == EULER)
        hipLaunchKernelGGL((batch_stage_one_kernel<float, EULER, false, STAGE>), g,
                           dim3(StageLds<float, EULER, false, TX, TY>::NTH), 0, st, d, it, ntiles);
    else if (bathy)
        hipLaunchKernelGGL((batch_stage_one_kernel<float, SWE, true, STAGE>), g,
                           dim3(StageLds<float, SWE, true, TX, TY>::NTH), 0, st, d, it, ntiles);
    else
        hipLaunchKernelGGL((batch_stage_one_kernel<float, SWE, false, STAGE>), g,
                           dim3(StageLds<float, SWE, false, TX, TY>::NTH), 0, st, d, it, ntiles);
}

hipError_t launch_batch_stage_one(int eqn, int bathy, int stage, const BatchSolve &d, const WorkItem &it, int grid,
                                  hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    if (it.tile_begin != 0) return hipErrorInvalidValue;
    const dim3 g(xcd_grid(grid));
    if (stage == 1) batch_stage_one_go<1>(eqn, bathy, g, d, it, grid, st);
    else batch_stage_one_go<2>(eqn, bathy, g, d, it, grid, st);
    return hipGetLastError();
}

hipError_t launch_batch_stage_list(int eqn, int bathy, int stage, const BatchSolve *solves, const WorkItem *items,
                                   const int *list, int wgs, hipStream_t st)
{
    if (wgs <= 0 || (wgs & 7)) return hipErrorInvalidValue;
    if (stage == 1) batch_stage_go<1>(eqn, bathy, dim3(wgs), solves, items, list, 0, 0, st);
    else batch_stage_go<2>(eqn, bathy, dim3(wgs), solves, items, list, 0, 0, st);
    return hipGetLastError();
}

hipError_t launch_rate(const StageDesc &d, const void *q, Ctl *ctl, unsigned long long *rates, int slot,
                       hipStream_t st)
{
    return d.prec == 1 ? rate_t<double>(d, q, ctl, rates, slot, st) : rate_t<float>(d, q, ctl, rates, slot, st);
}

template <typename T>
static hipError_t totals_t(const StageDesc &d, const void *q, double *partials, int max_blocks, double *out,
                           hipStream_t st)
{
    int n = d.nx * d.ny;
    int blocks = (n + 255) / 256;
    if (blocks > max_blocks) blocks = max_blocks;
    double dA = 1.0 / (d.rdx * d.rdy);
    int nv = d.eqn == EULER ? 4 : 3;
    if (d.eqn == EULER)
        hipLaunchKernelGGL((totals_partial_kernel<T, EULER>), dim3(blocks), dim3(256), 0, st, (const T *)q, n, dA,
                           d.g, partials);
    else
        hipLaunchKernelGGL((totals_partial_kernel<T, SWE>), dim3(blocks), dim3(256), 0, st, (const T *)q, n, dA,
                           d.g, partials);
    hipLaunchKernelGGL(totals_final_kernel, dim3(nv + 1), dim3(256), 0, st, partials, blocks, nv + 1, out);
    return hipGetLastError();
}

hipError_t launch_totals(const StageDesc &d, const void *q, double *partials, int max_blocks, double *out_dev,
                         hipStream_t st)
{
    return d.prec == 1 ? totals_t<double>(d, q, partials, max_blocks, out_dev, st)
                       : totals_t<float>(d, q, partials, max_blocks, out_dev, st);
}

template <typename T, int EQN, int FLUX>
static hipError_t face_r(const StageDesc &d, const void *q, void *fx, void *fy, hipStream_t st)
{
    int nf = (d.nx + 1) * d.ny + d.nx * (d.ny + 1);
    Phys<T> ph{(T)d.g, (T)__builtin_sqrt(d.g), (T)d.gamma, T(0)};  // exported fluxes carry the full pressure
    dim3 grid((nf + 255) / 256);
    if (d.recon == FIRST)
        hipLaunchKernelGGL((face_kernel<T, EQN, FLUX, FIRST>), grid, dim3(256), 0, st, (const T *)q, d.nx, d.ny,
                           d.bc_x, d.bc_y, ph, (T *)fx, (T *)fy);
    else
        hipLaunchKernelGGL((face_kernel<T, EQN, FLUX, MINMOD>), grid, dim3(256), 0, st, (const T *)q, d.nx, d.ny,
                           d.bc_x, d.bc_y, ph, (T *)fx, (T *)fy);
    return hipGetLastError();
}

template <typename T, int EQN>
static hipError_t face_f(const StageDesc &d, const void *q, void *fx, void *fy, hipStream_t st)
{
    switch (d.flux) {
    case RUSANOV: return face_r<T, EQN, RUSANOV>(d, q, fx, fy, st);
    case ROE: return face_r<T, EQN, ROE>(d, q, fx, fy, st);
    default: return face_r<T, EQN, HLLE>(d, q, fx, fy, st);
    }
}

template <typename T>
static hipError_t face_p(const StageDesc &d, const void *q, void *fx, void *fy, hipStream_t st)
{
    return d.eqn == EULER ? face_f<T, EULER>(d, q, fx, fy, st) : face_f<T, SWE>(d, q, fx, fy, st);
}

hipError_t launch_face_fluxes(const StageDesc &d, const void *q, void *fx, void *fy, hipStream_t st)
{
    return d.prec == 1 ? face_p<double>(d, q, fx, fy, st) : face_p<float>(d, q, fx, fy, st);
}

}  // namespace fvk
