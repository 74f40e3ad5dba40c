// C-ABI host side of libfv: configuration checks, workspace layout, step
// sequencing and the documented sync points.  All device work is enqueued on
// the caller's stream; Delta t stays on the device (three rotating rate slots:
// step n reads slot n%3, its last stage reduces into (n+1)%3 and clears
// (n+2)%3, so one launch per stage suffices and no memset is recorded).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "api_common.hpp"
#include "fv_internal.hpp"

namespace fvapi {

thread_local std::string g_err;

fv_status fail(fv_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

fv_status hip_fail(hipError_t e, const char *what)
{
    return fail(FV_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char *last_error() { return g_err.c_str(); }

}  // namespace fvapi

using fvapi::align256;
using fvapi::fail;
using fvapi::hip_fail;

namespace {

struct Layout {
    size_t ctl, rates, totals_out, partials, s1, s2;
    // buffers of the learned step (cfg.learned == 1)
    size_t act0, act1, z, s2l, small, lbatch;
    size_t total;
};

int nvar_of(const fv_config *c) { return c->eqn == FV_EULER ? 4 : 3; }

// A solve in the configuration the server runs (FP32, HLLE, MINMOD, Heun,
// CFL-controlled Delta t) steps through the server's stage arithmetic, so it
// computes bit-identical results alone and in a mix; its descriptor and the
// three per-step list entries (one per rotation of the CFL slots) are kept
// host-side and passed to the stage kernels by value.

// The learned step's descriptor and its two one-item lists (flag slot 0
// and 1) for the work-list kernels, as the server uses them.
constexpr size_t LB_TAB = 0, LB_ITEMS = 128, LB_N = 192, LBATCH_BYTES = 256;
static_assert(sizeof(cnn::LSolve) <= LB_ITEMS && LB_ITEMS + 2 * sizeof(cnn::LItem) <= LB_N, "learned batch layout");

bool runs_batched(const fv_config *c)
{
    return c->prec == FV_F32 && c->flux == FV_FLUX_HLLE && c->recon == FV_RECON_MINMOD && c->rk_stages == 2 &&
           !(c->dt_fixed > 0) && !c->learned;
}

fv_status validate(const fv_config *c)
{
    if (!c) return fail(FV_E_INVALID, "config is NULL");
    if (c->struct_size != sizeof(fv_config))
        return fail(FV_E_INVALID, "struct_size %u != sizeof(fv_config) %zu", c->struct_size, sizeof(fv_config));
    if (c->eqn != FV_SWE && c->eqn != FV_EULER) return fail(FV_E_INVALID, "eqn %d", c->eqn);
    if (c->prec != FV_F32 && c->prec != FV_F64) return fail(FV_E_INVALID, "prec %d", c->prec);
    if (c->nx < 4 || c->ny < 4) return fail(FV_E_INVALID, "grid %dx%d: each side must be >= 4", c->nx, c->ny);
    if ((int64_t)c->nx * c->ny > (int64_t)1 << 30) return fail(FV_E_INVALID, "grid too large");
    for (int bc : {c->bc_x, c->bc_y})
        if (bc != FV_BC_PERIODIC && bc != FV_BC_WALL) return fail(FV_E_INVALID, "boundary %d", bc);
    if (c->flux < FV_FLUX_HLLE || c->flux > FV_FLUX_ROE) return fail(FV_E_INVALID, "flux %d", c->flux);
    if (c->recon != FV_RECON_MINMOD && c->recon != FV_RECON_FIRST) return fail(FV_E_INVALID, "recon %d", c->recon);
    if (c->rk_stages < 1 || c->rk_stages > 3) return fail(FV_E_INVALID, "rk_stages %d", c->rk_stages);
    if (c->learned != 0 && c->learned != 1) return fail(FV_E_INVALID, "learned %d", c->learned);
    if (!(c->lx > 0) || !(c->ly > 0)) return fail(FV_E_INVALID, "domain size");
    if (!(c->dt_fixed > 0) && !(c->cfl > 0 && c->cfl <= 1)) return fail(FV_E_INVALID, "cfl %g not in (0,1]", c->cfl);
    if (c->eqn == FV_SWE && !(c->g > 0)) return fail(FV_E_INVALID, "g %g", c->g);
    if (c->eqn == FV_EULER && !(c->gamma > 1)) return fail(FV_E_INVALID, "gamma %g", c->gamma);
    if (!(c->h_ref >= 0)) return fail(FV_E_INVALID, "h_ref %g < 0", c->h_ref);
    return FV_OK;
}

Layout layout_of(const fv_config *c)
{
    Layout L;
    size_t es = c->prec == FV_F64 ? 8 : 4;
    size_t st = align256((size_t)nvar_of(c) * c->nx * c->ny * es);
    L.ctl = 0;
    L.rates = fvk::CTL_BYTES;
    L.totals_out = L.rates + fvk::RATE_BYTES;
    L.partials = L.totals_out + 256;
    L.s1 = L.partials + align256((size_t)fvk::TOTALS_MAX_BLOCKS * 5 * sizeof(double));
    L.s2 = L.s1 + st;
    size_t end = L.s2 + (c->rk_stages == 3 ? st : 0);
    if (c->learned) {
        size_t npix = (size_t)c->nx * c->ny;
        L.act0 = end;
        L.act1 = L.act0 + align256(npix * cnn::CH * 2);
        L.z = L.act1 + align256(npix * cnn::CH * 2);
        L.s2l = L.z + align256(npix * cnn::COUT * 4);
        L.small = L.s2l + st;
        L.lbatch = L.small + 256;
        end = L.lbatch + LBATCH_BYTES;
    } else {
        L.act0 = L.act1 = L.z = L.s2l = L.small = L.lbatch = 0;
    }
    L.total = end;
    return L;
}

}  // namespace

struct fv_solver {
    fv_config cfg;
    fvk::StageDesc d;
    void *q;
    const void *bed;
    char *ws;
    Layout L;
    hipStream_t stream;
    int64_t enq;  // steps enqueued since the last rate initialisation
    int64_t lsteps;  // learned steps enqueued (picks the slot of the step's flags)
    size_t state_bytes;
    bool batched;
    fvk::BatchSolve bd;  // batched: the descriptor and the three step entries, as uploaded
    fvk::WorkItem bi[3];
    fvk::Ctl *ctl() { return (fvk::Ctl *)(ws + L.ctl); }
    unsigned long long *rates() { return (unsigned long long *)(ws + L.rates); }
};

namespace {

fv_status init_rate(fv_solver *s)
{
    // rate slots, time and flags are reset by a host->device copy of a fresh
    // control block (ordered on the stream before any kernel that reads it)
    s->enq = 0;
    int slot = 0;
    hipError_t e = hipMemsetAsync(s->rates(), 0, fvk::RATE_BYTES, s->stream);
    if (e == hipSuccess) e = fvk::launch_rate(s->d, s->q, s->ctl(), s->rates(), slot, s->stream);
    if (e != hipSuccess) return hip_fail(e, "rate kernel");
    return FV_OK;
}

fv_status sync_and_check(fv_solver *s)
{
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int bad = 0;
    e = hipMemcpy(&bad, &s->ctl()->bad, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read flag");
    if (bad) return fail(FV_E_INADMISSIBLE, "a cell became inadmissible (h<=0, rho<=0, p<=0 or non-finite)");
    return FV_OK;
}

fv_status enqueue_step(fv_solver *s)
{
    const int n = (int)(s->enq % 3);
    const bool cfl = !(s->cfg.dt_fixed > 0);
    const int ri = n, ro = cfl ? (n + 1) % 3 : -1, rc = cfl ? (n + 2) % 3 : -1;
    char *S1 = s->ws + s->L.s1, *S2 = s->ws + s->L.s2;
    hipError_t e = hipSuccess;
    fvk::Ctl *ctl = s->ctl();
    if (s->batched) {
        // the server's stage arithmetic on the solve's descriptor, passed by
        // value (the copy in the workspace serves the learned kernels' list form)
        const int tiles = ((s->cfg.nx + fvk::TILE_X - 1) / fvk::TILE_X) * ((s->cfg.ny + fvk::TILE_Y - 1) / fvk::TILE_Y);
        e = fvk::launch_batch_stage_one(s->d.eqn, s->d.bathy, 1, s->bd, s->bi[n], tiles, s->stream);
        if (e == hipSuccess) e = fvk::launch_batch_stage_one(s->d.eqn, s->d.bathy, 2, s->bd, s->bi[n], tiles, s->stream);
        if (e != hipSuccess) return hip_fail(e, "stage launch");
        s->enq++;
        return FV_OK;
    }
    switch (s->cfg.rk_stages) {
    case 1:
        e = fvk::launch_stage(s->d, s->q, s->q, S1, s->bed, 0.0, 1.0, ctl, s->rates(), ri, ro, rc, 1, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s->q, S1, s->state_bytes, hipMemcpyDeviceToDevice, s->stream);
        break;
    case 2:
        e = fvk::launch_stage(s->d, s->q, s->q, S1, s->bed, 0.0, 1.0, ctl, s->rates(), ri, -1, -1, 0, s->stream);
        if (e == hipSuccess)
            e = fvk::launch_stage(s->d, S1, s->q, s->q, s->bed, 0.5, 0.5, ctl, s->rates(), ri, ro, rc, 1, s->stream);
        break;
    default:
        e = fvk::launch_stage(s->d, s->q, s->q, S1, s->bed, 0.0, 1.0, ctl, s->rates(), ri, -1, -1, 0, s->stream);
        if (e == hipSuccess)
            e = fvk::launch_stage(s->d, S1, s->q, S2, s->bed, 0.75, 0.25, ctl, s->rates(), ri, -1, -1, 0, s->stream);
        if (e == hipSuccess)
            e = fvk::launch_stage(s->d, S2, s->q, s->q, s->bed, 1.0 / 3.0, 2.0 / 3.0, ctl, s->rates(), ri, ro, rc, 1, s->stream);
        break;
    }
    if (e != hipSuccess) return hip_fail(e, "stage launch");
    s->enq++;
    return FV_OK;
}

// offsets inside the 256-byte block of learned counters
constexpr size_t SM_DT = 0, SM_BAD = 8, SM_NFB = 16, SM_REDONE = 24;

// The solve's descriptor for the learned kernels (device pointers into the
// solver's workspace and control block).
static cnn::LSolve lsolve_of(fv_solver *s)
{
    char *ws = s->ws, *sm = ws + s->L.small;
    cnn::LSolve d{};
    d.q = (float *)s->q;
    d.s1 = (float *)(ws + s->L.s1);
    d.s2 = (float *)(ws + s->L.s2l);
    d.z = (float *)(ws + s->L.z);
    d.dt = (const float *)(sm + SM_DT);
    d.flags = (int *)(sm + SM_BAD);
    d.nfb = (unsigned long long *)(sm + SM_NFB);
    d.redone = (unsigned long long *)(sm + SM_REDONE);
    d.fatal = &s->ctl()->bad;
    d.t = &s->ctl()->t;
    d.steps = &s->ctl()->step;
    d.nx = s->cfg.nx;
    d.ny = s->cfg.ny;
    d.rdx = (float)s->d.rdx;
    d.rdy = (float)s->d.rdy;
    d.g = (float)s->cfg.g;
    d.sqg = std::sqrt((float)s->cfg.g);
    d.h0 = (float)s->d.h0;
    return d;
}

fv_status upload_lbatch(fv_solver *s)
{
    alignas(16) char buf[LBATCH_BYTES];
    std::memset(buf, 0, sizeof buf);
    char *ws = s->ws;
    const cnn::LSolve d = lsolve_of(s);
    std::memcpy(buf + LB_TAB, &d, sizeof d);
    for (int p = 0; p < 2; p++) {
        cnn::LItem it{0, 0, 0, p};
        std::memcpy(buf + LB_ITEMS + p * sizeof it, &it, sizeof it);
    }
    const int one = 1;
    std::memcpy(buf + LB_N, &one, sizeof one);
    hipError_t e = hipMemcpyAsync(ws + s->L.lbatch, buf, sizeof buf, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // buf is on this stack frame
    if (e != hipSuccess) return hip_fail(e, "learned descriptor upload");
    return FV_OK;
}

// Descriptor and step list entries of the batch-of-one path (see
// runs_batched).
void batch_block(fv_solver *s)
{
    fvk::BatchSolve d{};
    d.q = s->q;
    d.s1 = s->ws + s->L.s1;
    d.bed = s->bed;
    d.ctl = s->ctl();
    d.rates = s->rates();
    d.nx = s->cfg.nx;
    d.ny = s->cfg.ny;
    d.bc_x = s->cfg.bc_x;
    d.bc_y = s->cfg.bc_y;
    d.rdx = s->d.rdx;
    d.rdy = s->d.rdy;
    d.g = s->cfg.g;
    d.sqg = std::sqrt(s->cfg.g);
    d.gamma = s->cfg.gamma;
    d.h0 = s->d.h0;
    d.cfl = s->cfg.cfl;
    d.dt_fixed = 0.0;
    s->bd = d;
    for (int k = 0; k < 3; k++) {
        fvk::WorkItem it{};
        it.solve = 0;
        it.tile_begin = 0;
        it.tiles_x = (s->cfg.nx + fvk::TILE_X - 1) / fvk::TILE_X;
        it.ri = (unsigned char)k;
        it.ro = (unsigned char)((k + 1) % 3);
        it.rc = (unsigned char)((k + 2) % 3);
        s->bi[k] = it;
    }
}

// The solver fields fv_init and fv_run_noalloc share (h0 is set by the caller).
void setup_solver(fv_solver *s, const fv_config *cfg, void *q, const void *bathy, char *ws, const Layout &L,
                  hipStream_t stream)
{
    s->cfg = *cfg;
    s->q = q;
    s->bed = bathy;
    s->ws = ws;
    s->L = L;
    s->stream = stream;
    s->enq = 0;
    s->lsteps = 0;
    s->state_bytes = (size_t)nvar_of(cfg) * cfg->nx * cfg->ny * (cfg->prec == FV_F64 ? 8 : 4);
    fvk::StageDesc &d = s->d;
    d.prec = cfg->prec;
    d.eqn = cfg->eqn;
    d.bathy = bathy ? 1 : 0;
    d.flux = cfg->flux;
    d.recon = cfg->recon;
    d.nx = cfg->nx;
    d.ny = cfg->ny;
    d.bc_x = cfg->bc_x;
    d.bc_y = cfg->bc_y;
    d.rdx = cfg->nx / cfg->lx;
    d.rdy = cfg->ny / cfg->ly;
    d.g = cfg->g;
    d.gamma = cfg->gamma;
    d.cfl = cfg->cfl;
    d.dt_fixed = cfg->dt_fixed;
    d.h0 = 0.0;
    s->batched = runs_batched(cfg);
}

}  // namespace

extern "C" {

int fv_nvar(const fv_config *cfg) { return cfg ? nvar_of(cfg) : 0; }

size_t fv_workspace_bytes(const fv_config *cfg)
{
    if (validate(cfg) != FV_OK) return 0;
    return layout_of(cfg).total;
}

fv_status fv_init(const fv_config *cfg, void *q, const void *bathy, void *workspace, size_t workspace_bytes,
                  void *stream, fv_solver **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    fv_status rc = validate(cfg);
    if (rc != FV_OK) return rc;
    if (!q || !workspace) return fail(FV_E_INVALID, "state or workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(FV_E_INVALID, "workspace must be 256-byte aligned");
    if (bathy && cfg->eqn != FV_SWE) return fail(FV_E_INVALID, "a bed is only defined for the shallow-water equations");
    Layout L = layout_of(cfg);
    if (workspace_bytes < L.total)
        return fail(FV_E_NOMEM, "workspace %zu bytes < required %zu", workspace_bytes, L.total);

    fv_solver *s = new fv_solver();
    setup_solver(s, cfg, q, bathy, (char *)workspace, L, (hipStream_t)stream);

    fvk::Ctl fresh;
    std::memset(&fresh, 0, sizeof fresh);
    hipError_t e = hipMemcpyAsync(s->ctl(), &fresh, sizeof fresh, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "control block upload");
    }
    if (cfg->learned) {
        // learned-step counters: dt (float), bad, pad, nfb, redone
        char small[256];
        std::memset(small, 0, sizeof small);
        float dtf = (float)cfg->dt_fixed;
        std::memcpy(small, &dtf, sizeof dtf);
        e = hipMemcpyAsync(s->ws + L.small, small, sizeof small, hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "learned counters upload");
        }
    }
    rc = init_rate(s);
    if (rc == FV_OK) rc = sync_and_check(s);
    if (rc == FV_OK && cfg->eqn == FV_SWE && cfg->h_ref > 0) {
        s->d.h0 = cfg->h_ref;
    } else if (rc == FV_OK && cfg->eqn == FV_SWE) {
        // reference depth of the pressure term: mean initial depth
        double tot[5];
        rc = fv_totals(s, tot);
        if (rc == FV_OK) s->d.h0 = tot[0] / (cfg->lx * cfg->ly);
    }
    if (rc == FV_OK && s->batched) batch_block(s);
    if (rc == FV_OK && cfg->learned) rc = upload_lbatch(s);
    if (rc != FV_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return FV_OK;
}

fv_status fv_step(fv_solver *s)
{
    if (!s) return fail(FV_E_INVALID, "solver is NULL");
    return enqueue_step(s);
}

fv_status fv_run(fv_solver *s, int64_t nsteps)
{
    if (!s) return fail(FV_E_INVALID, "solver is NULL");
    if (nsteps < 0) return fail(FV_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    for (int64_t k = 0; k < nsteps; k++) {
        fv_status rc = enqueue_step(s);
        if (rc != FV_OK) return rc;
    }
    return FV_OK;
}

fv_status fv_time(fv_solver *s, double *t, int64_t *step)
{
    if (!s) return fail(FV_E_INVALID, "solver is NULL");
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    fvk::Ctl c;
    e = hipMemcpy(&c, s->ctl(), sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read control block");
    if (t) *t = c.t;
    if (step) *step = c.step;
    if (c.bad) return fail(FV_E_INADMISSIBLE, "a cell became inadmissible at step %lld", (long long)c.step);
    return FV_OK;
}

fv_status fv_totals(fv_solver *s, double *out)
{
    if (!s || !out) return fail(FV_E_INVALID, "NULL argument");
    double *dev_out = (double *)(s->ws + s->L.totals_out);
    double *partials = (double *)(s->ws + s->L.partials);
    hipError_t e = fvk::launch_totals(s->d, s->q, partials, fvk::TOTALS_MAX_BLOCKS, dev_out, s->stream);
    if (e != hipSuccess) return hip_fail(e, "totals launch");
    e = hipMemcpyAsync(out, dev_out, (nvar_of(&s->cfg) + 1) * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "totals copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return FV_OK;
}

fv_status fv_get_state(fv_solver *s, void *dst, int dst_is_host)
{
    if (!s || !dst) return fail(FV_E_INVALID, "NULL argument");
    hipError_t e = hipMemcpyAsync(dst, s->q, s->state_bytes,
                                  dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "state copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return FV_OK;
}

fv_status fv_set_state(fv_solver *s, const void *src, int src_is_host)
{
    if (!s || !src) return fail(FV_E_INVALID, "NULL argument");
    hipError_t e = hipMemcpyAsync(s->q, src, s->state_bytes,
                                  src_is_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "state copy");
    fvk::Ctl c;
    e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(&c, s->ctl(), sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read control block");
    c.bad = 0;
    e = hipMemcpyAsync(s->ctl(), &c, sizeof c, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "control block upload");
    fv_status rc = init_rate(s);
    if (rc != FV_OK) return rc;
    return sync_and_check(s);
}

void *fv_state_ptr(fv_solver *s) { return s ? s->q : nullptr; }

double fv_reference_depth(const fv_solver *s) { return s ? s->d.h0 : 0.0; }

fv_status fv_set_stream(fv_solver *s, void *stream)
{
    if (!s) return fail(FV_E_INVALID, "solver is NULL");
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    s->stream = (hipStream_t)stream;
    return FV_OK;
}

fv_status fv_face_fluxes(fv_solver *s, void *fx, void *fy)
{
    if (!s || !fx || !fy) return fail(FV_E_INVALID, "NULL argument");
    if (s->bed) return fail(FV_E_UNSUPPORTED, "face export is defined for flat-bottom configurations");
    hipError_t e = fvk::launch_face_fluxes(s->d, s->q, fx, fy, s->stream);
    if (e != hipSuccess) return hip_fail(e, "face kernel");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return FV_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free stepping
//
// fv_run_noalloc runs the kernels of fv_init + fv_run on a device array the
// library holds, `scratch`, instead of a caller workspace.  Host code never
// passes the array's name to a kernel or copy (in host code it is only a
// stand-in for the device symbol): each device's address comes from
// hipGetSymbolAddress on that device's first call and is kept per device.
namespace {

constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
static_assert(NOALLOC_BYTES == FV_NOALLOC_SCRATCH_BYTES, "scratch size in the header");
constexpr int NOALLOC_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

fv_status scratch_on_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(FV_E_UNSUPPORTED, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255) != 0) return fail(FV_E_HIP, "scratch address %p not 256-byte aligned", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FV_OK;
}

}  // namespace

extern "C" {

size_t fv_noalloc_bytes(const fv_config *cfg)
{
    if (validate(cfg) != FV_OK) return 0;
    return layout_of(cfg).total;
}

fv_status fv_run_noalloc(const fv_config *cfg, void *q, const void *bathy, int64_t nsteps, void *stream,
                         fv_run_info *info_dev)
{
    fv_status rc = validate(cfg);
    if (rc != FV_OK) return rc;
    if (!q) return fail(FV_E_INVALID, "state is NULL");
    if (nsteps < 0) return fail(FV_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    if (bathy && cfg->eqn != FV_SWE) return fail(FV_E_INVALID, "a bed is only defined for the shallow-water equations");
    if (cfg->learned) return fail(FV_E_UNSUPPORTED, "the allocation-free path runs the classic scheme only (learned = 0)");
    if (cfg->eqn == FV_SWE && !(cfg->h_ref > 0))
        return fail(FV_E_INVALID, "the allocation-free path needs h_ref > 0 for shallow water (no reduction of the initial depth)");
    const Layout L = layout_of(cfg);
    if (L.total > NOALLOC_BYTES)
        return fail(FV_E_NOMEM, "this configuration needs %zu bytes of scratch; the allocation-free path holds %zu",
                    L.total, NOALLOC_BYTES);
    void *ws = nullptr;
    rc = scratch_on_current_device(&ws);
    if (rc != FV_OK) return rc;

    fv_solver s;
    setup_solver(&s, cfg, q, bathy, (char *)ws, L, (hipStream_t)stream);
    s.d.h0 = cfg->eqn == FV_SWE ? cfg->h_ref : 0.0;
    if (s.batched) batch_block(&s);
    hipError_t e = fvk::launch_reset(s.ctl(), s.rates(), s.stream);
    if (e == hipSuccess) e = fvk::launch_rate(s.d, s.q, s.ctl(), s.rates(), 0, s.stream);
    if (e != hipSuccess) return hip_fail(e, "reset and rate kernels");
    for (int64_t k = 0; k < nsteps; k++) {
        rc = enqueue_step(&s);
        if (rc != FV_OK) return rc;
    }
    if (info_dev) {
        e = fvk::launch_report(s.ctl(), info_dev, s.stream);
        if (e != hipSuccess) return hip_fail(e, "report kernel");
    }
    return FV_OK;
}

void fv_destroy(fv_solver *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

const char *fv_last_error(void) { return fvapi::last_error(); }

}  // extern "C"

// ------------------------------------------------------------ learned path

extern "C" {

size_t fv_model_param_count(void) { return cnn::NPARAM; }

size_t fv_model_workspace_bytes(const fv_model_desc *desc)
{
    if (!desc || desc->struct_size != sizeof(fv_model_desc) || desc->hidden != 32) return 0;
    return cnn::packed_layout().bytes;
}

fv_status fv_model_create(const fv_model_desc *desc, const float *params, void *workspace, size_t workspace_bytes,
                          void *stream, fv_model **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!desc || desc->struct_size != sizeof(fv_model_desc)) return fail(FV_E_INVALID, "model desc struct_size");
    if (desc->hidden != 32) return fail(FV_E_UNSUPPORTED, "hidden width %d (the kernels implement 32)", desc->hidden);
    if (desc->order < 0 || desc->order > 1) return fail(FV_E_INVALID, "constraint order %d", desc->order);
    if (desc->reserved0 != 0) return fail(FV_E_INVALID, "reserved0 must be 0");
    if (!params || !workspace) return fail(FV_E_INVALID, "params or workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(FV_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < cnn::packed_layout().bytes)
        return fail(FV_E_NOMEM, "model workspace %zu < %zu", workspace_bytes, cnn::packed_layout().bytes);
    fv_model *m = new fv_model();
    m->desc = *desc;
    m->params = params;
    m->packed = workspace;
    m->stream = (hipStream_t)stream;
    for (int c = 0; c < 3; c++) {
        m->nrm.mean[c] = desc->mean[c];
        m->nrm.inv_std[c] = desc->inv_std[c];
    }
    m->pr = cnn::make_projection(desc->order);
    hipError_t e = cnn::launch_pack(params, workspace, m->stream);
    if (e != hipSuccess) {
        delete m;
        return hip_fail(e, "pack kernel");
    }
    *out = m;
    return FV_OK;
}

fv_status fv_model_update(fv_model *m)
{
    if (!m) return fail(FV_E_INVALID, "model is NULL");
    hipError_t e = cnn::launch_pack(m->params, m->packed, m->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "pack kernel");
}

void fv_model_destroy(fv_model *m) { delete m; }

size_t fv_model_forward_scratch_bytes(int B, int nx, int ny)
{
    if (B <= 0 || nx <= 0 || ny <= 0) return 0;
    return 2 * align256((size_t)B * nx * ny * cnn::CH * 2);
}

fv_status fv_model_forward(const fv_model *m, const float *q, int B, int nx, int ny, float *z, void *scratch,
                           size_t scratch_bytes)
{
    if (!m || !q || !z || !scratch) return fail(FV_E_INVALID, "NULL argument");
    if (B <= 0 || nx < 16 || ny < 2 || nx % 16 || ((int64_t)nx * ny) % 64)
        return fail(FV_E_UNSUPPORTED, "network grids need nx %% 16 == 0 and nx*ny %% 64 == 0 (got %dx%d)", nx, ny);
    if (((uintptr_t)scratch & 255) != 0) return fail(FV_E_INVALID, "scratch must be 256-byte aligned");
    size_t need = fv_model_forward_scratch_bytes(B, nx, ny);
    if (scratch_bytes < need) return fail(FV_E_NOMEM, "scratch %zu < %zu", scratch_bytes, need);
    char *sc = (char *)scratch;
    size_t half = need / 2;
    void *acts[4] = {sc, sc + half, sc, sc + half};
    hipError_t e = cnn::launch_forward(m->packed, m->nrm, q, B, nx, ny, acts, z, m->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "network launch");
}

fv_status fv_model_forward_tiled(const fv_model *m, const float *q, int B, int nx, int ny, float *z)
{
    if (!m || !q || !z) return fail(FV_E_INVALID, "NULL argument");
    if (B <= 0 || nx < 8 || ny < 8 || nx % 8 || ny % 8)
        return fail(FV_E_UNSUPPORTED, "the tiled network pass needs nx %% 8 == 0 and ny %% 8 == 0 (got %dx%d)", nx, ny);
    hipError_t e = cnn::launch_forward_fused(m->packed, m->nrm, q, B, nx, ny, z, m->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "network launch");
}

// blend: the flux-limiter blend of the face fluxes; direct: the direct
// face-state scheme; callers pass either only where the two-launch branch
// below runs (HLLE, nx % 8 == ny % 8 == 0, below the split size).
static fv_status learned_step_impl(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats,
                                   int blend, int direct = 0)
{
    if (!s || !m) return fail(FV_E_INVALID, "NULL argument");
    const fv_config &c = s->cfg;
    if (c.eqn != FV_SWE || c.prec != FV_F32 || c.bc_x != FV_BC_PERIODIC || c.bc_y != FV_BC_PERIODIC || s->bed ||
        c.rk_stages != 2 || !(c.dt_fixed > 0) || !c.learned || c.nx % 16 || ((int64_t)c.nx * c.ny) % 64 ||
        (c.flux != FV_FLUX_HLLE && c.flux != FV_FLUX_RUSANOV))
        return fail(FV_E_UNSUPPORTED,
                    "learned steps need SWE, FP32, periodic, flat bed, Heun, dt_fixed > 0, learned = 1, "
                    "HLLE or Rusanov, nx %% 16 == 0 and nx*ny %% 64 == 0");
    if (nsteps < 0) return fail(FV_E_INVALID, "nsteps < 0");
    char *ws = s->ws;
    const Layout &L = s->L;
    float *q = (float *)s->q;
    float *S1 = (float *)(ws + L.s1), *S2 = (float *)(ws + L.s2l), *z = (float *)(ws + L.z);
    char *sm = ws + L.small;
    void *acts[4] = {ws + L.act0, ws + L.act1, ws + L.act0, ws + L.act1};
    cnn::StageBatch sb{};
    sb.B = 1;
    sb.nx = c.nx;
    sb.ny = c.ny;
    sb.rdx = (float)s->d.rdx;
    sb.rdy = (float)s->d.rdy;
    sb.g = (float)c.g;
    sb.h0 = (float)s->d.h0;
    sb.dt = (const float *)(sm + SM_DT);
    sb.bad = (int *)(sm + SM_BAD);
    sb.nfb = (unsigned long long *)(sm + SM_NFB);
    sb.fatal = &s->ctl()->bad;
    sb.pr = m->pr;
    sb.z = z;
    const int fl = c.flux == FV_FLUX_RUSANOV ? 1 : 0;  // kernel flux ids: 0 HLLE, 1 Rusanov
    hipError_t e = hipSuccess;
    if (fl == 0 && c.nx % 8 == 0 && c.ny % 8 == 0 &&
        cnn::ltiles_cnn(c.nx, c.ny) < 4 * cnn::fused_max_grid()) {
        // two launches per step, each the network pass with the learned
        // stage (the server's per-stage arithmetic, so bit-identical to the
        // same solve in a served mix): the step's output goes to the other
        // buffer of the pair (q, S2), its input stays for a redo, which the
        // next step's first launch carries out where needed; the call's last
        // step ends with the commit-or-redo and redo launches
        cnn::LSolve d = lsolve_of(s);
        float *X[2] = {q, S2};
        int *flags = (int *)(sm + SM_BAD);
        for (int64_t k = 0; k < nsteps && e == hipSuccess; k++, s->lsteps++) {
            const int par = (int)(s->lsteps & 1);
            d.q = X[k & 1];
            d.s2 = X[(k + 1) & 1];
            e = cnn::launch_conv_learned_one(1, m->packed, m->nrm, m->pr, d, par, k > 0 ? X[(k + 1) & 1] : nullptr,
                                             s->stream, blend, direct);
            if (e == hipSuccess)
                e = cnn::launch_conv_learned_one(2, m->packed, m->nrm, m->pr, d, par, nullptr, s->stream, blend, direct);
        }
        if (nsteps > 0 && e == hipSuccess) {
            // the last step's input xin and output xout: with an odd step
            // count (q, S2), commit S2 -> q or redo from q; with an even one
            // (S2, q), the result is in q already, or the step is redone from S2
            float *xin = X[(nsteps - 1) & 1], *xout = X[nsteps & 1];
            const int par = (int)((s->lsteps - 1) & 1);
            sb.bad = flags + par;
            sb.bad_next = flags + (par ^ 1);
            sb.redone = (unsigned long long *)(sm + SM_REDONE);
            sb.t = nullptr;  // advanced by each step's second launch
            sb.steps = nullptr;
            sb.qs = xin; sb.q0 = xin; sb.out = S1; sb.a0 = 0.f; sb.a1 = 1.f;
            sb.commit_src = xout == q ? nullptr : xout;
            sb.commit_dst = q;
            e = cnn::learned_stage(2, fl, sb, s->stream);
            sb.qs = S1; sb.q0 = xin; sb.out = q; sb.a0 = 0.5f; sb.a1 = 0.5f;
            if (e == hipSuccess) e = cnn::learned_stage(3, fl, sb, s->stream);
        }
        nsteps = 0;  // done; fall through to the statistics
    } else if (fl == 0 && c.nx % 8 == 0 && c.ny % 8 == 0) {
        // larger grids: the server's work-list kernels as a batch of one,
        // the network pass and the learned stage as separate launches, then
        // commit-or-redo and redo; bit-identical to the same solve in a
        // served mix
        const char *B = ws + L.lbatch;
        const auto *tab = (const cnn::LSolve *)(B + LB_TAB);
        const auto *items0 = (const cnn::LItem *)(B + LB_ITEMS);
        const int *nit = (const int *)(B + LB_N);
        const int tc = cnn::ltiles_cnn(c.nx, c.ny), ts = cnn::ltiles_st(c.nx, c.ny);
        if (blend || direct) return fail(FV_E_UNSUPPORTED, "blend or direct: grid too large for the fused form");
        for (int64_t k = 0; k < nsteps && e == hipSuccess; k++, s->lsteps++) {
            const cnn::LItem *it = items0 + (s->lsteps & 1);
            for (int stage = 1; stage <= 2 && e == hipSuccess; stage++) {
                e = cnn::launch_forward_batch(stage, m->packed, m->nrm, m->pr, tab, it, nit, tc, s->stream, 1);
                if (e == hipSuccess) e = cnn::launch_learned_batch(0, stage, tab, it, nit, ts, m->pr, s->stream, 1);
            }
            if (e == hipSuccess) e = cnn::launch_learned_batch(2, 0, tab, it, nit, ts, m->pr, s->stream, 1);
            if (e == hipSuccess) e = cnn::launch_learned_batch(3, 0, tab, it, nit, ts, m->pr, s->stream, 1);
        }
        nsteps = 0;  // done; fall through to the statistics
    }
    const bool fused = c.ny % 8 == 0;  // whole network in one launch per evaluation
    int *flags = (int *)(sm + SM_BAD);  // two slots: this step's and the next step's
    sb.redone = (unsigned long long *)(sm + SM_REDONE);
    sb.t = &s->ctl()->t;
    sb.steps = &s->ctl()->step;
    // the tiled network pass also applies the projection: z then holds alpha
    sb.alpha = fused ? 1 : 0;
    auto forward = [&](const float *in) {
        return fused ? cnn::launch_forward_fused(m->packed, m->nrm, in, 1, c.nx, c.ny, z, s->stream, &m->pr)
                     : cnn::launch_forward(m->packed, m->nrm, in, 1, c.nx, c.ny, acts, z, s->stream);
    };
    for (int64_t k = 0; k < nsteps && e == hipSuccess; k++, s->lsteps++) {
        sb.bad = flags + (s->lsteps & 1);
        sb.bad_next = flags + ((s->lsteps + 1) & 1);
        // stage 1: coefficients of q, q1 = q + dt L(q)
        e = forward(q);
        sb.qs = q; sb.q0 = q; sb.out = S1; sb.a0 = 0.f; sb.a1 = 1.f; sb.flagbit = 1;
        if (e == hipSuccess) e = cnn::learned_stage(0, fl, sb, s->stream);
        // stage 2: coefficients of q1, q2 = q/2 + (q1 + dt L(q1))/2
        if (e == hipSuccess) e = forward(S1);
        sb.qs = S1; sb.q0 = q; sb.out = S2; sb.a0 = 0.5f; sb.a1 = 0.5f; sb.flagbit = 2;
        if (e == hipSuccess) e = cnn::learned_stage(0, fl, sb, s->stream);
        // admissible: q <- S2; otherwise redo the step with the plain scheme
        sb.qs = q; sb.q0 = q; sb.out = S1; sb.a0 = 0.f; sb.a1 = 1.f;
        sb.commit_src = S2; sb.commit_dst = q;
        if (e == hipSuccess) e = cnn::learned_stage(2, fl, sb, s->stream);
        sb.qs = S1; sb.q0 = q; sb.out = q; sb.a0 = 0.5f; sb.a1 = 0.5f;
        if (e == hipSuccess) e = cnn::learned_stage(3, fl, sb, s->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "learned step launch");
    if (stats) {
        e = hipStreamSynchronize(s->stream);
        unsigned long long cnt[2];
        if (e == hipSuccess) e = hipMemcpy(cnt, sm + SM_NFB, sizeof cnt, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read learned counters");
        stats->fallback_faces = (int64_t)cnt[0];
        stats->redone_steps = (int64_t)cnt[1];
    }
    return FV_OK;
}

// Direct face-state scheme (thesis section 5.3): per stage the network pass
// (raw output in z) and the direct stage; then the learned step's
// commit-or-redo and redo launches.
// Heun steps of a scheme whose stages take the network's raw output (one
// network pass per stage, then the stage kernel): the direct face-state
// scheme (direct) or the learned scheme with the flux-limiter blend (blend).
// The end of a step (commit or plain redo) is the learned step's.
static fv_status raw_head_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats, int direct,
                               int blend)
{
    if (!s || !m) return fail(FV_E_INVALID, "NULL argument");
    const fv_config &c = s->cfg;
    if (c.eqn != FV_SWE || c.prec != FV_F32 || c.bc_x != FV_BC_PERIODIC || c.bc_y != FV_BC_PERIODIC || s->bed ||
        c.rk_stages != 2 || !(c.dt_fixed > 0) || !c.learned || c.nx % 16 || ((int64_t)c.nx * c.ny) % 64 ||
        (c.flux != FV_FLUX_HLLE && c.flux != FV_FLUX_RUSANOV))
        return fail(FV_E_UNSUPPORTED,
                    "%s steps need SWE, FP32, periodic, flat bed, Heun, dt_fixed > 0, learned = 1, "
                    "HLLE or Rusanov, nx %% 16 == 0 and nx*ny %% 64 == 0", direct ? "direct" : "blend");
    if (nsteps < 0) return fail(FV_E_INVALID, "nsteps < 0");
    char *ws = s->ws;
    const Layout &L = s->L;
    float *q = (float *)s->q;
    float *S1 = (float *)(ws + L.s1), *S2 = (float *)(ws + L.s2l), *z = (float *)(ws + L.z);
    char *sm = ws + L.small;
    void *acts[4] = {ws + L.act0, ws + L.act1, ws + L.act0, ws + L.act1};
    cnn::StageBatch sb{};
    sb.B = 1;
    sb.nx = c.nx;
    sb.ny = c.ny;
    sb.rdx = (float)s->d.rdx;
    sb.rdy = (float)s->d.rdy;
    sb.g = (float)c.g;
    sb.h0 = (float)s->d.h0;
    sb.dt = (const float *)(sm + SM_DT);
    sb.nfb = (unsigned long long *)(sm + SM_NFB);
    sb.fatal = &s->ctl()->bad;
    sb.pr = m->pr;
    sb.z = z;
    for (int v = 0; v < 3; v++) sb.sig[v] = 1.0f / m->nrm.inv_std[v];
    int *flags = (int *)(sm + SM_BAD);  // two slots: this step's and the next step's
    sb.redone = (unsigned long long *)(sm + SM_REDONE);
    sb.t = &s->ctl()->t;
    sb.steps = &s->ctl()->step;
    const int fl = c.flux == FV_FLUX_RUSANOV ? 1 : 0;
    // the network's raw output: one launch per evaluation (the tiled pass,
    // bit-identical) where the grid allows it, else one launch per layer
    const bool tiled = c.ny % 8 == 0;
    auto forward = [&](const float *in) {
        return tiled ? cnn::launch_forward_fused(m->packed, m->nrm, in, 1, c.nx, c.ny, z, s->stream, nullptr)
                     : cnn::launch_forward(m->packed, m->nrm, in, 1, c.nx, c.ny, acts, z, s->stream);
    };
    hipError_t e = hipSuccess;
    for (int64_t k = 0; k < nsteps && e == hipSuccess; k++, s->lsteps++) {
        sb.bad = flags + (s->lsteps & 1);
        sb.bad_next = flags + ((s->lsteps + 1) & 1);
        sb.direct = direct;
        sb.blend = blend;
        // stage 1: face states of q, q1 = q + dt L(q)
        e = forward(q);
        sb.qs = q; sb.q0 = q; sb.out = S1; sb.a0 = 0.f; sb.a1 = 1.f; sb.flagbit = 1;
        if (e == hipSuccess) e = cnn::learned_stage(0, fl, sb, s->stream);
        // stage 2: face states of q1, q2 = q/2 + (q1 + dt L(q1))/2
        if (e == hipSuccess) e = forward(S1);
        sb.qs = S1; sb.q0 = q; sb.out = S2; sb.a0 = 0.5f; sb.a1 = 0.5f; sb.flagbit = 2;
        if (e == hipSuccess) e = cnn::learned_stage(0, fl, sb, s->stream);
        // admissible: q <- S2; otherwise redo the step with the plain scheme
        sb.direct = 0;
        sb.blend = 0;
        sb.qs = q; sb.q0 = q; sb.out = S1; sb.a0 = 0.f; sb.a1 = 1.f;
        sb.commit_src = S2; sb.commit_dst = q;
        if (e == hipSuccess) e = cnn::learned_stage(2, fl, sb, s->stream);
        sb.qs = S1; sb.q0 = q; sb.out = q; sb.a0 = 0.5f; sb.a1 = 0.5f;
        if (e == hipSuccess) e = cnn::learned_stage(3, fl, sb, s->stream);
    }
    if (e != hipSuccess) return hip_fail(e, direct ? "direct step launch" : "blend step launch");
    if (stats) {
        e = hipStreamSynchronize(s->stream);
        unsigned long long cnt[2];
        if (e == hipSuccess) e = hipMemcpy(cnt, sm + SM_NFB, sizeof cnt, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read learned counters");
        stats->fallback_faces = (int64_t)cnt[0];
        stats->redone_steps = (int64_t)cnt[1];
    }
    return FV_OK;
}

fv_status fv_direct_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats)
{
    // HLLE grids of whole 8 x 8 tiles below the split size: the learned
    // step's two-launch form, the network pass (on the tile and a one-cell
    // ring) and the direct stage in one launch per stage; else the network's
    // raw output through HBM and a separate direct stage
    if (s && m && s->cfg.flux == FV_FLUX_HLLE && s->cfg.nx % 8 == 0 && s->cfg.ny % 8 == 0 &&
        cnn::ltiles_cnn(s->cfg.nx, s->cfg.ny) < 4 * cnn::fused_max_grid())
        return learned_step_impl(s, m, nsteps, stats, 0, 1);
    return raw_head_step(s, m, nsteps, stats, 1, 0);
}

fv_status fv_learned_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats)
{
    return learned_step_impl(s, m, nsteps, stats, 0);
}

fv_status fv_blend_step(fv_solver *s, const fv_model *m, int64_t nsteps, fv_learned_stats *stats)
{
    // HLLE grids of whole 8 x 8 tiles below the split size: the network pass
    // and the blended stage in one launch per stage (z stays in LDS); else
    // the network's raw output through HBM and a separate blended stage
    if (s && m && s->cfg.flux == FV_FLUX_HLLE && s->cfg.nx % 8 == 0 && s->cfg.ny % 8 == 0 &&
        cnn::ltiles_cnn(s->cfg.nx, s->cfg.ny) < 4 * cnn::fused_max_grid())
        return learned_step_impl(s, m, nsteps, stats, 1);
    return raw_head_step(s, m, nsteps, stats, 0, 1);
}

}  // extern "C"
