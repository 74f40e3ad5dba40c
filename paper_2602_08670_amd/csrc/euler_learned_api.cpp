// C ABI of the learned Euler step (thesis sections 2.5.3 and 6.2):
// configuration checks, workspace layout and the launch sequence of a Heun
// step (network pass, learned stage, twice; then commit-or-redo in two
// launches); training with the unrolled loss of eq 2.28.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/fv.h"
#include "api_common.hpp"
#include "cnn_internal.hpp"
#include "euler_learned_internal.hpp"
#include "fv_internal.hpp"

using fvapi::align256;
using fvapi::fail;
using fvapi::hip_fail;

namespace {

struct ELayout {
    size_t packed, act0, act1, z, s1, s2, flags, nfb, redone, fatal, bytes;
};

ELayout layout(const fv_euler_learned_config &c)
{
    ELayout L{};
    const size_t px = (size_t)c.B * c.nx * c.ny;
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off = align256(off + n);
        return o;
    };
    L.packed = take(cnn::euler_packed_layout().bytes);
    L.act0 = take(px * 32 * 2);
    L.act1 = take(px * 32 * 2);
    L.z = take(px * cnn::E_COUT * 4);
    L.s1 = take(px * 4 * 4);
    L.s2 = take(px * 4 * 4);
    L.flags = take((size_t)c.B * 2 * 4);
    L.nfb = take((size_t)c.B * 8);
    L.redone = take((size_t)c.B * 8);
    L.fatal = take((size_t)c.B * 4);
    L.bytes = off;
    return L;
}

fv_status validate(const fv_euler_learned_config *c)
{
    if (!c || c->struct_size != sizeof(fv_euler_learned_config)) return fail(FV_E_INVALID, "config struct_size");
    if (c->B < 1 || c->nx < 16 || c->ny < 4) return fail(FV_E_INVALID, "B %d, grid %d x %d", c->B, c->nx, c->ny);
    if (c->nx % 16) return fail(FV_E_INVALID, "nx %d is not a multiple of 16", c->nx);
    if ((double)c->B * c->nx * c->ny * cnn::E_COUT > 2147483647.0)
        return fail(FV_E_INVALID, "B * nx * ny too large");
    if (c->flux != FV_FLUX_HLLE && c->flux != FV_FLUX_RUSANOV) return fail(FV_E_INVALID, "flux %d", c->flux);
    if (c->order < 0 || c->order > 1) return fail(FV_E_INVALID, "constraint order %d", c->order);
    if (!(c->lx > 0.0) || !(c->ly > 0.0) || !(c->gamma > 1.0) || !(c->dt > 0.0))
        return fail(FV_E_INVALID, "lx, ly, dt must be > 0 and gamma > 1");
    for (int v = 0; v < 4; v++)
        if (!std::isfinite(c->mean[v]) || !std::isfinite(c->inv_std[v]))
            return fail(FV_E_INVALID, "normalisation of variable %d", v);
    return FV_OK;
}

}  // namespace

struct fv_euler_learned {
    fv_euler_learned_config cfg;
    const float *params;
    char *ws;
    ELayout L;
    hipStream_t stream;
    cnn::ENorm nrm;
    cnn::Proj pr;
    long long steps_enq = 0;  // steps enqueued: their parity picks the flag slot
};

extern "C" {

size_t fv_euler_net_param_count(void) { return (size_t)cnn::E_NPARAM; }

size_t fv_euler_learned_workspace_bytes(const fv_euler_learned_config *cfg)
{
    if (validate(cfg) != FV_OK) return 0;
    return layout(*cfg).bytes;
}

fv_status fv_euler_learned_create(const fv_euler_learned_config *cfg, const float *params, void *workspace,
                                  size_t workspace_bytes, void *stream, fv_euler_learned **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    fv_status rc = validate(cfg);
    if (rc != FV_OK) return rc;
    if (!params || !workspace) return fail(FV_E_INVALID, "params or workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(FV_E_INVALID, "workspace must be 256-byte aligned");
    const ELayout L = layout(*cfg);
    if (workspace_bytes < L.bytes) return fail(FV_E_NOMEM, "workspace %zu < %zu", workspace_bytes, L.bytes);
    fv_euler_learned *e = new fv_euler_learned();
    e->cfg = *cfg;
    e->params = params;
    e->ws = (char *)workspace;
    e->L = L;
    e->stream = (hipStream_t)stream;
    for (int v = 0; v < 4; v++) {
        e->nrm.mean[v] = cfg->mean[v];
        e->nrm.inv_std[v] = cfg->inv_std[v];
    }
    e->pr = cnn::make_projection(cfg->order);
    hipError_t h = cnn::launch_pack_euler(params, e->ws + L.packed, e->stream);
    if (h == hipSuccess) h = hipMemsetAsync(e->ws + L.flags, 0, L.bytes - L.flags, e->stream);
    if (h != hipSuccess) {
        delete e;
        return hip_fail(h, "Euler network pack / counter reset");
    }
    *out = e;
    return FV_OK;
}

fv_status fv_euler_learned_update(fv_euler_learned *e)
{
    if (!e) return fail(FV_E_INVALID, "handle is NULL");
    hipError_t h = cnn::launch_pack_euler(e->params, e->ws + e->L.packed, e->stream);
    return h == hipSuccess ? FV_OK : hip_fail(h, "Euler network pack");
}

fv_status fv_euler_learned_forward(fv_euler_learned *e, const float *q, float *z)
{
    if (!e || !q || !z) return fail(FV_E_INVALID, "NULL argument");
    const fv_euler_learned_config &c = e->cfg;
    hipError_t h = cnn::launch_forward_euler(e->ws + e->L.packed, e->nrm, q, c.B, c.nx, c.ny, e->ws + e->L.act0,
                                             e->ws + e->L.act1, z, e->stream);
    return h == hipSuccess ? FV_OK : hip_fail(h, "Euler network pass");
}

fv_status fv_euler_learned_forward_tiled(fv_euler_learned *e, const float *q, float *z)
{
    if (!e || !q || !z) return fail(FV_E_INVALID, "NULL argument");
    const fv_euler_learned_config &c = e->cfg;
    if (c.nx % 8 || c.ny % 8) return fail(FV_E_UNSUPPORTED, "the tiled pass needs nx and ny multiples of 8");
    hipError_t h = cnn::launch_forward_euler_fused(e->ws + e->L.packed, e->nrm, q, c.B, c.nx, c.ny, z, e->stream);
    return h == hipSuccess ? FV_OK : hip_fail(h, "Euler network pass");
}

fv_status fv_euler_learned_step(fv_euler_learned *e, float *q, int64_t nsteps)
{
    if (!e || !q) return fail(FV_E_INVALID, "NULL argument");
    if (nsteps < 0) return fail(FV_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    const fv_euler_learned_config &c = e->cfg;
    char *ws = e->ws;
    const ELayout &L = e->L;
    float *z = (float *)(ws + L.z), *S1 = (float *)(ws + L.s1), *S2 = (float *)(ws + L.s2);
    const int fl = c.flux;  // FV_FLUX_HLLE / FV_FLUX_RUSANOV are the kernels' flux ids
    eln::StageArgs a{};
    a.B = c.B;
    a.nx = c.nx;
    a.ny = c.ny;
    a.rdx = (float)(c.nx / c.lx);
    a.rdy = (float)(c.ny / c.ly);
    a.gamma = (float)c.gamma;
    a.dt = (float)c.dt;
    a.flags = (int *)(ws + L.flags);
    a.nfb = (unsigned long long *)(ws + L.nfb);
    a.redone = (unsigned long long *)(ws + L.redone);
    a.fatal = (int *)(ws + L.fatal);
    a.pr = e->pr;
    a.z = z;
    hipError_t h = hipSuccess;
    // the network pass in one launch where the grid is whole 8 x 8 tiles
    const bool tiled = c.nx % 8 == 0 && c.ny % 8 == 0;
    auto net = [&](const float *in) {
        return tiled ? cnn::launch_forward_euler_fused(ws + L.packed, e->nrm, in, c.B, c.nx, c.ny, z, e->stream)
                     : cnn::launch_forward_euler(ws + L.packed, e->nrm, in, c.B, c.nx, c.ny, ws + L.act0, ws + L.act1,
                                                 z, e->stream);
    };
    // network pass and learned stage in one launch per stage where the grid
    // is whole 8 x 8 tiles and every tile gets a workgroup of its own (with
    // more tiles a workgroup would run several tiles' network passes and face
    // epilogues in turn: the separate launches spread the stage wider), else
    // the network pass and the stage kernel, then commit-or-redo and redo
    const bool fused = tiled && (int64_t)c.B * (c.nx / 8) * (c.ny / 8) <= cnn::fused_euler_grid();
    auto learned = [&]() {
        hipError_t r = net(a.qs);
        return r == hipSuccess ? eln::stage(0, fl, a, e->stream) : r;
    };
    if (fused) {
        // two launches per step: the step's output goes to the other buffer
        // of the pair (q, S2), its input stays for a redo, which the next
        // step's first launch carries out where a solve's step was flagged;
        // the call's last step ends with the commit-or-redo and redo launches
        float *X[2] = {q, S2};
        for (int64_t k = 0; k < nsteps && h == hipSuccess; k++, e->steps_enq++) {
            a.parity = (int)(e->steps_enq & 1);
            a.qs = X[k & 1]; a.q0 = X[k & 1]; a.out = S1; a.a0 = 0.f; a.a1 = 1.f; a.flagbit = 1;
            h = cnn::launch_learned_euler(fl, ws + L.packed, e->nrm, a, e->stream, k > 0 ? X[(k + 1) & 1] : nullptr);
            a.qs = S1; a.q0 = X[k & 1]; a.out = X[(k + 1) & 1]; a.a0 = 0.5f; a.a1 = 0.5f; a.flagbit = 2;
            if (h == hipSuccess) h = cnn::launch_learned_euler(fl, ws + L.packed, e->nrm, a, e->stream);
        }
        if (nsteps > 0 && h == hipSuccess) {
            // the last step's input xin and output xout: with an odd step
            // count (q, S2), commit S2 -> q or redo from q; with an even one
            // (S2, q), the result is in q already, or the step is redone from S2
            float *xin = X[(nsteps - 1) & 1], *xout = X[nsteps & 1];
            a.parity = (int)((e->steps_enq - 1) & 1);
            a.qs = xin; a.q0 = xin; a.out = S1; a.a0 = 0.f; a.a1 = 1.f;
            a.commit_src = xout == q ? nullptr : xout;
            a.commit_dst = q;
            h = eln::stage(2, fl, a, e->stream);
            a.qs = S1; a.q0 = xin; a.out = q; a.a0 = 0.5f; a.a1 = 0.5f;
            if (h == hipSuccess) h = eln::stage(3, fl, a, e->stream);
        }
        return h == hipSuccess ? FV_OK : hip_fail(h, "learned Euler step launch");
    }
    for (int64_t k = 0; k < nsteps && h == hipSuccess; k++) {
        a.parity = (int)(e->steps_enq & 1);
        // stage 1: S1 = q + dt L(q)
        a.qs = q; a.q0 = q; a.out = S1; a.a0 = 0.f; a.a1 = 1.f; a.flagbit = 1;
        h = learned();
        // stage 2: S2 = q/2 + (S1 + dt L(S1))/2
        a.qs = S1; a.q0 = q; a.out = S2; a.a0 = 0.5f; a.a1 = 0.5f; a.flagbit = 2;
        if (h == hipSuccess) h = learned();
        // admissible solves commit S2; the others redo the step plainly
        a.qs = q; a.q0 = q; a.out = S1; a.a0 = 0.f; a.a1 = 1.f; a.commit_src = S2; a.commit_dst = q;
        if (h == hipSuccess) h = eln::stage(2, fl, a, e->stream);
        a.qs = S1; a.q0 = q; a.out = q; a.a0 = 0.5f; a.a1 = 0.5f;
        if (h == hipSuccess) h = eln::stage(3, fl, a, e->stream);
        e->steps_enq++;
    }
    return h == hipSuccess ? FV_OK : hip_fail(h, "learned Euler step launch");
}

fv_status fv_euler_learned_stats(fv_euler_learned *e, int64_t *fallback_faces, int64_t *redone_steps, int32_t *frozen)
{
    if (!e) return fail(FV_E_INVALID, "handle is NULL");
    const int B = e->cfg.B;
    std::vector<unsigned long long> nfb(B), red(B);
    std::vector<int> fat(B);
    hipError_t h = hipMemcpyAsync(nfb.data(), e->ws + e->L.nfb, (size_t)B * 8, hipMemcpyDeviceToHost, e->stream);
    if (h == hipSuccess)
        h = hipMemcpyAsync(red.data(), e->ws + e->L.redone, (size_t)B * 8, hipMemcpyDeviceToHost, e->stream);
    if (h == hipSuccess)
        h = hipMemcpyAsync(fat.data(), e->ws + e->L.fatal, (size_t)B * 4, hipMemcpyDeviceToHost, e->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(e->stream);
    if (h != hipSuccess) return hip_fail(h, "learned Euler counters");
    bool any = false;
    for (int b = 0; b < B; b++) {
        if (fallback_faces) fallback_faces[b] = (int64_t)nfb[b];
        if (redone_steps) redone_steps[b] = (int64_t)red[b];
        if (frozen) frozen[b] = fat[b];
        any = any || fat[b] != 0;
    }
    return any ? fail(FV_E_INADMISSIBLE, "a solve's plain redo was inadmissible; it is frozen") : FV_OK;
}

void fv_euler_learned_destroy(fv_euler_learned *e) { delete e; }

}  // extern "C"

// ------------------------------------------------------------------ training
namespace {

struct TLayout {
    size_t states, s1, acts, z, plain, s2, flags, nfb, redone, fatal, dz, contrib, G, Gn, gS1, bwd, lossp, loss,
        scale, total;
    size_t st, act, zb;
};

fv_status validate_train(const fv_euler_train_config *c)
{
    if (!c || c->struct_size != sizeof(fv_euler_train_config)) return fail(FV_E_INVALID, "train config struct_size");
    if (c->B < 1 || c->T < 1) return fail(FV_E_INVALID, "B and T must be >= 1");
    if (c->nx < 16 || c->nx % 16 || c->ny < 4) return fail(FV_E_INVALID, "grid %d x %d", c->nx, c->ny);
    if (c->flux != FV_FLUX_HLLE && c->flux != FV_FLUX_RUSANOV) return fail(FV_E_INVALID, "flux %d", c->flux);
    if (!(c->dt > 0) || !(c->lx > 0) || !(c->ly > 0) || !(c->gamma > 1.0))
        return fail(FV_E_INVALID, "dt, lx, ly must be positive and gamma > 1");
    for (int v = 0; v < 4; v++)
        if (!(c->scale[v] > 0)) return fail(FV_E_INVALID, "loss scale must be positive");
    if (!(c->lr > 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) || !(c->eps > 0))
        return fail(FV_E_INVALID, "Adam hyper-parameters");
    return FV_OK;
}

TLayout tlayout(const fv_euler_train_config *c)
{
    TLayout L;
    const size_t npix = (size_t)c->B * c->nx * c->ny;
    const int T = c->T;
    L.st = align256(npix * 4 * 4);
    L.act = align256(npix * 32 * 2);
    L.zb = align256(npix * cnn::E_COUT * 4);
    size_t o = 0;
    auto take = [&](size_t n) {
        const size_t r = o;
        o += align256(n);
        return r;
    };
    L.states = take((T + 1) * L.st);
    L.s1 = take(T * L.st);
    L.acts = take((size_t)T * 2 * 4 * L.act);
    L.z = take((size_t)T * 2 * L.zb);
    L.plain = take((size_t)T * c->B * 4);
    L.s2 = take(L.st);
    L.flags = take((size_t)c->B * 2 * 4);
    L.nfb = take((size_t)c->B * 8);
    L.redone = take((size_t)c->B * 8);
    L.fatal = take((size_t)c->B * 4);
    L.dz = take(npix * cnn::E_COUT * 2);
    L.contrib = take(npix * 2 * eln::ADJ_REC * 4);
    L.G = take(L.st);
    L.Gn = take(L.st);
    L.gS1 = take(L.st);
    L.bwd = take(cnn::backward_scratch_bytes_euler(c->B, c->nx, c->ny));
    L.lossp = take(1024 * 8);
    L.loss = take(8);
    L.scale = take(16);
    L.total = o;
    return L;
}

}  // namespace

struct fv_euler_trainer {
    fv_euler_train_config cfg;
    fv_euler_learned *net;
    float *grads, *am, *av;
    char *ws;
    TLayout L;
    int64_t adam_t = 0;
    int last_T = 0;
    float *st(int t) { return (float *)(ws + L.states + (size_t)t * L.st); }
    float *s1(int t) { return (float *)(ws + L.s1 + (size_t)t * L.st); }
    void *act(int t, int stage, int l) { return ws + L.acts + (((size_t)t * 2 + stage) * 4 + l) * L.act; }
    float *zb(int t, int stage) { return (float *)(ws + L.z + ((size_t)t * 2 + stage) * L.zb); }
    int *plain(int t) { return (int *)(ws + L.plain) + (size_t)t * cfg.B; }
};

extern "C" {

size_t fv_euler_train_workspace_bytes(const fv_euler_train_config *cfg)
{
    if (validate_train(cfg) != FV_OK) return 0;
    return tlayout(cfg).total;
}

fv_status fv_euler_train_create(const fv_euler_train_config *cfg, fv_euler_learned *net, float *grads,
                                float *adam_m, float *adam_v, void *workspace, size_t workspace_bytes,
                                fv_euler_trainer **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    fv_status rc = validate_train(cfg);
    if (rc != FV_OK) return rc;
    if (!net || !grads || !adam_m || !adam_v || !workspace) return fail(FV_E_INVALID, "NULL argument");
    if (((uintptr_t)workspace & 255) != 0) return fail(FV_E_INVALID, "workspace must be 256-byte aligned");
    const TLayout L = tlayout(cfg);
    if (workspace_bytes < L.total) return fail(FV_E_NOMEM, "workspace %zu < %zu", workspace_bytes, L.total);
    fv_euler_trainer *tr = new fv_euler_trainer();
    tr->cfg = *cfg;
    tr->net = net;
    tr->grads = grads;
    tr->am = adam_m;
    tr->av = adam_v;
    tr->ws = (char *)workspace;
    tr->L = L;
    hipError_t e = hipMemcpyAsync(tr->ws + L.scale, cfg->scale, 4 * sizeof(float), hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) {
        delete tr;
        return hip_fail(e, "trainer setup");
    }
    *out = tr;
    return FV_OK;
}

fv_status fv_euler_train_step(fv_euler_trainer *tr, const float *q0, const float *targets, int T, double *loss,
                              fv_learned_stats *stats)
{
    if (!tr || !q0 || !targets || !loss) return fail(FV_E_INVALID, "NULL argument");
    const fv_euler_train_config &c = tr->cfg;
    if (T < 1 || T > c.T) return fail(FV_E_INVALID, "T = %d outside 1..%d", T, c.T);
    fv_euler_learned *net = tr->net;
    hipStream_t st = net->stream;
    const int B = c.B, nx = c.nx, ny = c.ny;
    const size_t nst = (size_t)B * 4 * nx * ny;
    char *ws = tr->ws;
    const TLayout &L = tr->L;
    const char *packed = net->ws + net->L.packed;
    const int fl = c.flux;
    hipError_t e = hipMemcpyAsync(tr->st(0), q0, nst * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.flags, 0, L.dz - L.flags, st);  // flags, counters, frozen

    eln::StageArgs a{};
    a.B = B;
    a.nx = nx;
    a.ny = ny;
    a.rdx = (float)(nx / c.lx);
    a.rdy = (float)(ny / c.ly);
    a.gamma = (float)c.gamma;
    a.dt = (float)c.dt;
    a.flags = (int *)(ws + L.flags);
    a.nfb = (unsigned long long *)(ws + L.nfb);
    a.redone = (unsigned long long *)(ws + L.redone);
    a.fatal = (int *)(ws + L.fatal);
    a.pr = net->pr;
    float *S2 = (float *)(ws + L.s2);

    // ---------------------------------------------------------------- forward
    for (int t = 0; t < T && e == hipSuccess; t++) {
        a.parity = t & 1;
        void *a0[4] = {tr->act(t, 0, 0), tr->act(t, 0, 1), tr->act(t, 0, 2), tr->act(t, 0, 3)};
        void *a1[4] = {tr->act(t, 1, 0), tr->act(t, 1, 1), tr->act(t, 1, 2), tr->act(t, 1, 3)};
        e = cnn::launch_forward_euler_keep(packed, net->nrm, tr->st(t), B, nx, ny, a0, tr->zb(t, 0), st);
        a.qs = tr->st(t); a.q0 = tr->st(t); a.out = tr->s1(t); a.z = tr->zb(t, 0);
        a.a0 = 0.f; a.a1 = 1.f; a.flagbit = 1; a.record = nullptr;
        if (e == hipSuccess) e = eln::stage(0, fl, a, st);
        if (e == hipSuccess)
            e = cnn::launch_forward_euler_keep(packed, net->nrm, tr->s1(t), B, nx, ny, a1, tr->zb(t, 1), st);
        a.qs = tr->s1(t); a.q0 = tr->st(t); a.out = S2; a.z = tr->zb(t, 1);
        a.a0 = 0.5f; a.a1 = 0.5f; a.flagbit = 2;
        if (e == hipSuccess) e = eln::stage(0, fl, a, st);
        // admissible solves commit S2; the others redo the step plainly (its
        // first stage overwrites the saved stage input, so the reverse pass
        // sees the plain step)
        a.qs = tr->st(t); a.q0 = tr->st(t); a.out = tr->s1(t); a.a0 = 0.f; a.a1 = 1.f;
        a.commit_src = S2; a.commit_dst = tr->st(t + 1);
        if (e == hipSuccess) e = eln::stage(2, fl, a, st);
        a.qs = tr->s1(t); a.q0 = tr->st(t); a.out = tr->st(t + 1); a.a0 = 0.5f; a.a1 = 0.5f;
        a.record = tr->plain(t);
        if (e == hipSuccess) e = eln::stage(3, fl, a, st);
        a.record = nullptr;
    }

    // ------------------------------------------------------ loss and reverse
    float *G = (float *)(ws + L.G), *Gn = (float *)(ws + L.Gn), *gS1 = (float *)(ws + L.gS1);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.loss, 0, 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(G, 0, nst * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(tr->grads, 0, (size_t)cnn::E_NPARAM * 4, st);
    eln::AdjArgs ad{};
    ad.B = B;
    ad.nx = nx;
    ad.ny = ny;
    ad.rdx = a.rdx;
    ad.rdy = a.rdy;
    ad.gamma = a.gamma;
    ad.pr = net->pr;
    ad.contrib = (float *)(ws + L.contrib);
    ad.dz = (__bf16 *)(ws + L.dz);
    for (int t = T; t >= 1 && e == hipSuccess; t--) {
        e = cnn::launch_loss(tr->st(t), targets + (size_t)(t - 1) * nst, (const float *)(ws + L.scale), B, nx, ny, G,
                             (double *)(ws + L.lossp), 1024, (double *)(ws + L.loss), st, 4);
        const int k = t - 1;  // step k maps st(k) -> st(k+1)
        void *a0[4] = {tr->act(k, 0, 0), tr->act(k, 0, 1), tr->act(k, 0, 2), tr->act(k, 0, 3)};
        void *a1[4] = {tr->act(k, 1, 0), tr->act(k, 1, 1), tr->act(k, 1, 2), tr->act(k, 1, 3)};
        ad.plain = tr->plain(k);
        // stage 2: out = q/2 + (S1 + dt L(S1))/2
        ad.qs = tr->s1(k); ad.z = tr->zb(k, 1); ad.gout = G; ad.wscale = 0.5f * (float)c.dt;
        if (e == hipSuccess) e = eln::adjoint(fl, ad, gS1, 0.5f, 0, st);
        if (e == hipSuccess)
            e = cnn::launch_backward_euler(packed, net->nrm, tr->s1(k), B, nx, ny, a1, ad.dz, gS1, tr->grads,
                                           ws + L.bwd, st);
        // stage 1: S1 = q + dt L(q), after the q/2 term of stage 2
        if (e == hipSuccess) e = cnn::launch_scale(Gn, G, 0.5f, nst, st);
        ad.qs = tr->st(k); ad.z = tr->zb(k, 0); ad.gout = gS1; ad.wscale = (float)c.dt;
        if (e == hipSuccess) e = eln::adjoint(fl, ad, Gn, 1.0f, 1, st);
        if (e == hipSuccess)
            e = cnn::launch_backward_euler(packed, net->nrm, tr->st(k), B, nx, ny, a0, ad.dz, Gn, tr->grads,
                                           ws + L.bwd, st);
        float *tmp = G;
        G = Gn;
        Gn = tmp;
    }
    if (e != hipSuccess) return hip_fail(e, "training step launch");
    if (G != (float *)(ws + L.G)) {
        e = hipMemcpyAsync(ws + L.G, G, nst * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "copy input gradient");
    }
    tr->last_T = T;
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(loss, ws + L.loss, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read loss");
    if (stats) {
        std::vector<unsigned long long> nfb(B), red(B);
        e = hipMemcpy(nfb.data(), ws + L.nfb, (size_t)B * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(red.data(), ws + L.redone, (size_t)B * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read counters");
        stats->fallback_faces = stats->redone_steps = 0;
        for (int b = 0; b < B; b++) {
            stats->fallback_faces += (int64_t)nfb[b];
            stats->redone_steps += (int64_t)red[b];
        }
    }
    return FV_OK;
}

fv_status fv_euler_train_input_grad(fv_euler_trainer *tr, float *dst)
{
    if (!tr || !dst) return fail(FV_E_INVALID, "NULL argument");
    const size_t n = (size_t)tr->cfg.B * 4 * tr->cfg.nx * tr->cfg.ny * 4;
    hipError_t e = hipMemcpyAsync(dst, tr->ws + tr->L.G, n, hipMemcpyDeviceToDevice, tr->net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->net->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "copy input gradient");
}

fv_status fv_euler_adam_step(fv_euler_trainer *tr)
{
    if (!tr) return fail(FV_E_INVALID, "trainer is NULL");
    const fv_euler_train_config &c = tr->cfg;
    tr->adam_t++;
    const float bc1 = 1.0f - (float)std::pow((double)c.beta1, (double)tr->adam_t);
    const float bc2 = 1.0f - (float)std::pow((double)c.beta2, (double)tr->adam_t);
    fv_euler_learned *net = tr->net;
    hipError_t e = cnn::launch_adam((float *)net->params, tr->grads, tr->am, tr->av, cnn::E_NPARAM, c.lr, c.beta1,
                                    c.beta2, c.eps, bc1, bc2, net->stream);
    if (e == hipSuccess) e = cnn::launch_pack_euler(net->params, net->ws + net->L.packed, net->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "adam step");
}

fv_status fv_euler_train_set_lr(fv_euler_trainer *tr, float lr)
{
    if (!tr) return fail(FV_E_INVALID, "trainer is NULL");
    if (!(lr > 0.0f)) return fail(FV_E_INVALID, "learning rate %g <= 0", (double)lr);
    tr->cfg.lr = lr;
    return FV_OK;
}

void fv_euler_train_destroy(fv_euler_trainer *tr)
{
    if (!tr) return;
    (void)hipStreamSynchronize(tr->net->stream);
    delete tr;
}

}  // extern "C"
