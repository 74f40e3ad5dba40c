// C-ABI host side of training: unrolled learned rollout with saved stages,
// the loss of eq 2.28, the reverse pass and Adam.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "api_common.hpp"

using fvapi::align256;
using fvapi::fail;
using fvapi::hip_fail;

namespace {

struct TrainLayout {
    size_t states, s1, acts, z, plain, s2, bad, dt, nfb, redone, fatal, dz, contrib, G, Gn, gS1, bwd, lossp, loss,
        scale, total;
    size_t st, act, zb;  // per-unit sizes
};

fv_status validate(const fv_train_config *c)
{
    if (!c || c->struct_size != sizeof(fv_train_config)) return fail(FV_E_INVALID, "train config struct_size");
    if (c->B < 1 || c->T < 1) return fail(FV_E_INVALID, "B and T must be >= 1");
    if (c->nx < 16 || c->ny < 4 || c->nx % 16 || ((int64_t)c->nx * c->ny) % 64)
        return fail(FV_E_UNSUPPORTED, "training grids need nx %% 16 == 0 and nx*ny %% 64 == 0");
    if (c->flux != FV_FLUX_HLLE && c->flux != FV_FLUX_RUSANOV) return fail(FV_E_UNSUPPORTED, "flux %d", c->flux);
    if (!(c->dt > 0) || !(c->lx > 0) || !(c->ly > 0) || !(c->g > 0) || !(c->h_ref > 0))
        return fail(FV_E_INVALID, "dt, lx, ly, g and h_ref must be positive");
    for (int v = 0; v < 3; v++)
        if (!(c->scale[v] > 0)) return fail(FV_E_INVALID, "loss scale must be positive");
    if (!(c->lr > 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) || !(c->eps > 0))
        return fail(FV_E_INVALID, "Adam hyper-parameters");
    if ((c->direct != 0 && c->direct != 1) || (c->blend != 0 && c->blend != 1) || (c->direct && c->blend))
        return fail(FV_E_INVALID, "direct and blend must be 0 or 1, not both 1");
    return FV_OK;
}

TrainLayout layout_of(const fv_train_config *c)
{
    TrainLayout L;
    const size_t npix = (size_t)c->B * c->nx * c->ny;
    const int T = c->T;
    L.st = align256(npix * 3 * 4);
    L.act = align256(npix * 32 * 2);
    L.zb = align256(npix * 72 * 4);
    size_t o = 0;
    L.states = o;
    o += (T + 1) * L.st;
    L.s1 = o;
    o += T * L.st;
    L.acts = o;
    o += (size_t)T * 2 * 4 * L.act;
    L.z = o;
    o += (size_t)T * 2 * L.zb;
    L.plain = o;
    o += align256((size_t)T * c->B * 4);
    L.s2 = o;
    o += L.st;
    L.bad = o;
    o += align256(c->B * 4);
    L.dt = o;
    o += align256(c->B * 4);
    L.nfb = o;
    o += align256(c->B * 8);
    L.redone = o;
    o += align256(c->B * 8);
    L.fatal = o;
    o += align256(c->B * 4);
    L.dz = o;
    o += align256(npix * cnn::DZ_CH * 2);
    L.contrib = o;
    o += align256(npix * 2 * cnn::ADJ_REC * 4);
    L.G = o;
    o += L.st;
    L.Gn = o;
    o += L.st;
    L.gS1 = o;
    o += L.st;
    L.bwd = o;
    o += align256(cnn::backward_scratch_bytes(c->B, c->nx, c->ny));
    L.lossp = o;
    o += align256(1024 * 8);
    L.loss = o;
    o += 256;
    L.scale = o;
    o += 256;
    L.total = o;
    return L;
}

}  // namespace

struct fv_trainer {
    fv_train_config cfg;
    fv_model *m;
    float *grads, *am, *av;
    char *ws;
    TrainLayout L;
    int64_t adam_t;
    int last_T;
    float *st(int t) { return (float *)(ws + L.states + (size_t)t * L.st); }
    float *s1(int t) { return (float *)(ws + L.s1 + (size_t)t * L.st); }
    void *act(int t, int stage, int l) { return ws + L.acts + (((size_t)t * 2 + stage) * 4 + l) * L.act; }
    float *zb(int t, int stage) { return (float *)(ws + L.z + ((size_t)t * 2 + stage) * L.zb); }
    int *plain(int t) { return (int *)(ws + L.plain) + (size_t)t * cfg.B; }
};

extern "C" {

size_t fv_train_workspace_bytes(const fv_train_config *cfg)
{
    if (validate(cfg) != FV_OK) return 0;
    return layout_of(cfg).total;
}

fv_status fv_train_create(const fv_train_config *cfg, fv_model *m, float *grads, float *adam_m, float *adam_v,
                          void *workspace, size_t workspace_bytes, fv_trainer **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    fv_status rc = validate(cfg);
    if (rc != FV_OK) return rc;
    if (!m || !grads || !adam_m || !adam_v || !workspace) return fail(FV_E_INVALID, "NULL argument");
    if (((uintptr_t)workspace & 255) != 0) return fail(FV_E_INVALID, "workspace must be 256-byte aligned");
    TrainLayout L = layout_of(cfg);
    if (workspace_bytes < L.total) return fail(FV_E_NOMEM, "workspace %zu < %zu", workspace_bytes, L.total);
    fv_trainer *tr = new fv_trainer();
    tr->cfg = *cfg;
    tr->m = m;
    tr->grads = grads;
    tr->am = adam_m;
    tr->av = adam_v;
    tr->ws = (char *)workspace;
    tr->L = L;
    tr->adam_t = 0;
    tr->last_T = 0;
    std::vector<float> dts(cfg->B, (float)cfg->dt);
    hipError_t e = hipMemcpyAsync(tr->ws + L.dt, dts.data(), dts.size() * 4, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tr->ws + L.scale, cfg->scale, 3 * sizeof(float), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(tr->ws + L.bad, 0, align256(cfg->B * 4), m->stream);
    // dz's padding channels (72 .. DZ_CH-1) stay zero: the adjoint writes 0 .. 71
    if (e == hipSuccess) e = hipMemsetAsync(tr->ws + L.dz, 0, L.contrib - L.dz, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        delete tr;
        return hip_fail(e, "trainer setup");
    }
    *out = tr;
    return FV_OK;
}

fv_status fv_train_step(fv_trainer *tr, const float *q0, const float *targets, int T, double *loss,
                        fv_learned_stats *stats)
{
    if (!tr || !q0 || !targets || !loss) return fail(FV_E_INVALID, "NULL argument");
    const fv_train_config &c = tr->cfg;
    if (T < 1 || T > c.T) return fail(FV_E_INVALID, "T = %d outside 1..%d", T, c.T);
    hipStream_t st = tr->m->stream;
    const int B = c.B, nx = c.nx, ny = c.ny;
    const size_t nst = (size_t)B * 3 * nx * ny;
    char *ws = tr->ws;
    const TrainLayout &L = tr->L;
    const int fl = c.flux == FV_FLUX_RUSANOV ? 1 : 0;
    hipError_t e = hipMemcpyAsync(tr->st(0), q0, nst * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.nfb, 0, align256(B * 8) * 2, st);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.fatal, 0, align256(B * 4), st);

    cnn::StageBatch sb{};
    sb.B = B;
    sb.nx = nx;
    sb.ny = ny;
    sb.rdx = (float)(nx / c.lx);
    sb.rdy = (float)(ny / c.ly);
    sb.g = (float)c.g;
    sb.h0 = (float)c.h_ref;
    sb.dt = (const float *)(ws + L.dt);
    sb.bad = (int *)(ws + L.bad);
    sb.nfb = (unsigned long long *)(ws + L.nfb);
    sb.fatal = (int *)(ws + L.fatal);
    sb.pr = tr->m->pr;
    for (int v = 0; v < 3; v++) sb.sig[v] = 1.0f / tr->m->nrm.inv_std[v];
    float *S2 = (float *)(ws + L.s2);

    // ---------------------------------------------------------------- forward
    for (int t = 0; t < T && e == hipSuccess; t++) {
        void *a0[4] = {tr->act(t, 0, 0), tr->act(t, 0, 1), tr->act(t, 0, 2), tr->act(t, 0, 3)};
        void *a1[4] = {tr->act(t, 1, 0), tr->act(t, 1, 1), tr->act(t, 1, 2), tr->act(t, 1, 3)};
        e = cnn::launch_forward(tr->m->packed, tr->m->nrm, tr->st(t), B, nx, ny, a0, tr->zb(t, 0), st);
        sb.qs = tr->st(t); sb.q0 = tr->st(t); sb.out = tr->s1(t); sb.z = tr->zb(t, 0);
        sb.a0 = 0.f; sb.a1 = 1.f; sb.flagbit = 1; sb.direct = c.direct; sb.blend = c.blend;
        if (e == hipSuccess) e = cnn::learned_stage(0, fl, sb, st);
        if (e == hipSuccess) e = cnn::launch_forward(tr->m->packed, tr->m->nrm, tr->s1(t), B, nx, ny, a1, tr->zb(t, 1), st);
        sb.qs = tr->s1(t); sb.q0 = tr->st(t); sb.out = S2; sb.z = tr->zb(t, 1);
        sb.a0 = 0.5f; sb.a1 = 0.5f; sb.flagbit = 2;
        if (e == hipSuccess) e = cnn::learned_stage(0, fl, sb, st);
        if (e == hipSuccess) e = cnn::launch_commit(tr->st(t + 1), S2, sb.bad, (size_t)3 * nx * ny, B, st);
        // solves whose learned step was inadmissible: plain step, which also
        // overwrites the saved stage input so the reverse pass sees it
        sb.direct = 0;
        sb.blend = 0;
        sb.qs = tr->st(t); sb.q0 = tr->st(t); sb.out = tr->s1(t); sb.a0 = 0.f; sb.a1 = 1.f;
        if (e == hipSuccess) e = cnn::learned_stage(1, fl, sb, st);
        sb.qs = tr->s1(t); sb.q0 = tr->st(t); sb.out = tr->st(t + 1); sb.a0 = 0.5f; sb.a1 = 0.5f;
        if (e == hipSuccess) e = cnn::learned_stage(1, fl, sb, st);
        if (e == hipSuccess)
            e = cnn::launch_finish(sb.bad, (unsigned long long *)(ws + L.redone), tr->plain(t), B, sb.dt, nullptr,
                                   nullptr, st);
    }

    // ------------------------------------------------------ loss and reverse
    float *G = (float *)(ws + L.G), *Gn = (float *)(ws + L.Gn), *gS1 = (float *)(ws + L.gS1);
    if (e == hipSuccess) e = hipMemsetAsync(ws + L.loss, 0, 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(G, 0, nst * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(tr->grads, 0, (size_t)cnn::NPARAM * 4, st);
    cnn::AdjStage as;
    as.direct = c.direct;
    as.blend = c.blend;
    for (int v = 0; v < 3; v++) as.sig[v] = 1.0f / tr->m->nrm.inv_std[v];
    as.dt = (float)c.dt;
    as.B = B;
    as.nx = nx;
    as.ny = ny;
    as.rdx = sb.rdx;
    as.rdy = sb.rdy;
    as.g = sb.g;
    as.h0 = sb.h0;
    as.pr = tr->m->pr;
    as.contrib = (float *)(ws + L.contrib);
    as.dz = ws + L.dz;
    for (int t = T; t >= 1 && e == hipSuccess; t--) {
        e = cnn::launch_loss(tr->st(t), targets + (size_t)(t - 1) * nst, (const float *)(ws + L.scale), B, nx, ny, G,
                             (double *)(ws + L.lossp), 1024, (double *)(ws + L.loss), st);
        const int k = t - 1;  // step k maps st(k) -> st(k+1)
        void *a0[4] = {tr->act(k, 0, 0), tr->act(k, 0, 1), tr->act(k, 0, 2), tr->act(k, 0, 3)};
        void *a1[4] = {tr->act(k, 1, 0), tr->act(k, 1, 1), tr->act(k, 1, 2), tr->act(k, 1, 3)};
        // stage 2: out = q/2 + (S1 + dt L(S1))/2
        as.qs = tr->s1(k); as.z = tr->zb(k, 1); as.gout = G; as.a1 = 0.5f; as.plain = tr->plain(k);
        as.gqs = gS1; as.accumulate = 0;
        if (e == hipSuccess) e = cnn::launch_adjoint(fl, as, st);
        if (e == hipSuccess)
            e = cnn::launch_backward(tr->m->packed, tr->m->nrm, tr->s1(k), B, nx, ny, a1, as.dz, gS1, tr->grads,
                                     ws + L.bwd, st);
        // stage 1: S1 = q + dt L(q); the q/2 term of stage 2 first
        if (e == hipSuccess) e = cnn::launch_scale(Gn, G, 0.5f, nst, st);
        as.qs = tr->st(k); as.z = tr->zb(k, 0); as.gout = gS1; as.a1 = 1.0f; as.gqs = Gn; as.accumulate = 1;
        if (e == hipSuccess) e = cnn::launch_adjoint(fl, as, st);
        if (e == hipSuccess)
            e = cnn::launch_backward(tr->m->packed, tr->m->nrm, tr->st(k), B, nx, ny, a0, as.dz, Gn, tr->grads,
                                     ws + L.bwd, st);
        float *tmp = G;
        G = Gn;
        Gn = tmp;
    }
    if (e != hipSuccess) return hip_fail(e, "training step launch");
    // keep d loss / d q0 in the L.G slot
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
        e = hipMemcpy(nfb.data(), ws + L.nfb, B * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(red.data(), ws + L.redone, B * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read counters");
        stats->fallback_faces = stats->redone_steps = 0;
        for (int b = 0; b < B; b++) {
            stats->fallback_faces += (int64_t)nfb[b];
            stats->redone_steps += (int64_t)red[b];
        }
    }
    return FV_OK;
}

fv_status fv_train_input_grad(fv_trainer *tr, float *dst)
{
    if (!tr || !dst) return fail(FV_E_INVALID, "NULL argument");
    size_t n = (size_t)tr->cfg.B * 3 * tr->cfg.nx * tr->cfg.ny * 4;
    hipError_t e = hipMemcpyAsync(dst, tr->ws + tr->L.G, n, hipMemcpyDeviceToDevice, tr->m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->m->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "copy input gradient");
}

fv_status fv_train_state(fv_trainer *tr, int t, float *dst)
{
    if (!tr || !dst) return fail(FV_E_INVALID, "NULL argument");
    if (t < 0 || t > tr->last_T) return fail(FV_E_INVALID, "t = %d outside 0..%d", t, tr->last_T);
    size_t n = (size_t)tr->cfg.B * 3 * tr->cfg.nx * tr->cfg.ny * 4;
    hipError_t e = hipMemcpyAsync(dst, tr->st(t), n, hipMemcpyDeviceToDevice, tr->m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->m->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "copy state");
}

fv_status fv_adam_step(fv_trainer *tr)
{
    if (!tr) return fail(FV_E_INVALID, "trainer is NULL");
    const fv_train_config &c = tr->cfg;
    tr->adam_t++;
    float bc1 = 1.0f - (float)__builtin_pow(c.beta1, (double)tr->adam_t);
    float bc2 = 1.0f - (float)__builtin_pow(c.beta2, (double)tr->adam_t);
    hipError_t e = cnn::launch_adam((float *)tr->m->params, tr->grads, tr->am, tr->av, cnn::NPARAM, c.lr, c.beta1,
                                    c.beta2, c.eps, bc1, bc2, tr->m->stream);
    if (e == hipSuccess) e = cnn::launch_pack(tr->m->params, tr->m->packed, tr->m->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "adam step");
}

fv_status fv_train_set_lr(fv_trainer *tr, float lr)
{
    if (!tr) return fail(FV_E_INVALID, "trainer is NULL");
    if (!(lr > 0.0f)) return fail(FV_E_INVALID, "learning rate %g <= 0", (double)lr);
    tr->cfg.lr = lr;
    return FV_OK;
}

void fv_train_destroy(fv_trainer *tr)
{
    if (!tr) return;
    (void)hipStreamSynchronize(tr->m->stream);
    delete tr;
}

fv_status fv_coarsen(const float *fine, int nvar, int nx, int ny, int factor, float *coarse, void *stream)
{
    if (!fine || !coarse) return fail(FV_E_INVALID, "NULL argument");
    if (nvar < 1 || factor < 1 || nx % factor || ny % factor)
        return fail(FV_E_INVALID, "grid %dx%d not divisible by %d", nx, ny, factor);
    hipError_t e = cnn::launch_coarsen(fine, nvar, nx, ny, factor, coarse, (hipStream_t)stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "coarsen launch");
}

}  // extern "C"
