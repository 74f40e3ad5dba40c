// C-ABI host side of the spherical shallow-water path (thesis sections 2.4,
// 3.3): configuration checks, workspace layout and step sequencing.  Delta t
// stays on the device with the planar path's three rotating rate slots.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "api_common.hpp"
#include "sphere_internal.hpp"

using fvapi::align256;
using fvapi::fail;
using fvapi::hip_fail;

namespace {

struct SphLayout {
    size_t ctl, rates, totals_out, partials;
    size_t cen, nsum, inv_area, rate_fac, area, xf, yf;
    size_t s1, s2;
    size_t total;
};

size_t es_of(const fv_sphere_config *c) { return c->prec == FV_F64 ? 8 : 4; }

SphLayout sph_layout(const fv_sphere_config *c)
{
    SphLayout L;
    const size_t es = es_of(c), P = (size_t)2 * c->n * c->n, PY = P + (size_t)2 * c->n;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.ctl = take(fvk::CTL_BYTES);
    L.rates = take(fvk::RATE_BYTES);
    L.totals_out = take(256);
    L.partials = take((size_t)fvk::TOTALS_MAX_BLOCKS * 2 * sizeof(double));
    L.cen = take(3 * P * es);
    L.nsum = take(3 * P * es);
    L.inv_area = take(P * es);
    L.rate_fac = take(P * es);
    L.area = take(P * sizeof(double));
    L.xf = take(10 * P * es);
    L.yf = take(10 * PY * es);
    L.s1 = take(4 * P * es);
    L.s2 = take(c->rk_stages == 3 ? 4 * P * es : 0);
    L.total = o;
    return L;
}

fv_status sph_validate(const fv_sphere_config *c)
{
    if (!c) return fail(FV_E_INVALID, "config is NULL");
    if (c->struct_size != sizeof(fv_sphere_config))
        return fail(FV_E_INVALID, "struct_size %u != sizeof(fv_sphere_config) %zu", c->struct_size,
                    sizeof(fv_sphere_config));
    if (c->prec != FV_F32 && c->prec != FV_F64) return fail(FV_E_INVALID, "prec %d", c->prec);
    if (c->n < 4 || c->n > 8192) return fail(FV_E_INVALID, "n = %d outside 4..8192", c->n);
    if (c->flux < FV_FLUX_HLLE || c->flux > FV_FLUX_ROE) return fail(FV_E_INVALID, "flux %d", c->flux);
    if (c->recon != FV_RECON_MINMOD && c->recon != FV_RECON_FIRST) return fail(FV_E_INVALID, "recon %d", c->recon);
    if (c->rk_stages < 1 || c->rk_stages > 3) return fail(FV_E_INVALID, "rk_stages %d", c->rk_stages);
    if (!(c->dt_fixed > 0) && !(c->cfl > 0 && c->cfl <= 1)) return fail(FV_E_INVALID, "cfl %g not in (0,1]", c->cfl);
    if (!(c->g > 0)) return fail(FV_E_INVALID, "g %g", c->g);
    if (!std::isfinite(c->omega)) return fail(FV_E_INVALID, "omega %g", c->omega);
    if (c->reserved0 != 0) return fail(FV_E_INVALID, "reserved0 must be 0");
    return FV_OK;
}

template <typename T> sph::Geometry<T> geometry_of(char *ws, const SphLayout &L)
{
    sph::Geometry<T> G;
    G.cen = (T *)(ws + L.cen);
    G.nsum = (T *)(ws + L.nsum);
    G.inv_area = (T *)(ws + L.inv_area);
    G.rate_fac = (T *)(ws + L.rate_fac);
    G.area = (double *)(ws + L.area);
    G.xf = (T *)(ws + L.xf);
    G.yf = (T *)(ws + L.yf);
    return G;
}

}  // namespace

struct fv_sphere {
    fv_sphere_config cfg;
    void *q;
    char *ws;
    SphLayout L;
    hipStream_t stream;
    int64_t enq;
    fvk::Ctl *ctl() { return (fvk::Ctl *)(ws + L.ctl); }
    unsigned long long *rates() { return (unsigned long long *)(ws + L.rates); }
};

namespace {

template <typename T> hipError_t stage(fv_sphere *s, const T *qs, T *out, double a0, double a1, int last, int ri,
                                       int ro, int rc)
{
    const fv_sphere_config &c = s->cfg;
    sph::CellArgs<T> a;
    a.qs = qs;
    a.q0 = (const T *)s->q;
    a.out = out;
    a.G = geometry_of<T>(s->ws, s->L);
    a.n = c.n;
    a.g = (T)c.g;
    a.omega = (T)c.omega;
    a.a0 = (T)a0;
    a.a1 = (T)a1;
    a.cfl = c.cfl;
    a.dt_fixed = c.dt_fixed;
    a.ctl = s->ctl();
    a.rates = s->rates();
    a.rate_in = ri;
    a.rate_out = ro;
    a.rate_clear = rc;
    a.last = last;
    return sph::stage<T>(c.flux, c.recon, a, s->stream);
}

template <typename T> hipError_t step(fv_sphere *s)
{
    const int n = (int)(s->enq % 3);
    const bool cfl = !(s->cfg.dt_fixed > 0);
    const int ri = n, ro = cfl ? (n + 1) % 3 : -1, rc = cfl ? (n + 2) % 3 : -1;
    T *q = (T *)s->q, *S1 = (T *)(s->ws + s->L.s1), *S2 = (T *)(s->ws + s->L.s2);
    hipError_t e;
    switch (s->cfg.rk_stages) {
    case 1:
        e = stage<T>(s, q, q, 0.0, 1.0, 1, ri, ro, rc);
        break;
    case 2:
        e = stage<T>(s, q, S1, 0.0, 1.0, 0, ri, -1, -1);
        if (e == hipSuccess) e = stage<T>(s, S1, q, 0.5, 0.5, 1, ri, ro, rc);
        break;
    default:
        e = stage<T>(s, q, S1, 0.0, 1.0, 0, ri, -1, -1);
        if (e == hipSuccess) e = stage<T>(s, S1, S2, 0.75, 0.25, 0, ri, -1, -1);
        if (e == hipSuccess) e = stage<T>(s, S2, q, 1.0 / 3.0, 2.0 / 3.0, 1, ri, ro, rc);
        break;
    }
    if (e == hipSuccess) s->enq++;
    return e;
}

}  // namespace

extern "C" {

size_t fv_sphere_workspace_bytes(const fv_sphere_config *cfg)
{
    if (sph_validate(cfg) != FV_OK) return 0;
    return sph_layout(cfg).total;
}

fv_status fv_sphere_init(const fv_sphere_config *cfg, void *q, void *workspace, size_t workspace_bytes, void *stream,
                         fv_sphere **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    fv_status rc = sph_validate(cfg);
    if (rc != FV_OK) return rc;
    if (!q || !workspace) return fail(FV_E_INVALID, "state or workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(FV_E_INVALID, "workspace must be 256-byte aligned");
    const SphLayout L = sph_layout(cfg);
    if (workspace_bytes < L.total) return fail(FV_E_NOMEM, "workspace %zu bytes < required %zu", workspace_bytes, L.total);
    fv_sphere *s = new fv_sphere();
    s->cfg = *cfg;
    s->q = q;
    s->ws = (char *)workspace;
    s->L = L;
    s->stream = (hipStream_t)stream;
    s->enq = 0;
    fvk::Ctl fresh;
    std::memset(&fresh, 0, sizeof fresh);
    hipError_t e = hipMemcpyAsync(s->ctl(), &fresh, sizeof fresh, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->rates(), 0, fvk::RATE_BYTES, s->stream);
    if (cfg->prec == FV_F64) {
        sph::Geometry<double> G = geometry_of<double>(s->ws, L);
        if (e == hipSuccess) e = sph::geometry<double>(G, cfg->n, s->stream);
        if (e == hipSuccess) e = sph::rate<double>((const double *)q, G, cfg->n, cfg->g, s->ctl(), s->rates(), 0, s->stream);
    } else {
        sph::Geometry<float> G = geometry_of<float>(s->ws, L);
        if (e == hipSuccess) e = sph::geometry<float>(G, cfg->n, s->stream);
        if (e == hipSuccess) e = sph::rate<float>((const float *)q, G, cfg->n, cfg->g, s->ctl(), s->rates(), 0, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpy(&bad, &s->ctl()->bad, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "sphere initialisation");
    }
    if (bad) {
        delete s;
        return fail(FV_E_INADMISSIBLE, "initial state not admissible (h <= 0 or a non-finite value)");
    }
    *out = s;
    return FV_OK;
}

fv_status fv_sphere_run(fv_sphere *s, int64_t nsteps)
{
    if (!s) return fail(FV_E_INVALID, "solver is NULL");
    if (nsteps < 0) return fail(FV_E_INVALID, "nsteps %lld < 0", (long long)nsteps);
    for (int64_t k = 0; k < nsteps; k++) {
        hipError_t e = s->cfg.prec == FV_F64 ? step<double>(s) : step<float>(s);
        if (e != hipSuccess) return hip_fail(e, "sphere step launch");
    }
    return FV_OK;
}

fv_status fv_sphere_time(fv_sphere *s, double *t, int64_t *steps)
{
    if (!s) return fail(FV_E_INVALID, "solver is NULL");
    hipError_t e = hipStreamSynchronize(s->stream);
    fvk::Ctl c;
    if (e == hipSuccess) e = hipMemcpy(&c, s->ctl(), sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read control block");
    if (t) *t = c.t;
    if (steps) *steps = c.step;
    if (c.bad) return fail(FV_E_INADMISSIBLE, "a cell became inadmissible at step %lld", (long long)c.step);
    return FV_OK;
}

fv_status fv_sphere_centres(fv_sphere *s, void *dst)
{
    if (!s || !dst) return fail(FV_E_INVALID, "NULL argument");
    const size_t bytes = 3 * (size_t)2 * s->cfg.n * s->cfg.n * es_of(&s->cfg);
    hipError_t e = hipMemcpyAsync(dst, s->ws + s->L.cen, bytes, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "copy centres");
}

fv_status fv_sphere_totals(fv_sphere *s, double *out)
{
    if (!s || !out) return fail(FV_E_INVALID, "NULL argument");
    double *dev = (double *)(s->ws + s->L.totals_out), *part = (double *)(s->ws + s->L.partials);
    const double *area = (const double *)(s->ws + s->L.area);
    hipError_t e = s->cfg.prec == FV_F64
                       ? sph::totals<double>((const double *)s->q, area, s->cfg.n, s->cfg.g, part,
                                             fvk::TOTALS_MAX_BLOCKS, dev, s->stream)
                       : sph::totals<float>((const float *)s->q, area, s->cfg.n, s->cfg.g, part,
                                            fvk::TOTALS_MAX_BLOCKS, dev, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? FV_OK : hip_fail(e, "sphere totals");
}

void fv_sphere_destroy(fv_sphere *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

}  // extern "C"
