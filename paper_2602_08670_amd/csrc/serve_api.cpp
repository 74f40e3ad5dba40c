// Serving: continuous batching of many independent solves on one GPU.
//
// Requests (shallow water over a bed, or Euler; square grids; their own step
// counts) wait in a FIFO queue.  At every round boundary the server admits
// queued requests whose device footprint fits the free part of the memory
// pool (first fit, later requests may pass one that does not fit), uploads
// their state and computes their first CFL rate.  A round then advances all
// active solves by up to K steps: for every step the host builds a list of
// the solves still running at that step per equation type (where their
// workgroups start in the launch, and their CFL slots at that step) -- a
// solve with fewer remaining steps simply drops out of the later lists --
// and each stage of each step is one batched launch over all tiles of the
// listed solves.  Shallow-water requests always run the bed kernel (a zero
// bed when none is given).  After the round, finished solves are copied back and their memory
// returns to the pool, so the next round can admit newly arrived requests
// while the long-running ones continue.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include "api_common.hpp"
#include "cnn_internal.hpp"
#include "fv_internal.hpp"

using fvapi::align256;
using fvapi::fail;
using fvapi::hip_fail;

namespace {

struct Req {
    int64_t id;
    fv_request r;
    std::vector<float> q0, bed, result;
    int state = 0;  // 0 queued, 1 active, 2 done, 3 failed
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t off = 0, bytes = 0;
    int slot = -1;
    int64_t done_steps = 0;
    int tiles_x = 0, tiles = 0;
    double sim_time = 0;
    size_t q_off, s1_off, bed_off, ctl_off, rates_off;
    size_t s2_off, z_off, small_off;  // learned requests
    int64_t fallback_faces = 0, redone_steps = 0;
    int rounds_queued = 0;  // rounds this request stayed queued
    int unfit = 0;          // rounds it did not fit (admission ageing)
    int nvar() const { return r.eqn == FV_EULER ? 4 : 3; }
    bool learned() const { return r.learned != 0; }
};

double side(const fv_request &r) { return r.lx > 0 ? r.lx : 1.0; }

// learned counters block: dt (float) at 0, two flag slots at 8, fallback
// faces at 16, redone steps at 24
constexpr size_t LS_DT = 0, LS_FLAGS = 8, LS_NFB = 16, LS_REDONE = 24, LS_BYTES = 256;

size_t req_bytes(const fv_request *r)
{
    size_t n2 = (size_t)r->n * r->n;
    if (r->learned)  // q, S1, S2, alpha (rounds with the separate network pass), control block, counters
        return 3 * align256(3 * n2 * 4) + align256(n2 * cnn::COUT * 4) + fvk::CTL_BYTES + LS_BYTES;
    int nvar = r->eqn == FV_EULER ? 4 : 3;
    size_t b = 2 * align256(nvar * n2 * 4) + fvk::CTL_BYTES + fvk::RATE_BYTES;
    if (r->eqn == FV_SWE) b += align256(n2 * 4);
    return b;
}

}  // namespace

// A captured round: its kernel nodes in launch order, each with the list
// whose tile count sets its grid before a replay (kind 0: plain stage list
// [step][type], 1: network pass of a step's learned list, 2: learned stage).
struct GraphNode {
    hipGraphNode_t node;
    hipKernelNodeParams p;
    int kind, idx;
};
struct RoundGraph {
    hipGraph_t g = nullptr;  // kept alive: the nodes are updated through it
    hipGraphExec_t x = nullptr;
    std::vector<GraphNode> nodes;
};

struct fv_server {
    fv_server_config cfg;
    char *pool;
    size_t pool_bytes;
    hipStream_t stream;
    std::chrono::steady_clock::time_point t0;
    // pool regions
    size_t tab_off, items_off, nitems_off, scratch_off, ltab_off, litems_off, lnitems_off, act_off, heap_off;
    std::map<size_t, size_t> free_list;  // offset -> size
    // host side
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::vector<int> free_slots;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    int64_t next_id = 1;
    fvk::WorkItem *h_items = nullptr;  // pinned
    int *h_nitems = nullptr;
    std::vector<fvk::BatchSolve> h_tab;
    cnn::LItem *h_litems = nullptr;    // pinned
    int *h_lnitems = nullptr;
    std::vector<cnn::LSolve> h_ltab;
    hipStream_t own_stream = nullptr;  // created when the caller passes the null stream
    // captured rounds, keyed by the kinds of work present | steps << 5
    std::map<int, RoundGraph> graphs;
    int64_t rounds = 0, replays = 0, grid_updates = 0, layered_rounds = 0;
    int cnn_cap = 256;  // most workgroups of a network-pass launch
    int split_at = 1024;  // network tiles from which a round's learned steps use separate launches
    int layered_at = 768;  // 16 x 16 tiles from which such a round's network pass runs layer by layer (-1: never)
    double launch_s = 0, wait_s = 0;  // host time enqueueing rounds' work, and waiting for it
    double capture_s = 0;             // host time capturing and instantiating graphs
    double admit_s = 0, retire_s = 0;  // host time admitting requests and retiring finished ones

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes;
                size_t noff = it->first + bytes;
                free_list.erase(it);
                if (rest) free_list[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_list.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_list.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_list.erase(nx);
        }
        if (it != free_list.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_list.erase(it);
            }
        }
    }
};

namespace {

void free_host(fv_server *s)
{
    if (s->h_items) (void)hipHostFree(s->h_items);
    if (s->h_nitems) (void)hipHostFree(s->h_nitems);
    if (s->h_litems) (void)hipHostFree(s->h_litems);
    if (s->h_lnitems) (void)hipHostFree(s->h_lnitems);
    s->h_items = nullptr;
    s->h_nitems = nullptr;
    s->h_litems = nullptr;
    s->h_lnitems = nullptr;
}

// one list per step and equation type, one item per active solve; list
// headers on the device: plain {items, tiles}, learned {items, network
// tiles, stage tiles, 0}
constexpr int HDR = 2, LHDR = 4;
constexpr size_t ACT_BYTES = 2 * 32 * 2;  // per cell: two BF16 32-channel activations
size_t items_capacity(const fv_server_config *c) { return (size_t)c->steps_per_round * 2 * c->max_solves; }

fv_status validate(const fv_server_config *c)
{
    if (!c || c->struct_size != sizeof(fv_server_config)) return fail(FV_E_INVALID, "server config struct_size");
    if (c->max_solves < 1 || c->steps_per_round < 1 || c->max_items < 1)
        return fail(FV_E_INVALID, "max_solves, steps_per_round and max_items must be >= 1");
    if (c->max_items > (uint64_t)1 << 31) return fail(FV_E_INVALID, "max_items above 2^31");
    if (c->direct != 0 && c->direct != 1) return fail(FV_E_INVALID, "direct must be 0 or 1");
    if (c->learned_split < 0 || c->learned_layered < -1) return fail(FV_E_INVALID, "learned_split < 0 or learned_layered < -1");
    if (c->act_pixels > ((uint64_t)1 << 34)) return fail(FV_E_INVALID, "act_pixels above 2^34");
    if (c->max_bypass < -1) return fail(FV_E_INVALID, "max_bypass %d < -1", c->max_bypass);
    if (c->reserved0 != 0) return fail(FV_E_INVALID, "reserved0 must be 0");
    return FV_OK;
}

// reference-depth reductions of a round's admissions: the totals partials,
// then one block of 8 doubles of output per solve slot
size_t scratch_bytes(const fv_server_config *c)
{
    return (size_t)fvk::TOTALS_MAX_BLOCKS * 5 * 8 + (size_t)c->max_solves * 8 * sizeof(double);
}

// learned solves: one list per step, one item per active learned solve
size_t litems_capacity(const fv_server_config *c) { return (size_t)c->steps_per_round * c->max_solves; }

size_t overhead(const fv_server_config *c)
{
    size_t o = align256(sizeof(fvk::BatchSolve) * c->max_solves);
    o += align256(items_capacity(c) * sizeof(fvk::WorkItem));
    o += align256((size_t)c->steps_per_round * 2 * HDR * sizeof(int));
    o += align256(scratch_bytes(c));
    o += align256(sizeof(cnn::LSolve) * c->max_solves);
    o += align256(litems_capacity(c) * sizeof(cnn::LItem));
    o += align256((size_t)c->steps_per_round * LHDR * sizeof(int));
    o += align256((size_t)c->act_pixels * ACT_BYTES);
    return o;
}

fv_status validate_req(const fv_request *r)
{
    if (!r || r->struct_size != sizeof(fv_request)) return fail(FV_E_INVALID, "request struct_size");
    if (r->eqn != FV_SWE && r->eqn != FV_EULER) return fail(FV_E_INVALID, "eqn %d", r->eqn);
    if (r->n < 8) return fail(FV_E_INVALID, "grid side %d < 8", r->n);
    if (r->bc != FV_BC_PERIODIC && r->bc != FV_BC_WALL) return fail(FV_E_INVALID, "bc %d", r->bc);
    if (r->steps < 0) return fail(FV_E_INVALID, "steps < 0");
    if (r->reserved1 != 0 || (r->learned != 0 && r->learned != 1)) return fail(FV_E_INVALID, "learned / reserved1");
    if (!(r->lx >= 0)) return fail(FV_E_INVALID, "domain side lx < 0");
    if (r->learned) {
        if (r->eqn != FV_SWE || r->bc != FV_BC_PERIODIC || r->bed || r->n % 16 || !(r->dt_fixed > 0) || !(r->g > 0))
            return fail(FV_E_INVALID, "learned requests: SWE, periodic, no bed, n %% 16 == 0, dt_fixed > 0, g > 0");
        if (!(r->h_ref >= 0)) return fail(FV_E_INVALID, "h_ref < 0");
        if (!r->q0) return fail(FV_E_INVALID, "initial state is NULL");
        return FV_OK;
    }
    if (!(r->cfl > 0 && r->cfl <= 1)) return fail(FV_E_INVALID, "cfl");
    if (!r->q0) return fail(FV_E_INVALID, "initial state is NULL");
    if (r->eqn == FV_EULER && r->bed) return fail(FV_E_INVALID, "a bed is only defined for shallow water");
    return FV_OK;
}

// Upload an admitted request and compute its first CFL rate (and reference
// depth for shallow water) exactly as fv_init does for a single solve.
fv_status admit_learned(fv_server *s, Req *q, std::vector<Req *> &need_h0)
{
    const fv_request &r = q->r;
    const size_t n2 = (size_t)r.n * r.n, st = align256(3 * n2 * 4);
    q->q_off = q->off;
    q->s1_off = q->q_off + st;
    q->s2_off = q->s1_off + st;
    q->z_off = q->s2_off + st;
    q->ctl_off = q->z_off + align256(n2 * cnn::COUT * 4);
    q->small_off = q->ctl_off + fvk::CTL_BYTES;
    char *P = s->pool;
    char small[LS_BYTES];
    std::memset(small, 0, sizeof small);
    const float dtf = (float)r.dt_fixed;
    std::memcpy(small + LS_DT, &dtf, sizeof dtf);
    hipError_t e = hipMemcpyAsync(P + q->q_off, q->q0.data(), 3 * n2 * 4, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(P + q->ctl_off, 0, fvk::CTL_BYTES, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(P + q->small_off, small, sizeof small, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // `small` is on this stack frame
    if (e != hipSuccess) return hip_fail(e, "admission upload");
    cnn::LSolve &d = s->h_ltab[q->slot];
    d = cnn::LSolve{};
    d.q = (float *)(P + q->q_off);
    d.s1 = (float *)(P + q->s1_off);
    d.s2 = (float *)(P + q->s2_off);
    d.z = (float *)(P + q->z_off);
    d.dt = (const float *)(P + q->small_off + LS_DT);
    d.flags = (int *)(P + q->small_off + LS_FLAGS);
    d.nfb = (unsigned long long *)(P + q->small_off + LS_NFB);
    d.redone = (unsigned long long *)(P + q->small_off + LS_REDONE);
    fvk::Ctl *ctl = (fvk::Ctl *)(P + q->ctl_off);
    d.fatal = &ctl->bad;
    d.t = &ctl->t;
    d.steps = &ctl->step;
    d.nx = d.ny = r.n;
    d.rdx = d.rdy = (float)(r.n / side(r));
    d.g = (float)r.g;
    d.sqg = std::sqrt((float)r.g);
    d.h0 = (float)r.h_ref;
    if (!(r.h_ref > 0)) need_h0.push_back(q);
    return FV_OK;
}

fv_status admit(fv_server *s, Req *q, std::vector<Req *> &need_h0)
{
    if (q->learned()) return admit_learned(s, q, need_h0);
    const fv_request &r = q->r;
    size_t n2 = (size_t)r.n * r.n;
    int nvar = q->nvar();
    q->q_off = q->off;
    q->s1_off = q->q_off + align256(nvar * n2 * 4);
    size_t o = q->s1_off + align256(nvar * n2 * 4);
    q->bed_off = 0;
    if (r.eqn == FV_SWE) {
        q->bed_off = o;
        o += align256(n2 * 4);
    }
    q->ctl_off = o;
    q->rates_off = o + fvk::CTL_BYTES;
    char *P = s->pool;
    hipError_t e = hipMemcpyAsync(P + q->q_off, q->q0.data(), nvar * n2 * 4, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && r.eqn == FV_SWE) {
        if (q->bed.empty()) e = hipMemsetAsync(P + q->bed_off, 0, n2 * 4, s->stream);
        else e = hipMemcpyAsync(P + q->bed_off, q->bed.data(), n2 * 4, hipMemcpyHostToDevice, s->stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(P + q->ctl_off, 0, fvk::CTL_BYTES + fvk::RATE_BYTES, s->stream);
    if (e != hipSuccess) return hip_fail(e, "admission upload");
    fvk::BatchSolve &d = s->h_tab[q->slot];
    d.q = P + q->q_off;
    d.s1 = P + q->s1_off;
    d.bed = r.eqn == FV_SWE ? P + q->bed_off : nullptr;
    d.ctl = P + q->ctl_off;
    d.rates = P + q->rates_off;
    d.nx = d.ny = r.n;
    d.bc_x = d.bc_y = r.bc;
    d.rdx = d.rdy = r.n / side(r);
    d.g = r.g;
    d.sqg = std::sqrt(r.g);
    d.gamma = r.gamma;
    d.h0 = r.eqn == FV_SWE ? r.h_ref : 0.0;
    d.cfl = r.cfl;
    d.dt_fixed = 0.0;
    fvk::StageDesc sd{};
    sd.prec = 0;
    sd.eqn = r.eqn;
    sd.bathy = r.eqn == FV_SWE;
    sd.nx = sd.ny = r.n;
    sd.bc_x = sd.bc_y = r.bc;
    sd.rdx = sd.rdy = r.n / side(r);
    sd.g = r.g;
    sd.gamma = r.gamma;
    e = fvk::launch_rate(sd, P + q->q_off, (fvk::Ctl *)(P + q->ctl_off), (unsigned long long *)(P + q->rates_off), 0,
                         s->stream);
    if (e != hipSuccess) return hip_fail(e, "admission rate kernel");
    if (r.eqn == FV_SWE && !(r.h_ref > 0)) need_h0.push_back(q);
    q->tiles_x = (r.n + fvk::TILE_X - 1) / fvk::TILE_X;
    q->tiles = q->tiles_x * ((r.n + fvk::TILE_Y - 1) / fvk::TILE_Y);
    return FV_OK;
}

// Launches of steps 0..nsteps-1 of a round over the uploaded lists, kinds
// of work in mask (1 SWE, 2 Euler, 4 learned, 8 learned steps with the
// network pass and the learned stage as separate launches, 16 that network
// pass layer by layer).  rec == NULL: direct launches
// of one workgroup per tile with the given per-list tile counts, empty lists
// skipped.  rec != NULL (graph capture): every launch of the mask, the tile
// counts read from the list headers, each node recorded in rec; its grid is
// a placeholder set before each replay.
hipError_t enqueue_steps(fv_server *s, int mask, int nsteps, const int *grids, const int *lgrid_cnn,
                         const int *lgrid_st, const int *lgrid_h, std::vector<GraphNode> *rec)
{
    char *P = s->pool;
    const size_t ncap = (size_t)s->cfg.max_solves;
    const fvk::BatchSolve *tab = (const fvk::BatchSolve *)(P + s->tab_off);
    const fvk::WorkItem *d_items = (const fvk::WorkItem *)(P + s->items_off);
    const int *d_nitems = (const int *)(P + s->nitems_off);
    const cnn::LSolve *ltab = (const cnn::LSolve *)(P + s->ltab_off);
    const cnn::LItem *d_litems = (const cnn::LItem *)(P + s->litems_off);
    const int *d_lnitems = (const int *)(P + s->lnitems_off);
    const fv_model *m = s->cfg.model;
    auto record = [&](int kind, int idx) -> hipError_t {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const hipGraphNode_t *deps = nullptr;
        size_t nd = 0;
        hipError_t e = hipStreamGetCaptureInfo_v2(s->stream, &cs, nullptr, nullptr, &deps, &nd);
        if (e != hipSuccess) return e;
        if (cs != hipStreamCaptureStatusActive || nd != 1 || !deps) return hipErrorStreamCaptureInvalidated;
        rec->push_back(GraphNode{deps[0], hipKernelNodeParams{}, kind, idx});
        return hipSuccess;
    };
    hipError_t e = hipSuccess;
    for (int k = 0; k < nsteps && e == hipSuccess; k++) {
        for (int stage = 1; stage <= 2 && e == hipSuccess; stage++)
            for (int type = 0; type < 2 && e == hipSuccess; type++) {
                if (!(mask >> type & 1)) continue;
                const size_t li = (size_t)k * 2 + type;
                const int eqn = type == 1 ? FV_EULER : FV_SWE;
                const fvk::WorkItem *it = d_items + li * ncap;
                const int *hdr = d_nitems + li * HDR;
                if (!rec) {
                    e = fvk::launch_batch_stage(eqn, type == 0, stage, tab, it, hdr, grids[li], s->stream);
                } else {
                    e = fvk::launch_batch_stage_list(eqn, type == 0, stage, tab, it, hdr, 8, s->stream);
                    if (e == hipSuccess) e = record(0, (int)li);
                }
            }
        if (!(mask & 4) || e != hipSuccess || (!rec && !lgrid_st[k])) continue;
        // learned solves: the network pass and learned stage of every
        // learned solve in one launch per stage (coefficients on chip), or,
        // with mask bit 8, a network-pass launch writing alpha (with mask
        // bit 16: five launches, one per layer) and a learned-stage launch
        // per stage; then commit-or-redo and redo.
        // Kind -2: fused pass, -1: network pass, >= 0: learned-stage mode.
        const cnn::LItem *it = d_litems + (size_t)k * ncap;
        const int *hdr = d_lnitems + (size_t)k * LHDR;
        const bool split = mask & 8;
        const int fmode[4] = {-2, -2, 2, 3}, fstg[4] = {1, 2, 0, 0};
        const int smode[6] = {-1, 0, -1, 0, 2, 3}, sstg[6] = {1, 1, 2, 2, 0, 0};
        const int nl = split ? 6 : 4;
        for (int j = 0; j < nl && e == hipSuccess; j++) {
            const int md = split ? smode[j] : fmode[j], sg = split ? sstg[j] : fstg[j];
            if (md == -1 && (mask & 16)) {
                void *a0 = P + s->act_off, *a1 = P + s->act_off + (size_t)s->cfg.act_pixels * (ACT_BYTES / 2);
                for (int layer = 0; layer < 5 && e == hipSuccess; layer++) {
                    e = cnn::launch_layer_list(layer, sg, m->packed, m->nrm, m->pr, ltab, it, hdr,
                                               rec ? 1 : lgrid_h[k], a0, a1, s->stream);
                    if (e == hipSuccess && rec) e = record(3, k);
                }
                continue;
            }
            if (!rec) {
                if (md == -2) e = cnn::launch_conv_learned(sg, m->packed, m->nrm, m->pr, ltab, it, hdr, lgrid_cnn[k],
                                                           s->stream);
                else if (md == -1) e = cnn::launch_forward_batch(sg, m->packed, m->nrm, m->pr, ltab, it, hdr,
                                                                 lgrid_cnn[k], s->stream);
                else e = cnn::launch_learned_batch(md, sg, ltab, it, hdr, lgrid_st[k], m->pr, s->stream);
            } else {
                if (md == -2) e = cnn::launch_conv_learned_list(sg, m->packed, m->nrm, m->pr, ltab, it, hdr, 1, s->stream);
                else if (md == -1) e = cnn::launch_forward_batch_list(sg, m->packed, m->nrm, m->pr, ltab, it, hdr, 1,
                                                                      s->stream);
                else e = cnn::launch_learned_batch_list(md, sg, ltab, it, hdr, 1, m->pr, s->stream);
                if (e == hipSuccess) e = record(md < 0 ? 1 : 2, k);
            }
        }
    }
    return e;
}

// The captured graph of a round's launches for (mask, nsteps), captured and
// instantiated on first use.
fv_status round_graph(fv_server *s, int mask, int nsteps, RoundGraph **out)
{
    const int key = mask | nsteps << 5;
    auto f = s->graphs.find(key);
    if (f != s->graphs.end()) {
        *out = &f->second;
        return FV_OK;
    }
    RoundGraph rg;
    const double t0 = s->now();
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    const hipError_t le = enqueue_steps(s, mask, nsteps, nullptr, nullptr, nullptr, nullptr, &rg.nodes);
    e = hipStreamEndCapture(s->stream, &rg.g);
    if (e == hipSuccess) e = le;
    for (size_t i = 0; i < rg.nodes.size() && e == hipSuccess; i++)
        e = hipGraphKernelNodeGetParams(rg.nodes[i].node, &rg.nodes[i].p);
    if (e == hipSuccess) e = hipGraphInstantiate(&rg.x, rg.g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (rg.g) (void)hipGraphDestroy(rg.g);
        return hip_fail(e, "graph capture");
    }
    *out = &(s->graphs[key] = rg);
    s->capture_s += s->now() - t0;
    return FV_OK;
}

// Before a replay: every node's grid from its list's tile count (at least
// one workgroup: an empty list's launch reads 0 tiles and does nothing).
hipError_t set_grids(fv_server *s, RoundGraph *rg, const int *grids, const int *lgrid_cnn, const int *lgrid_st,
                     const int *lgrid_h)
{
    for (GraphNode &n : rg->nodes) {
        int want;
        if (n.kind == 0) want = grids[n.idx] ? fvk::xcd_grid(grids[n.idx]) : 8;
        else if (n.kind == 1) want = lgrid_cnn[n.idx] ? (lgrid_cnn[n.idx] < s->cnn_cap ? lgrid_cnn[n.idx] : s->cnn_cap) : 1;
        else if (n.kind == 3) want = lgrid_h[n.idx] ? lgrid_h[n.idx] : 1;
        else want = lgrid_st[n.idx] ? lgrid_st[n.idx] : 1;
        if ((int)n.p.gridDim.x == want) continue;
        n.p.gridDim.x = (unsigned)want;
        const hipError_t e = hipGraphExecKernelNodeSetParams(rg->x, n.node, &n.p);
        if (e != hipSuccess) return e;
        s->grid_updates++;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t fv_server_pool_overhead(const fv_server_config *cfg) { return validate(cfg) == FV_OK ? overhead(cfg) : 0; }

size_t fv_request_bytes(const fv_request *r) { return validate_req(r) == FV_OK ? req_bytes(r) : 0; }

fv_status fv_server_create(const fv_server_config *cfg, void *pool, size_t pool_bytes, void *stream,
                           fv_server **out)
{
    if (!out) return fail(FV_E_INVALID, "out is NULL");
    *out = nullptr;
    fv_status rc = validate(cfg);
    if (rc != FV_OK) return rc;
    if (!pool || ((uintptr_t)pool & 255)) return fail(FV_E_INVALID, "pool must be a 256-byte aligned device buffer");
    size_t ov = overhead(cfg);
    if (pool_bytes < ov + 65536) return fail(FV_E_NOMEM, "pool %zu bytes < tables %zu + 64 KiB", pool_bytes, ov);
    auto s = std::make_unique<fv_server>();
    s->cfg = *cfg;
    s->pool = (char *)pool;
    s->pool_bytes = pool_bytes;
    s->stream = (hipStream_t)stream;
    s->t0 = std::chrono::steady_clock::now();
    s->tab_off = 0;
    s->items_off = align256(sizeof(fvk::BatchSolve) * cfg->max_solves);
    s->nitems_off = s->items_off + align256(items_capacity(cfg) * sizeof(fvk::WorkItem));
    s->scratch_off = s->nitems_off + align256((size_t)cfg->steps_per_round * 2 * HDR * sizeof(int));
    s->ltab_off = s->scratch_off + align256(scratch_bytes(cfg));
    s->litems_off = s->ltab_off + align256(sizeof(cnn::LSolve) * cfg->max_solves);
    s->lnitems_off = s->litems_off + align256(litems_capacity(cfg) * sizeof(cnn::LItem));
    s->act_off = s->lnitems_off + align256((size_t)cfg->steps_per_round * LHDR * sizeof(int));
    s->heap_off = ov;
    s->free_list[s->heap_off] = pool_bytes - s->heap_off;
    s->h_tab.assign(cfg->max_solves, fvk::BatchSolve{});
    s->h_ltab.assign(cfg->max_solves, cnn::LSolve{});
    for (int i = cfg->max_solves - 1; i >= 0; i--) s->free_slots.push_back(i);
    hipError_t e = hipHostMalloc((void **)&s->h_items, items_capacity(cfg) * sizeof(fvk::WorkItem), 0);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->h_nitems, (size_t)cfg->steps_per_round * 2 * HDR * sizeof(int), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_litems, litems_capacity(cfg) * sizeof(cnn::LItem), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_lnitems, (size_t)cfg->steps_per_round * LHDR * sizeof(int), 0);
    if (e != hipSuccess) {
        free_host(s.get());
        return hip_fail(e, "pinned work-list buffers");
    }
    if (cfg->model) s->cnn_cap = cnn::fused_max_grid();
    s->split_at = cfg->learned_split > 0 ? cfg->learned_split : 4 * s->cnn_cap;
    s->layered_at = cfg->learned_layered > 0 ? cfg->learned_layered : (cfg->learned_layered == 0 ? 768 : -1);
    if (!stream) {
        // graphs cannot be captured on the null stream: the server then
        // runs on a stream of its own (default priority)
        e = hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            free_host(s.get());
            return hip_fail(e, "server stream");
        }
        s->stream = s->own_stream;
    }
    *out = s.release();
    return FV_OK;
}

fv_status fv_server_submit(fv_server *s, const fv_request *r, int64_t *id)
{
    if (!s || !id) return fail(FV_E_INVALID, "NULL argument");
    fv_status rc = validate_req(r);
    if (rc != FV_OK) return rc;
    if (r->learned && !s->cfg.model) return fail(FV_E_INVALID, "a learned request needs a server model");
    {
        const uint64_t n = (uint64_t)r->n;
        const uint64_t own = r->learned ? (uint64_t)cnn::ltiles_st(r->n, r->n)
                                        : ((n + fvk::TILE_X - 1) / fvk::TILE_X) * ((n + fvk::TILE_Y - 1) / fvk::TILE_Y);
        const uint64_t own_cnn = r->learned ? (uint64_t)cnn::ltiles_cnn(r->n, r->n) : 0;
        if (own > s->cfg.max_items || own_cnn > s->cfg.max_items)
            return fail(FV_E_NOMEM, "request needs more than max_items = %llu tiles in one launch",
                        (unsigned long long)s->cfg.max_items);
    }
    if (req_bytes(r) > s->pool_bytes - s->heap_off)
        return fail(FV_E_NOMEM, "request needs %zu bytes, the pool holds %zu", req_bytes(r), s->pool_bytes - s->heap_off);
    auto q = std::make_unique<Req>();
    q->id = s->next_id++;
    q->r = *r;
    size_t n2 = (size_t)r->n * r->n;
    q->q0.assign(r->q0, r->q0 + (size_t)q->nvar() * n2);
    if (r->bed) q->bed.assign(r->bed, r->bed + n2);
    q->r.q0 = nullptr;
    q->r.bed = nullptr;
    q->bytes = req_bytes(r);
    q->t_submit = s->now();
    *id = q->id;
    s->queue.push_back(q.get());
    s->reqs[q->id] = std::move(q);
    return FV_OK;
}

fv_status fv_server_round(fv_server *s, int32_t *n_active, int32_t *n_queued)
{
    if (!s) return fail(FV_E_INVALID, "server is NULL");
    const int K = s->cfg.steps_per_round;
    char *P = s->pool;
    // ---- admission (FIFO, later requests may pass one that does not fit,
    // unless it has not fitted for max_bypass rounds: then nothing behind it
    // is admitted until it is)
    const double ta0 = s->now();
    const int max_bypass = s->cfg.max_bypass == 0 ? 8 : s->cfg.max_bypass;
    bool blocked = false;
    std::vector<Req *> admitted, need_h0;
    // tiles per launch of each kind (plain SWE, Euler, learned network pass,
    // learned stage): a request is admitted only while its launches stay
    // within max_items
    uint64_t tiles[4] = {0, 0, 0, 0};
    auto kind_tiles = [](const Req *q, uint64_t t[4]) {
        const int n = q->r.n;
        if (q->learned()) {
            t[2] += (uint64_t)cnn::ltiles_cnn(n, n);
            t[3] += (uint64_t)cnn::ltiles_st(n, n);
        } else {
            t[q->r.eqn == FV_EULER ? 1 : 0] +=
                (uint64_t)((n + fvk::TILE_X - 1) / fvk::TILE_X) * ((n + fvk::TILE_Y - 1) / fvk::TILE_Y);
        }
    };
    for (Req *q : s->active) kind_tiles(q, tiles);
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Req *q = *it;
        if (blocked) {
            q->rounds_queued++;
            ++it;
            continue;
        }
        size_t off;
        uint64_t after[4] = {tiles[0], tiles[1], tiles[2], tiles[3]};
        kind_tiles(q, after);
        bool fits = true;
        for (int k = 0; k < 4; k++) fits = fits && after[k] <= s->cfg.max_items;
        if (fits && !s->free_slots.empty() && s->alloc(q->bytes, &off)) {
            for (int k = 0; k < 4; k++) tiles[k] = after[k];
            q->off = off;
            q->slot = s->free_slots.back();
            s->free_slots.pop_back();
            fv_status rc = admit(s, q, need_h0);
            if (rc != FV_OK) return rc;
            q->state = 1;
            q->t_admit = s->now();
            admitted.push_back(q);
            s->active.push_back(q);
            it = s->queue.erase(it);
        } else {
            q->rounds_queued++;
            if (max_bypass > 0 && ++q->unfit >= max_bypass) blocked = true;
            ++it;
        }
    }
    hipError_t e = hipSuccess;
    if (!need_h0.empty()) {
        // reference depth = mean initial depth, as fv_init computes it: the
        // round's reductions are enqueued back to back (each into its own
        // output block; they share the partials, in stream order), read back
        // with one copy and one synchronisation
        double *partials = (double *)(P + s->scratch_off);
        double *outs = partials + (size_t)fvk::TOTALS_MAX_BLOCKS * 5;
        for (size_t k = 0; k < need_h0.size() && e == hipSuccess; k++) {
            const Req *q = need_h0[k];
            fvk::StageDesc sd{};
            sd.prec = 0;
            sd.eqn = FV_SWE;
            sd.nx = sd.ny = q->r.n;
            sd.rdx = sd.rdy = q->r.n / side(q->r);
            sd.g = q->r.g;
            e = fvk::launch_totals(sd, P + q->q_off, partials, fvk::TOTALS_MAX_BLOCKS, outs + 8 * k, s->stream);
        }
        std::vector<double> tot(8 * need_h0.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(tot.data(), outs, tot.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "reference depth");
        for (size_t k = 0; k < need_h0.size(); k++) {
            const Req *q = need_h0[k];
            const double h0 = tot[8 * k] / (side(q->r) * side(q->r));  // mean depth = mass / area
            if (q->learned()) s->h_ltab[q->slot].h0 = (float)h0;
            else s->h_tab[q->slot].h0 = h0;
        }
    }
    if (!admitted.empty()) {
        e = hipMemcpyAsync(P + s->tab_off, s->h_tab.data(), sizeof(fvk::BatchSolve) * s->cfg.max_solves,
                           hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P + s->ltab_off, s->h_ltab.data(), sizeof(cnn::LSolve) * s->cfg.max_solves,
                               hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return hip_fail(e, "solve table upload");
    }
    s->admit_s += s->now() - ta0;
    // ---- work-lists of the round: one list per [step][type] (type 0 = SWE,
    // 1 = Euler) of the solves still running at that step, packed back to
    // back; tiles per launch are capped by max_items
    const size_t ncap = (size_t)s->cfg.max_solves;
    std::vector<int> counts((size_t)K * 2, 0), grids((size_t)K * 2, 0);
    std::vector<int> lcounts((size_t)K, 0), lgrid_cnn((size_t)K, 0), lgrid_st((size_t)K, 0), lgrid_h((size_t)K, 0);
    bool all16 = true;  // every learned side a multiple of 16 (the layer-by-layer pass's tiles)
    for (int k = 0; k < K; k++)
        for (Req *q : s->active) {
            if (q->r.steps - q->done_steps <= k) continue;
            if (q->learned()) {
                const int tc = cnn::ltiles_cnn(q->r.n, q->r.n), ts = cnn::ltiles_st(q->r.n, q->r.n);
                if ((uint64_t)lgrid_cnn[k] + tc > s->cfg.max_items || (uint64_t)lgrid_st[k] + ts > s->cfg.max_items)
                    return fail(FV_E_NOMEM, "more than max_items = %llu tiles in one launch",
                                (unsigned long long)s->cfg.max_items);
                cnn::LItem &w = s->h_litems[(size_t)k * ncap + lcounts[k]];
                w.solve = q->slot;
                w.tb_cnn = lgrid_cnn[k];
                w.tb_st = lgrid_st[k];
                w.parity = (int)((q->done_steps + k) & 1);
                w.tb_h = lgrid_h[k];
                lcounts[k]++;
                lgrid_cnn[k] += tc;
                lgrid_st[k] += ts;
                if (q->r.n % 16) all16 = false;
                else lgrid_h[k] += (q->r.n / 16) * (q->r.n / 16);
                continue;
            }
            int type = q->r.eqn == FV_EULER ? 1 : 0;
            size_t li = (size_t)k * 2 + type;
            if ((uint64_t)grids[li] + q->tiles > s->cfg.max_items)
                return fail(FV_E_NOMEM, "more than max_items = %llu tiles in one launch",
                            (unsigned long long)s->cfg.max_items);
            fvk::WorkItem &w = s->h_items[li * ncap + counts[li]];
            int64_t st = q->done_steps + k;
            w.solve = q->slot;
            w.tile_begin = grids[li];
            w.tiles_x = q->tiles_x;
            w.ri = (unsigned char)(st % 3);
            w.ro = (unsigned char)((st + 1) % 3);
            w.rc = (unsigned char)((st + 2) % 3);
            w.pad = 0;
            counts[li]++;
            grids[li] += q->tiles;
        }
    int mask = 0, nsteps = 0;  // kinds of work present (1 SWE, 2 Euler, 4 learned), last non-empty step + 1
    for (int k = 0; k < K; k++) {
        const int m = (counts[(size_t)k * 2] ? 1 : 0) | (counts[(size_t)k * 2 + 1] ? 2 : 0) | (lcounts[k] ? 4 : 0);
        if (m) nsteps = k + 1;
        mask |= m;
    }
    // many learned tiles: separate network-pass and learned-stage launches
    // (the network pass then strides over tiles at full occupancy of the
    // learned stage); few: one launch per stage, coefficients on chip
    if ((mask & 4) && lgrid_cnn[0] >= s->split_at) mask |= 8;
    // many more: the network pass layer by layer (activations in the pool's
    // scratch; a step's lists only shrink over the round)
    if ((mask & 8) && all16 && s->layered_at > 0 && lgrid_h[0] >= s->layered_at &&
        (uint64_t)lgrid_h[0] * 256 <= s->cfg.act_pixels)
        mask |= 16;
    for (size_t li = 0; li < counts.size(); li++) {
        s->h_nitems[li * HDR] = counts[li];
        s->h_nitems[li * HDR + 1] = grids[li];
    }
    fvk::WorkItem *d_items = (fvk::WorkItem *)(P + s->items_off);
    int *d_nitems = (int *)(P + s->nitems_off);
    size_t used = 0;  // the lists are uploaded up to the last non-empty one
    for (size_t li = 0; li < counts.size(); li++)
        if (counts[li]) used = li * ncap + counts[li];
    e = hipMemcpyAsync(d_items, s->h_items, used * sizeof(fvk::WorkItem), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_nitems, s->h_nitems, (size_t)K * 2 * HDR * sizeof(int), hipMemcpyHostToDevice,
                           s->stream);
    // learned lists
    cnn::LItem *d_litems = (cnn::LItem *)(P + s->litems_off);
    int *d_lnitems = (int *)(P + s->lnitems_off);
    size_t lused = 0;
    for (int k = 0; k < K; k++) {
        s->h_lnitems[k * LHDR] = lcounts[k];
        s->h_lnitems[k * LHDR + 1] = lgrid_cnn[k];
        s->h_lnitems[k * LHDR + 2] = lgrid_st[k];
        s->h_lnitems[k * LHDR + 3] = lgrid_h[k];
        if (lcounts[k]) lused = (size_t)k * ncap + lcounts[k];
    }
    if (e == hipSuccess && lused)
        e = hipMemcpyAsync(d_litems, s->h_litems, lused * sizeof(cnn::LItem), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && lused)
        e = hipMemcpyAsync(d_lnitems, s->h_lnitems, (size_t)K * LHDR * sizeof(int), hipMemcpyHostToDevice,
                           s->stream);
    if (e != hipSuccess) return hip_fail(e, "work-list upload");
    if (nsteps) s->rounds++;
    if (nsteps && (mask & 16)) s->layered_rounds++;
    const double tl0 = s->now();
    if (s->cfg.direct) {
        e = enqueue_steps(s, mask, nsteps, grids.data(), lgrid_cnn.data(), lgrid_st.data(), lgrid_h.data(), nullptr);
    } else if (nsteps) {
        // the round's launches are one captured graph per (kinds present,
        // steps rounded up to a power of two); between replays only the
        // work-lists uploaded above and the launch grids change
        int ng = 1;
        while (ng < nsteps) ng <<= 1;
        if (ng > K) ng = K;
        RoundGraph *rg = nullptr;
        fv_status rc = round_graph(s, mask, ng, &rg);
        if (rc != FV_OK) return rc;
        e = set_grids(s, rg, grids.data(), lgrid_cnn.data(), lgrid_st.data(), lgrid_h.data());
        if (e == hipSuccess) e = hipGraphLaunch(rg->x, s->stream);
        s->replays++;
    }
    const double tl1 = s->now();
    s->launch_s += tl1 - tl0;
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "round");
    s->wait_s += s->now() - tl1;
    // ---- retire finished solves
    double tnow = s->now();
    for (auto it = s->active.begin(); it != s->active.end();) {
        Req *q = *it;
        int64_t adv = q->r.steps - q->done_steps < K ? q->r.steps - q->done_steps : K;
        q->done_steps += adv;
        if (q->done_steps < q->r.steps) {
            ++it;
            continue;
        }
        size_t n = (size_t)q->nvar() * q->r.n * q->r.n;
        q->result.resize(n);
        fvk::Ctl c;
        e = hipMemcpy(q->result.data(), P + q->q_off, n * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(&c, P + q->ctl_off, sizeof c, hipMemcpyDeviceToHost);
        if (e == hipSuccess && q->learned()) {
            unsigned long long cnt[2];
            e = hipMemcpy(cnt, P + q->small_off + LS_NFB, sizeof cnt, hipMemcpyDeviceToHost);
            q->fallback_faces = (int64_t)cnt[0];
            q->redone_steps = (int64_t)cnt[1];
        }
        if (e != hipSuccess) return hip_fail(e, "result copy");
        q->sim_time = c.t;
        q->state = c.bad ? 3 : 2;
        q->t_done = tnow;
        s->release(q->off, q->bytes);
        s->free_slots.push_back(q->slot);
        q->slot = -1;
        it = s->active.erase(it);
    }
    s->retire_s += s->now() - tnow;
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return FV_OK;
}

fv_status fv_server_get_stats(fv_server *s, fv_server_stats *out)
{
    if (!s || !out) return fail(FV_E_INVALID, "NULL argument");
    *out = fv_server_stats{};
    out->rounds = s->rounds;
    out->graph_replays = s->replays;
    out->grid_updates = s->grid_updates;
    out->graphs_captured = (int32_t)s->graphs.size();
    out->layered_rounds = (int32_t)s->layered_rounds;
    out->host_launch_s = s->launch_s;
    out->host_wait_s = s->wait_s;
    out->host_capture_s = s->capture_s;
    out->host_admit_s = s->admit_s;
    out->host_retire_s = s->retire_s;
    return FV_OK;
}

fv_status fv_server_info(fv_server *s, int64_t id, fv_request_info *info)
{
    if (!s || !info) return fail(FV_E_INVALID, "NULL argument");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(FV_E_INVALID, "unknown request %lld", (long long)id);
    const Req &q = *it->second;
    info->state = q.state;
    info->rounds_queued = q.rounds_queued;
    info->steps_done = q.done_steps;
    info->t_submit = q.t_submit;
    info->t_admit = q.t_admit;
    info->t_done = q.t_done;
    info->sim_time = q.sim_time;
    info->fallback_faces = q.fallback_faces;
    info->redone_steps = q.redone_steps;
    return FV_OK;
}

fv_status fv_server_result(fv_server *s, int64_t id, float *dst)
{
    if (!s || !dst) return fail(FV_E_INVALID, "NULL argument");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(FV_E_INVALID, "unknown request %lld", (long long)id);
    const Req &q = *it->second;
    if (q.state < 2) return fail(FV_E_INVALID, "request %lld is not finished", (long long)id);
    std::memcpy(dst, q.result.data(), q.result.size() * 4);
    return q.state == 3 ? fail(FV_E_INADMISSIBLE, "request %lld became inadmissible", (long long)id) : FV_OK;
}

fv_status fv_server_release(fv_server *s, int64_t id)
{
    if (!s) return fail(FV_E_INVALID, "server is NULL");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second->state < 2) return fail(FV_E_INVALID, "request is not finished");
    s->reqs.erase(it);
    return FV_OK;
}

void fv_server_destroy(fv_server *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto &g : s->graphs) {
        if (g.second.x) (void)hipGraphExecDestroy(g.second.x);
        if (g.second.g) (void)hipGraphDestroy(g.second.g);
    }
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    free_host(s);
    delete s;
}

}  // extern "C"
