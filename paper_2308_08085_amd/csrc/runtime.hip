// runtime.hip -- host runtime behind the C ABI of include/amr_lbm.h: arena
// carve-up, the recursive sub-cycled schedule (optionally replayed from a HIP
// graph), tagging and adaptation sequencing, field access.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "runtime_internal.h"

using namespace amr;

namespace {
thread_local std::string g_err;
}  // namespace

namespace amr {

amr_status fail(amr_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

LevelParams level_params(const amr_handle *h) {
    LevelParams lp;
    for (int L = 0; L < kMaxLevels; L++) {
        lp.par[L] = L < h->lmax ? h->par[L] : 0;
        lp.omega[L] = L < h->lmax ? 1.0 / h->tau[L] : 0.0;
        lp.r_cf[L] = L + 1 < h->lmax ? h->tau[L + 1] / (2.0 * h->tau[L]) : 0.0;
        lp.r_fc[L] = L + 1 < h->lmax ? 2.0 * h->tau[L] / h->tau[L + 1] : 0.0;
    }
    return lp;
}

}  // namespace amr

namespace {

int nroot_of(const amr_config *c) { return c->root[0] * c->root[1] * (c->dim == 3 ? c->root[2] : 1); }

amr_status validate(const amr_config *c) {
    if (!c) return fail(AMR_ERR_ARG, "config is NULL");
    if (!((c->dim == 2 && c->q == 9) || (c->dim == 3 && (c->q == 19 || c->q == 27))))
        return fail(AMR_ERR_ARG, "unsupported lattice dim=%d q=%d", c->dim, c->q);
    if (c->max_levels < 1 || c->max_levels > kMaxLevels)
        return fail(AMR_ERR_ARG, "max_levels must be in [1, %d]", kMaxLevels);
    for (int a = 0; a < c->dim; a++)
        if (c->root[a] < 1) return fail(AMR_ERR_ARG, "root[%d] must be >= 1", a);
    if (c->dim == 2 && c->root[2] != 1) return fail(AMR_ERR_ARG, "root[2] must be 1 in 2-D");
    const long long nroot = (long long)c->root[0] * c->root[1] * (c->dim == 3 ? c->root[2] : 1);
    if (c->max_blocks < nroot) return fail(AMR_ERR_ARG, "max_blocks (%d) < root blocks (%lld)", c->max_blocks, nroot);
    const long long mb = c->dim == 2 ? 16 : 64;
    if ((long long)c->max_blocks * mb > (1ll << 31) - 1 || (long long)c->max_blocks * c->max_levels > (1ll << 31) - 1)
        return fail(AMR_ERR_ARG, "max_blocks too large for 32-bit cell offsets");
    if (c->storage < AMR_F64 || c->storage > AMR_BF16S) return fail(AMR_ERR_ARG, "unknown storage %d", c->storage);
    if (!(c->nu0 > 0.0)) return fail(AMR_ERR_ARG, "nu0 must be positive");
    if (c->interp != AMR_INTERP_LINEAR && c->interp != AMR_INTERP_CUBIC)
        return fail(AMR_ERR_ARG, "unknown interpolation %d", c->interp);
    for (int f = 0; f < 6; f++)
        if (c->face_kind[f] != AMR_FACE_VELOCITY && c->face_kind[f] != AMR_FACE_OUTFLOW)
            return fail(AMR_ERR_ARG, "face_kind[%d] invalid", f);
    return AMR_OK;
}

void make_layout(const amr_config *c, Layout *L) {
    const size_t cap = (size_t)c->max_blocks, lmax = (size_t)c->max_levels;
    const size_t mb = c->dim == 2 ? 16 : 64, nb = c->dim == 2 ? 9 : 27, q = (size_t)c->q;
    const size_t capc = cap * mb, sb = storage_bytes(c->storage);
    const size_t nroot = (size_t)nroot_of(c);
    const size_t fslots = q * capc + cap * (size_t)halo_entries(c->q);  // rows + halo records
    size_t t = 0;
    auto take = [&](size_t bytes) {
        size_t o = align256(t);
        t = o + bytes;
        return o;
    };
    L->f[0] = take(fslots * sb);
    L->f[1] = take(fslots * sb);
    L->hid = take(cap * 4);
    L->parent = take(cap * 4);
    L->fresh = take(cap);
    L->U = take(3 * capc * 8);
    L->nbr = take(nb * cap * 4);
    L->nbrc = take(nb * cap * 4);
    L->X = take(3 * cap * 4);
    L->level = take(cap);
    L->status = take(cap);
    L->tag = take(cap);
    L->ldes = take(cap);
    L->viol = take(cap);
    L->bflag = take(cap);
    L->gmask = take(cap * 8);
    L->imask = take(cap * 8);
    L->ids = take(lmax * cap * 4);
    L->ids_tmp = take(lmax * cap * 4);
    L->iface = take(lmax * cap * 4);
    L->refl = take(lmax * cap * 4);
    L->sweep = take(lmax * cap * 4);
    L->order = take(lmax * cap * 4);
    L->force = take(cap * 3 * 8);
    L->solidl = take(lmax * cap * 4);
    L->gap = take(cap * 4);
    L->first = take(cap * 4);
    L->rlist = take(cap * 4);
    L->clist = take(cap * 4);
    L->cnt = take(cap * 4);
    L->off = take(cap * 4);
    L->rank = take(lmax * cap * 4);
    L->bins = take(lmax * cap);
    L->scan_part = take(((lmax * cap + 1023) / 1024 + 1) * kMaxLevels * 4);
    L->crit = take(cap * 8);
    L->part4 = take(cap * 32);
    L->solid = take(nroot);
    L->solid_list = take(nroot * 4);
    L->ctr = take(sizeof(DevCounters));
    size_t need = capc * (q > 4 ? q : 4) * 8;
    size_t sbytes = need < (size_t(1) << 20) ? (size_t(1) << 20) : (need > (size_t(64) << 20) ? (size_t(64) << 20) : need);
    L->staging_bytes = sbytes;
    L->staging = take(sbytes);
    L->total = align256(t);
}


hipEvent_t take_event(amr_handle *h) {
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// distribution bytes a launch must move: every cell of a processed block reads
// and writes Q populations (collide-stream, plus the block's links, flags and
// list entry); a ghost fill of level L reads each interface parent's cells and
// writes the ghost cells of its children; an average writes each targeted
// parent cell from 2^d fine cells (both plus the children's cell masks).
double launch_bytes(const amr_handle *h, int kind, double blocks, int L) {
    const double q = h->c.q, mb = h->c.mb, nc = h->c.nc, sb = (double)storage_bytes(h->c.storage);
    const double links = h->c.nb * 4.0 + 1.0 + 4.0;
    if (kind == 0) return blocks * (2.0 * q * mb * sb + links);
    if (kind == 1) return blocks * (q * mb * sb + 8.0 * nc) + h->ghost_w[L] * q * sb;
    return blocks * 8.0 * nc + h->avg_w[L] * (nc + 1.0) * q * sb;
}

template <typename F>
void timed_launch(amr_handle *h, int kind, int blocks, int L, F &&fn) {
    if (!h->profiling || blocks <= 0) {
        fn();
        return;
    }
    hipEvent_t a = take_event(h), b = take_event(h);
    if (a) hipEventRecord(a, h->c.stream);
    fn();
    if (b) hipEventRecord(b, h->c.stream);
    if (a && b) h->timed.push_back({kind, a, b, (double)blocks, launch_bytes(h, kind, blocks, L)});
}

// Outside profiled runs (which time each kernel on its own) BGK sweeps save
// launch gaps (~10 us each): a sweep with ordinary stores adds the momentum
// exchange itself (the variant needs at most 3 more VGPRs, with no loss of
// occupancy), and on small levels the ghost interpolation into level L+1 joins
// the sweep.  Large levels keep the interpolation apart: the joined kernel
// needs more registers (99 VGPRs for D3Q27 at 16-bit storage against 68) and
// their launches are long.
static bool join_launches(const amr_handle *h) { return h->c.coll == AMR_COLLIDE_BGK && !h->profiling; }

static bool small_level(const amr_handle *h, int L) {
    return h->nids[L] <= (h->c.dim == 3 ? 16384 : 65536);  // blocks of 64 / 16 cells
}

// The blocks a sweep of level L processes, in launch order: every block of the
// level's ID set (Sec. "Grid Advancement"), or with AMR_FIELD_SKIP_PARENTS all
// but the refined blocks none of whose children has an N_SKIP link.  Such a
// deep parent touches no coarser leaf: its stale cells reach only neighbouring
// parents, on their sides away from any coarse leaf, where the interface
// averaging of every step stops them before the cells that linear
// interpolation reads; the next synchronisation averages them all again.
// Leaf results are unchanged bit for bit (tested).
static const int32_t *sweep_list(const amr_handle *h, int L, int *n) {
    const size_t at = (size_t)L * h->c.m.cap;
    *n = h->skip_parents ? h->nsweep[L] : h->nids[L];
    return (h->skip_parents ? h->c.sweep : h->c.order) + at;
}

// fused: the sweep was launched together with the ghost interpolation into
// level L+1 (launch_interp_collide); exchanged: that launch also added the
// momentum exchange
void collide_stream(amr_handle *h, int L, bool fused = false, bool exchanged = false) {
    const LevelParams lp = level_params(h);
    const bool exchange = h->force_on && h->nsolid[L] > 0;
    int n = 0;
    const int32_t *list = sweep_list(h, L, &n);
    if (!fused)
        timed_launch(h, 0, n, L, [&] {
            exchanged = launch_collide_stream(h->c, list, n, L, lp, h->bc, exchange && join_launches(h));
        });
    h->par[L] ^= 1;
    // momentum exchange with solid blocks, from the buffer just written
    if (exchange && !exchanged)
        launch_exchange(h->c, h->c.solidl + (size_t)L * h->c.m.cap, h->nsolid[L], L, level_params(h));
}

// recursive sub-cycled advancement (Sec. "Grid Advancement")
void step_level(amr_handle *h, int L) {
    if (L == h->lmax - 1) {
        collide_stream(h, L);
        return;
    }
    const size_t cap = (size_t)h->c.m.cap;
    const bool fuse = h->niface[L] > 0 && join_launches(h) && small_level(h, L);
    bool exchanged = false;
    if (fuse) {
        const LevelParams lp = level_params(h);
        int n = 0;
        const int32_t *list = sweep_list(h, L, &n);
        exchanged = launch_interp_collide(h->c, h->c.iface + L * cap, h->niface[L], list, n, L, lp, h->bc,
                                          h->force_on && h->nsolid[L] > 0);
    } else if (h->niface[L] > 0) {
        const LevelParams lp = level_params(h);
        timed_launch(h, 1, h->niface[L], L, [&] { launch_interp(h->c, h->c.iface + L * cap, h->niface[L], lp, 0); });
    }
    collide_stream(h, L, fuse, exchanged);
    step_level(h, L + 1);
    step_level(h, L + 1);
    if (h->niface[L] > 0) {
        const LevelParams lp = level_params(h);
        timed_launch(h, 2, h->niface[L], L, [&] { launch_average(h->c, h->c.iface + L * cap, h->niface[L], lp, 0); });
    }
}

amr_status collect_timings(amr_handle *h) {
    HIP_TRY(hipStreamSynchronize(h->c.stream));
    for (auto &t : h->timed) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
        h->kstats[t.kind][0] += 1.0;
        h->kstats[t.kind][1] += ms;
        h->kstats[t.kind][2] += t.blocks;
        h->kstats[t.kind][3] += t.bytes;
        h->event_pool.push_back(t.a);
        h->event_pool.push_back(t.b);
    }
    h->timed.clear();
    return AMR_OK;
}

amr_status read_counters(amr_handle *h, DevCounters *out) {
    HIP_TRY(hipMemcpyAsync(out, h->c.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, h->c.stream));
    HIP_TRY(hipStreamSynchronize(h->c.stream));
    return AMR_OK;
}

amr_status refresh_counts(amr_handle *h) {
    DevCounters dc;
    amr_status s = read_counters(h, &dc);
    if (s != AMR_OK) return s;
    for (int L = 0; L < kMaxLevels; L++) {
        h->nids[L] = L < h->lmax ? dc.nids[L] : 0;
        h->niface[L] = L < h->lmax ? dc.niface[L] : 0;
        h->nref[L] = L < h->lmax ? dc.nref[L] : 0;
        h->nsweep[L] = L < h->lmax ? dc.nsweep[L] : 0;
        h->nsolid[L] = L < h->lmax ? dc.nsolid[L] : 0;
        h->ghost_w[L] = L < h->lmax ? (double)dc.ghost_w[L] : 0.0;
        h->avg_w[L] = L < h->lmax ? (double)dc.avg_w[L] : 0.0;
    }
    h->gtop = dc.gtop;
    return AMR_OK;
}

void drop_graphs(amr_handle *h) {
    for (int i = 0; i < 2; i++)
        if (h->gexec[i]) {
            hipGraphExecDestroy(h->gexec[i]);
            h->gexec[i] = nullptr;
        }
    h->graph_ok = false;
}

amr_status sync_checked(amr_handle *h) {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->c.stream));
    return AMR_OK;
}

}  // namespace

extern "C" {

const char *amr_last_error(void) { return g_err.c_str(); }

amr_status amr_query_bytes(const amr_config *cfg, uint64_t *arena_bytes) {
    amr_status s = validate(cfg);
    if (s != AMR_OK) return s;
    if (!arena_bytes) return fail(AMR_ERR_ARG, "arena_bytes is NULL");
    Layout L;
    make_layout(cfg, &L);
    *arena_bytes = L.total;
    return AMR_OK;
}

amr_status amr_create(const amr_config *cfg, void *dev_arena, uint64_t arena_bytes, void *hip_stream, amr_t **out) {
    amr_status s = validate(cfg);
    if (s != AMR_OK) return s;
    if (!out) return fail(AMR_ERR_ARG, "out is NULL");
    if (!dev_arena) return fail(AMR_ERR_ARG, "dev_arena is NULL");
    if (((uintptr_t)dev_arena & 255) != 0) return fail(AMR_ERR_ARG, "dev_arena must be 256-byte aligned");
    Layout lay;
    make_layout(cfg, &lay);
    if (arena_bytes < lay.total)
        return fail(AMR_ERR_CAPACITY, "arena of %llu bytes is smaller than the %llu bytes required",
                    (unsigned long long)arena_bytes, (unsigned long long)lay.total);
    amr_handle *h = new amr_handle();
    h->cfg = *cfg;
    h->cfg.solid_root = nullptr;
    h->lay = lay;
    h->lmax = cfg->max_levels;
    const int nroot = nroot_of(cfg);
    if (cfg->solid_root) h->solid.assign(cfg->solid_root, cfg->solid_root + nroot);
    char *a = (char *)dev_arena;
    Ctx &c = h->c;
    c.dim = cfg->dim;
    c.q = cfg->q;
    c.nb = cfg->dim == 2 ? 9 : 27;
    c.mb = cfg->dim == 2 ? 16 : 64;
    c.nc = cfg->dim == 2 ? 4 : 8;
    c.storage = cfg->storage;
    c.nroot = nroot;
    for (int ax = 0; ax < 3; ax++) {
        c.root[ax] = ax < cfg->dim ? cfg->root[ax] : 1;
        c.periodic[ax] = ax < cfg->dim ? (cfg->periodic[ax] ? 1 : 0) : 0;
    }
    for (int f = 0; f < 6; f++) {
        c.face_prio[f] = cfg->face_prio[f];
        c.face_kind[f] = cfg->face_kind[f];
        h->bc.kind[f] = cfg->face_kind[f];
        for (int ax = 0; ax < 3; ax++) h->bc.u[f][ax] = cfg->face_u[f][ax];
    }
    c.m.cap = cfg->max_blocks;
    c.m.capc = (int64_t)cfg->max_blocks * c.mb;
    c.m.lmax = cfg->max_levels;
    c.m.halo_base = (int64_t)cfg->max_blocks * c.q * c.mb;
    c.m.nh = halo_entries(cfg->q);
    c.m.interp = cfg->interp;
    c.m.hid = (int32_t *)(a + lay.hid);
    c.m.parent = (int32_t *)(a + lay.parent);
    c.m.fresh = (int8_t *)(a + lay.fresh);
    c.U = (double *)(a + lay.U);
    c.m.nbr = (int32_t *)(a + lay.nbr);
    c.m.nbrc = (int32_t *)(a + lay.nbrc);
    c.m.X = (int32_t *)(a + lay.X);
    c.m.level = (int8_t *)(a + lay.level);
    c.m.status = (int8_t *)(a + lay.status);
    c.m.tag = (int8_t *)(a + lay.tag);
    c.m.ldes = (int8_t *)(a + lay.ldes);
    c.m.viol = (int8_t *)(a + lay.viol);
    c.m.bflag = (uint8_t *)(a + lay.bflag);
    c.m.gmask = (uint64_t *)(a + lay.gmask);
    c.m.imask = (uint64_t *)(a + lay.imask);
    c.f[0] = a + lay.f[0];
    c.f[1] = a + lay.f[1];
    c.ids = (int32_t *)(a + lay.ids);
    c.ids_tmp = (int32_t *)(a + lay.ids_tmp);
    c.iface = (int32_t *)(a + lay.iface);
    c.refl = (int32_t *)(a + lay.refl);
    c.sweep = (int32_t *)(a + lay.sweep);
    c.order = (int32_t *)(a + lay.order);
    c.m.force = (double *)(a + lay.force);
    c.solidl = (int32_t *)(a + lay.solidl);
    c.gap = (int32_t *)(a + lay.gap);
    c.first = (int32_t *)(a + lay.first);
    c.rlist = (int32_t *)(a + lay.rlist);
    c.clist = (int32_t *)(a + lay.clist);
    c.cnt = (int32_t *)(a + lay.cnt);
    c.off = (int32_t *)(a + lay.off);
    c.rank = (int32_t *)(a + lay.rank);
    c.bins = (int8_t *)(a + lay.bins);
    c.scan_part = (int32_t *)(a + lay.scan_part);
    c.crit = (double *)(a + lay.crit);
    c.part4 = (double *)(a + lay.part4);
    c.solid = h->solid.empty() ? nullptr : (uint8_t *)(a + lay.solid);
    c.solid_list = (int32_t *)(a + lay.solid_list);
    c.ctr = (DevCounters *)(a + lay.ctr);
    c.staging = a + lay.staging;
    c.staging_bytes = lay.staging_bytes;
    c.stream_bytes = kStreamingBytes;
    c.coll = AMR_COLLIDE_BGK;
    c.s_high = 1.0;
    c.stream = (hipStream_t)hip_stream;
    std::vector<int32_t> slist;
    for (int B = 0; B < (int)h->solid.size(); B++)
        if (h->solid[B]) slist.push_back(B);
    c.n_solid = (int)slist.size();
    const double tau0 = 0.5 + 3.0 * cfg->nu0;
    for (int L = 0; L < kMaxLevels; L++) {
        h->tau[L] = 0.5 + std::ldexp(tau0 - 0.5, L);  // tau*_L = 1/2 + 2^L (tau*_0 - 1/2)
        h->par[L] = 0;
    }
    // level-0 launch order: the active root blocks along the Morton curve of
    // their root coordinates; the finer levels inherit it (child index =
    // Morton digit), so blocks processed together are spatial neighbours
    std::vector<int32_t> root_order;
    {
        std::vector<std::pair<uint64_t, int32_t>> keyed;
        for (int B = 0; B < nroot; B++) {
            if (!h->solid.empty() && h->solid[B]) continue;
            const uint32_t x[3] = {(uint32_t)(B % c.root[0]), (uint32_t)((B / c.root[0]) % c.root[1]),
                                   (uint32_t)(B / (c.root[0] * c.root[1]))};
            uint64_t key = 0;
            for (int bit = 0; bit < 21; bit++)
                for (int ax = 0; ax < c.dim; ax++) key |= (uint64_t)((x[ax] >> bit) & 1u) << (bit * c.dim + ax);
            keyed.push_back({key, B});
        }
        std::stable_sort(keyed.begin(), keyed.end(),
                         [](const std::pair<uint64_t, int32_t> &a, const std::pair<uint64_t, int32_t> &b) {
                             return a.first < b.first;
                         });
        for (auto &kv : keyed) root_order.push_back(kv.second);
    }
    // the fixed device array of amr_mass_mom_static, resolved once per GPU
    double *mass_chunks = nullptr;
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) e = mass_scratch(h->device, &mass_chunks);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.order, root_order.data(), root_order.size() * 4, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e == hipSuccess && !h->solid.empty()) {
        e = hipMemcpyAsync(c.solid, h->solid.data(), h->solid.size(), hipMemcpyHostToDevice, c.stream);
        if (e == hipSuccess && !slist.empty())
            e = hipMemcpyAsync(c.solid_list, slist.data(), slist.size() * 4, hipMemcpyHostToDevice, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(c.ctr, 0, sizeof(DevCounters), c.stream);
    if (e != hipSuccess) {
        delete h;
        return fail(AMR_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    launch_fill_rest(c);
    launch_force_reset(c);
    launch_init_mesh(c);
    s = sync_checked(h);
    if (s == AMR_OK) s = refresh_counts(h);
    if (s != AMR_OK) {
        delete h;
        return s;
    }
    *out = h;
    return AMR_OK;
}

amr_status amr_destroy(amr_t *h) {
    if (!h) return AMR_OK;
    hipStreamSynchronize(h->c.stream);
    drop_graphs(h);
    for (auto &t : h->timed) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    for (auto e : h->event_pool) hipEventDestroy(e);
    for (auto e : h->step_ev)
        if (e) hipEventDestroy(e);
    delete h;
    return AMR_OK;
}

amr_status lbm_step(amr_t *h, int32_t n, uint32_t flags) {
    if (!h) return fail(AMR_ERR_ARG, "handle is NULL");
    if (n < 0) return fail(AMR_ERR_ARG, "n_coarse_steps must be >= 0");
    h->profiling = (flags & AMR_PROFILE) != 0;
    const bool use_graph = (flags & AMR_USE_GRAPH) != 0 && !h->profiling;
    for (int32_t sidx = 0; sidx < n; sidx++) {
        if (use_graph) {
            const int p0 = h->par[0];
            if (!h->graph_ok) {
                // capture one coarse step for each parity of level 0; every level
                // other than 0 returns to its parity at the end of a coarse step
                for (int k = 0; k < 2; k++) {
                    hipGraph_t g;
                    HIP_TRY(hipStreamBeginCapture(h->c.stream, hipStreamCaptureModeThreadLocal));
                    step_level(h, 0);
                    HIP_TRY(hipStreamEndCapture(h->c.stream, &g));
                    hipError_t e = hipGraphInstantiate(&h->gexec[(p0 + k) & 1], g, nullptr, nullptr, 0);
                    hipGraphDestroy(g);
                    if (e != hipSuccess) {
                        drop_graphs(h);
                        return fail(AMR_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
                    }
                }
                h->graph_ok = true;
                // capturing advanced the host-side parities by two steps; level 0 is back
            }
            HIP_TRY(hipGraphLaunch(h->gexec[h->par[0]], h->c.stream));
            h->par[0] ^= 1;
        } else {
            step_level(h, 0);
        }
    }
    HIP_TRY(hipGetLastError());
    if (h->force_on)
        for (int L = 0; L < h->lmax; L++) h->force_sweeps[L] += (double)n * (double)(1 << L);
    if (h->profiling) {
        amr_status ps = collect_timings(h);
        h->profiling = false;
        if (ps != AMR_OK) return ps;
    }
    if (flags & AMR_CHECK_FINITE) {
        launch_mass(h->c, level_params(h));
        double mass[4];
        HIP_TRY(hipMemcpyAsync(mass, h->c.ctr->mass, sizeof(mass), hipMemcpyDeviceToHost, h->c.stream));
        HIP_TRY(hipStreamSynchronize(h->c.stream));
        for (int a = 0; a < 4; a++)
            if (!std::isfinite(mass[a])) return fail(AMR_ERR_UNSTABLE, "non-finite mass/momentum after lbm_step");
    }
    return AMR_OK;
}

// event k of the adaptation-step timings, recorded on the handle's stream
static amr_status mark(amr_handle *h, int k) {
    if (!h->step_ev[k]) HIP_TRY(hipEventCreate(&h->step_ev[k]));
    HIP_TRY(hipEventRecord(h->step_ev[k], h->c.stream));
    return AMR_OK;
}

// milliseconds between two recorded events (the stream has been synchronised)
static double between(const amr_handle *h, int a, int b) {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, h->step_ev[a], h->step_ev[b]) == hipSuccess ? double(ms) : 0.0;
}

amr_status amr_tag(amr_t *h, const amr_tag_params *p, const int8_t *tags_in, int8_t *tags_out) {
    if (!h) return fail(AMR_ERR_ARG, "handle is NULL");
    if (!tags_in && !p) return fail(AMR_ERR_ARG, "criterion parameters are NULL");
    if (!tags_in && p->kind != AMR_TAG_VORTICITY_REL && p->kind != AMR_TAG_DISTANCE && p->kind != AMR_TAG_LADDER)
        return fail(AMR_ERR_ARG, "unknown criterion kind %d", p->kind);
    if (!tags_in && p->kind == AMR_TAG_LADDER && !(std::isfinite(p->n_start) && std::isfinite(p->n_inc)))
        return fail(AMR_ERR_ARG, "n_start and n_inc must be finite");
    Ctx &c = h->c;
    const size_t cap = (size_t)c.m.cap;
    amr_status ms;
    if ((ms = mark(h, 0)) != AMR_OK) return ms;
    // pre-adaptation synchronisation.  With the vorticity criterion the
    // averaging, which reads every child, also writes the velocities of the
    // children whose cells the ghost interpolation below leaves alone; the
    // velocity pass then covers level 0 and the rest.
    const bool vort = !tags_in && (p->kind == AMR_TAG_VORTICITY_REL || p->kind == AMR_TAG_LADDER);
    const bool averaged = vort && h->sync_velocity;
    for (int L = h->lmax - 2; L >= 0; L--)
        launch_average(c, c.refl + L * cap, h->nref[L], level_params(h), 1, averaged ? c.U : nullptr);
    if ((ms = mark(h, 1)) != AMR_OK) return ms;
    for (int L = 0; L <= h->lmax - 2; L++)
        if (h->niface[L] > 0) launch_interp(c, c.iface + L * cap, h->niface[L], level_params(h), 0);
    if ((ms = mark(h, 2)) != AMR_OK) return ms;
    launch_crit_reset(c);
    if (tags_in) {
        HIP_TRY(hipMemcpyAsync(c.m.tag, tags_in, cap, hipMemcpyHostToDevice, c.stream));
    } else if (p->kind == AMR_TAG_VORTICITY_REL || p->kind == AMR_TAG_LADDER) {
        const LevelParams lp = level_params(h);
        for (int L = 0; L < h->lmax; L++) {
            if (averaged && L > 0)
                launch_velocity(c, c.iface + (L - 1) * cap, h->niface[L - 1], L, lp, true);
            else
                launch_velocity(c, c.ids + L * cap, h->nids[L], L, lp);
        }
        for (int L = 0; L < h->lmax; L++) launch_vorticity(c, c.ids + L * cap, h->nids[L], L, lp);
        if (p->kind == AMR_TAG_LADDER) {
            LadderParams lad;
            lad.scale = 4.0 * c.root[0];  // domain length along x in root cells
            for (int k = 0; k < kMaxLevels; k++) {
                const double t = p->n_start - k * p->n_inc;
                lad.thr[k] = t > 1.0 ? INFINITY : std::exp2(t);
            }
            launch_tag_vorticity(c, p->theta, &lad);
        } else {
            launch_tag_vorticity(c, p->theta, nullptr);
        }
    } else {
        launch_tag_distance(c, p->d_spec, p->freeze);
    }
    launch_effective_tags(c);
    if ((ms = mark(h, 3)) != AMR_OK) return ms;
    if (tags_out) HIP_TRY(hipMemcpyAsync(tags_out, c.m.tag, cap, hipMemcpyDeviceToHost, c.stream));
    const amr_status s = sync_checked(h);
    if (s != AMR_OK) return s;
    for (int k = 0; k < 3; k++) h->step_ms[AMR_T_SYNC_AVERAGE + k] = between(h, k, k + 1);
    return AMR_OK;
}

amr_status amr_adapt(amr_t *h, amr_adapt_stats *stats) {
    if (!h) return fail(AMR_ERR_ARG, "handle is NULL");
    Ctx &c = h->c;
    amr_status s;
    if ((s = mark(h, 4)) != AMR_OK) return s;
    launch_effective_tags(c);
    if ((s = mark(h, 5)) != AMR_OK) return s;
    DevCounters dc;
    s = read_counters(h, &dc);
    if (s != AMR_OK) return s;
    const int n_ref = dc.n_ref, n_coa = dc.n_coa;
    for (int k = AMR_T_PREP; k < AMR_T_STEPS; k++) h->step_ms[k] = 0.0;
    h->step_ms[AMR_T_PREP] = between(h, 4, 5);
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->n_free = dc.gtop;
        for (int L = 0; L < h->lmax; L++) stats->level_blocks[L] = h->nids[L];
        for (int k = 0; k < AMR_T_STEPS; k++) stats->step_ms[k] = h->step_ms[k];
    }
    if (n_ref == 0 && n_coa == 0) return AMR_OK;
    if ((long long)c.nc * n_ref > dc.gtop)
        return fail(AMR_ERR_CAPACITY, "%d refinements need %d free block IDs, %d left", n_ref, c.nc * n_ref, dc.gtop);
    const LevelParams lp = level_params(h);
    // blocks are created and removed: the momentum-exchange sums restart
    launch_force_reset(c);
    for (int L = 0; L < kMaxLevels; L++) h->force_sweeps[L] = 0.0;
    if ((s = mark(h, 6)) != AMR_OK) return s;
    launch_adapt_assign(c, n_ref);
    if ((s = mark(h, 7)) != AMR_OK) return s;
    launch_adapt_build(c, n_ref);
    if ((s = mark(h, 8)) != AMR_OK) return s;
    launch_connectivity(c, c.m.cap);
    if ((s = mark(h, 9)) != AMR_OK) return s;
    // S7: every cell of the new children from their parents' data; after the
    // connectivity rebuild, since populations are stored by their source cell
    if (n_ref > 0) {
        launch_interp(c, c.rlist, n_ref, lp, 1);
        launch_refresh_neighbours(c, c.rlist, n_ref, lp);
    }
    if ((s = mark(h, 10)) != AMR_OK) return s;
    s = sync_checked(h);
    if (s != AMR_OK) return s;
    for (int k = 0; k < 4; k++) h->step_ms[AMR_T_ASSIGN + k] = between(h, 6 + k, 7 + k);
    s = read_counters(h, &dc);
    if (s != AMR_OK) return s;
    s = refresh_counts(h);
    if (s != AMR_OK) return s;
    drop_graphs(h);
    if (stats) {
        stats->n_refine = n_ref;
        stats->n_coarsen = dc.n_coa;
        stats->n_reverted = dc.n_rev;
        stats->n_free = dc.gtop;
        for (int L = 0; L < h->lmax; L++) stats->level_blocks[L] = h->nids[L];
        for (int k = 0; k < AMR_T_STEPS; k++) stats->step_ms[k] = h->step_ms[k];
    }
    return AMR_OK;
}

amr_status amr_set_collision(amr_t *h, int32_t kind, double s_high) {
    if (!h) return fail(AMR_ERR_ARG, "handle is NULL");
    if (kind == AMR_COLLIDE_BGK) {
        if (h->c.coll != AMR_COLLIDE_BGK) {
            h->c.coll = AMR_COLLIDE_BGK;
            drop_graphs(h);
        }
        return AMR_OK;
    }
    if (kind != AMR_COLLIDE_MRT && kind != AMR_COLLIDE_MRT_MFMA)
        return fail(AMR_ERR_ARG, "unknown collision kind %d", kind);
    if (h->c.q != 27) return fail(AMR_ERR_ARG, "the moment-space collision is implemented for D3Q27 only");
    if (kind == AMR_COLLIDE_MRT_MFMA && h->c.storage == AMR_F64)
        return fail(AMR_ERR_ARG, "AMR_COLLIDE_MRT_MFMA needs a storage with FP32 arithmetic");
    if (!(s_high > 0.0 && s_high < 2.0)) return fail(AMR_ERR_ARG, "s_high must lie in (0, 2), not %g", s_high);
    if (h->batches > 0) return fail(AMR_ERR_ARG, "the handle is in a batch, which advances BGK members only");
    if (kind != h->c.coll || s_high != h->c.s_high) {
        h->c.coll = kind;
        h->c.s_high = s_high;
        drop_graphs(h);  // captured steps hold the collide kernels and the rate
    }
    return AMR_OK;
}

amr_status amr_mass_mom_static(amr_t *h, double *out_dev) {
    if (!h) return fail(AMR_ERR_ARG, "handle is NULL");
    if (!out_dev) return fail(AMR_ERR_ARG, "out_dev is NULL");
    if ((int64_t)h->c.m.cap > mass_static_max_blocks())
        return fail(AMR_ERR_CAPACITY, "amr_mass_mom_static serves meshes of at most %lld blocks, this one has %d",
                    (long long)mass_static_max_blocks(), h->c.m.cap);
    double *chunks = nullptr;
    HIP_TRY(mass_scratch(h->device, &chunks));
    launch_mass_static(h->c, level_params(h), chunks, out_dev);
    HIP_TRY(hipGetLastError());
    return AMR_OK;
}

amr_status amr_fields(amr_t *h, int32_t op, int32_t kind, int32_t sim, void *buf, uint64_t bytes) {
    if (!h) return fail(AMR_ERR_ARG, "handle is NULL");
    if (sim != 0) return fail(AMR_ERR_ARG, "sim must be 0");
    if (op != AMR_GET && op != AMR_SET) return fail(AMR_ERR_ARG, "op must be AMR_GET or AMR_SET");
    if (op == AMR_SET && kind == AMR_FIELD_KERNEL_STATS) {
        memset(h->kstats, 0, sizeof(h->kstats));
        return AMR_OK;
    }
    if (kind == AMR_FIELD_FORCE_ON) {
        if (!buf || bytes < 4) return fail(AMR_ERR_ARG, "AMR_FIELD_FORCE_ON needs an int32 buffer");
        int32_t *v = (int32_t *)buf;
        if (op == AMR_GET) {
            *v = h->force_on ? 1 : 0;
            return AMR_OK;
        }
        if (*v != 0 && *v != 1) return fail(AMR_ERR_ARG, "AMR_FIELD_FORCE_ON takes 0 or 1, not %d", *v);
        if ((*v == 1) != h->force_on) {
            h->force_on = *v == 1;
            drop_graphs(h);  // captured steps hold the exchange launches, or not
        }
        return AMR_OK;
    }
    if (kind == AMR_FIELD_SYNC_VELOCITY) {
        if (!buf || bytes < 4) return fail(AMR_ERR_ARG, "AMR_FIELD_SYNC_VELOCITY needs an int32 buffer");
        int32_t *v = (int32_t *)buf;
        if (op == AMR_GET) {
            *v = h->sync_velocity ? 1 : 0;
            return AMR_OK;
        }
        if (*v != 0 && *v != 1) return fail(AMR_ERR_ARG, "AMR_FIELD_SYNC_VELOCITY takes 0 or 1, not %d", *v);
        h->sync_velocity = *v == 1;
        return AMR_OK;
    }
    if (kind == AMR_FIELD_SKIP_PARENTS) {
        if (!buf || bytes < 4) return fail(AMR_ERR_ARG, "AMR_FIELD_SKIP_PARENTS needs an int32 buffer");
        int32_t *v = (int32_t *)buf;
        if (op == AMR_GET) {
            *v = h->skip_parents ? 1 : 0;
            return AMR_OK;
        }
        if (*v != 0 && *v != 1) return fail(AMR_ERR_ARG, "AMR_FIELD_SKIP_PARENTS takes 0 or 1, not %d", *v);
        if (*v == 1 && h->c.m.interp != AMR_INTERP_LINEAR)
            return fail(AMR_ERR_ARG, "AMR_FIELD_SKIP_PARENTS needs linear interpolation (cubic stencils reach "
                                     "into neighbouring parents)");
        if ((*v == 1) != h->skip_parents) {
            h->skip_parents = *v == 1;
            drop_graphs(h);  // captured steps hold the sweep lists' counts
        }
        return AMR_OK;
    }
    if (kind == AMR_FIELD_STREAM_BYTES) {
        if (!buf || bytes < 8) return fail(AMR_ERR_ARG, "AMR_FIELD_STREAM_BYTES needs an int64 buffer");
        int64_t *v = (int64_t *)buf;
        if (op == AMR_GET) {
            *v = h->c.stream_bytes;
            return AMR_OK;
        }
        if (*v < 0) return fail(AMR_ERR_ARG, "AMR_FIELD_STREAM_BYTES must be >= 0, not %lld", (long long)*v);
        if (*v != h->c.stream_bytes) {
            h->c.stream_bytes = *v;
            drop_graphs(h);  // captured steps hold the store policy of each launch
        }
        return AMR_OK;
    }
    if (op == AMR_SET && kind == AMR_FIELD_FORCE) {
        launch_force_reset(h->c);
        for (int L = 0; L < kMaxLevels; L++) h->force_sweeps[L] = 0.0;
        return sync_checked(h);
    }
    if (op == AMR_SET && kind != AMR_FIELD_RHO_U && kind != AMR_FIELD_BLOCK_F)
        return fail(AMR_ERR_ARG, "kind %d cannot be set", kind);
    Ctx &c = h->c;
    const size_t cap = (size_t)c.m.cap;
    const int q = c.q, mb = c.mb, nb = c.nb;
    hipStream_t st = c.stream;
    auto need = [&](uint64_t n) -> amr_status {
        if (!buf && n > 0) return fail(AMR_ERR_ARG, "buffer is NULL");
        if (bytes < n) return fail(AMR_ERR_ARG, "buffer of %llu bytes is too small: %llu bytes required",
                                   (unsigned long long)bytes, (unsigned long long)n);
        return AMR_OK;
    };
    amr_status s;
    const LevelParams lp = level_params(h);
    switch (kind) {
    case AMR_FIELD_N_OUT:
    case AMR_FIELD_CELLS:
    case AMR_FIELD_F:
    case AMR_FIELD_RHO_U: {
        if (kind == AMR_FIELD_RHO_U && op == AMR_SET) {
            const int64_t ncell = (int64_t)c.nroot * mb;
            if ((s = need((uint64_t)ncell * 32)) != AMR_OK) return s;
            const int per = (int)(c.staging_bytes / (32 * (size_t)mb));
            for (int b0 = 0; b0 < c.nroot; b0 += per) {
                const int b1 = b0 + per < c.nroot ? b0 + per : c.nroot;
                HIP_TRY(hipMemcpyAsync(c.staging, (const char *)buf + (size_t)b0 * mb * 32, (size_t)(b1 - b0) * mb * 32,
                                       hipMemcpyHostToDevice, st));
                launch_set_rho_u_root(c, (const double *)c.staging, b0, b1);
                HIP_TRY(hipStreamSynchronize(st));
            }
            drop_graphs(h);
            return sync_checked(h);
        }
        launch_out_count(c);
        DevCounters dc;
        if ((s = read_counters(h, &dc)) != AMR_OK) return s;
        const int64_t n_out = dc.n_out;
        if (kind == AMR_FIELD_N_OUT) {
            if ((s = need(8)) != AMR_OK) return s;
            memcpy(buf, &n_out, 8);
            return AMR_OK;
        }
        const size_t row = kind == AMR_FIELD_CELLS ? 8 : (kind == AMR_FIELD_RHO_U ? 32 : (size_t)q * 8);
        if ((s = need((uint64_t)n_out * row)) != AMR_OK) return s;
        std::vector<int32_t> off(cap + 1);
        HIP_TRY(hipMemcpyAsync(off.data(), c.off, cap * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        off[cap] = (int32_t)n_out;
        const int per_blocks = (int)(c.staging_bytes / (row * mb));
        for (int b0 = 0; b0 < (int)cap; b0 += per_blocks) {
            const int b1 = b0 + per_blocks < (int)cap ? b0 + per_blocks : (int)cap;
            const int64_t rows = off[b1] - off[b0];
            if (rows == 0) continue;
            launch_out_gather(c, kind, b0, b1, off[b0], c.staging, lp);
            HIP_TRY(hipMemcpyAsync((char *)buf + (size_t)off[b0] * row, c.staging, rows * row,
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        return sync_checked(h);
    }
    case AMR_FIELD_BLOCK_F: {
        const size_t row = (size_t)mb * q * 8;
        if ((s = need(cap * row)) != AMR_OK) return s;
        const int per_blocks = (int)(c.staging_bytes / row);
        for (int b0 = 0; b0 < (int)cap; b0 += per_blocks) {
            const int b1 = b0 + per_blocks < (int)cap ? b0 + per_blocks : (int)cap;
            char *hb = (char *)buf + (size_t)b0 * row;
            const size_t nbytes = (size_t)(b1 - b0) * row;
            if (op == AMR_SET) HIP_TRY(hipMemcpyAsync(c.staging, hb, nbytes, hipMemcpyHostToDevice, st));
            launch_block_f(c, op == AMR_SET, b0, b1, (double *)c.staging, lp);
            if (op == AMR_GET) HIP_TRY(hipMemcpyAsync(hb, c.staging, nbytes, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        return sync_checked(h);
    }
    case AMR_FIELD_LEVEL:
    case AMR_FIELD_STATUS: {
        if ((s = need(cap)) != AMR_OK) return s;
        HIP_TRY(hipMemcpyAsync(buf, kind == AMR_FIELD_LEVEL ? (void *)c.m.level : (void *)c.m.status, cap,
                               hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_COORD: {
        if ((s = need(cap * 12)) != AMR_OK) return s;
        HIP_TRY(hipMemcpyAsync(buf, c.m.X, cap * 12, hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_NBR:
    case AMR_FIELD_NBR_CHILD: {
        if ((s = need(cap * nb * 4)) != AMR_OK) return s;
        HIP_TRY(hipMemcpyAsync(buf, kind == AMR_FIELD_NBR ? c.m.nbr : c.m.nbrc, cap * nb * 4, hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_IDSET: {
        const size_t lmax = (size_t)h->lmax;
        if ((s = need((lmax + lmax * cap) * 4)) != AMR_OK) return s;
        int32_t *o = (int32_t *)buf;
        for (size_t L = 0; L < lmax; L++) o[L] = h->nids[L];
        HIP_TRY(hipMemcpyAsync(o + lmax, c.ids, lmax * cap * 4, hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_GAP: {
        if ((s = need((1 + cap) * 4)) != AMR_OK) return s;
        int32_t *o = (int32_t *)buf;
        o[0] = h->gtop;
        if (h->gtop > 0) HIP_TRY(hipMemcpyAsync(o + 1, c.gap, (size_t)h->gtop * 4, hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_COUNTS: {
        if ((s = need((size_t)h->lmax * 4)) != AMR_OK) return s;
        memcpy(buf, h->nids, (size_t)h->lmax * 4);
        return AMR_OK;
    }
    case AMR_FIELD_MASS_MOM: {
        if ((s = need(32)) != AMR_OK) return s;
        launch_mass(c, lp);
        HIP_TRY(hipMemcpyAsync(buf, c.ctr->mass, 32, hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_CRIT: {
        if ((s = need(cap * 8)) != AMR_OK) return s;
        HIP_TRY(hipMemcpyAsync(buf, c.crit, cap * 8, hipMemcpyDeviceToHost, st));
        return sync_checked(h);
    }
    case AMR_FIELD_KERNEL_STATS: {
        if ((s = need(sizeof(h->kstats))) != AMR_OK) return s;
        memcpy(buf, h->kstats, sizeof(h->kstats));
        return AMR_OK;
    }
    case AMR_FIELD_PARITY: {
        if ((s = need((size_t)h->lmax * 4)) != AMR_OK) return s;
        memcpy(buf, h->par, (size_t)h->lmax * 4);
        return AMR_OK;
    }
    case AMR_FIELD_FORCE: {
        if ((s = need((size_t)h->lmax * 4 * 8)) != AMR_OK) return s;
        double *dev = (double *)c.staging;  // >= 1 MB
        launch_force_sum(c, dev);
        std::vector<double> tot((size_t)h->lmax * 3);
        HIP_TRY(hipMemcpyAsync(tot.data(), dev, tot.size() * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double *out = (double *)buf;
        for (int L = 0; L < h->lmax; L++) {
            for (int a = 0; a < 3; a++) out[L * 4 + a] = tot[(size_t)L * 3 + a];
            out[L * 4 + 3] = h->force_sweeps[L];
        }
        return AMR_OK;
    }
    default:
        return fail(AMR_ERR_ARG, "unknown field kind %d", kind);
    }
}

}  // extern "C"
