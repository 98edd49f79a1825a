// batch.hip -- many independent simulations advanced together.  Simulations
// are grouped by (lattice, storage); each group advances every level sweep of
// all its members in one persistent launch (collide-stream, ghost
// interpolation, interface averaging), with the work items rebuilt on the
// device from each member's own lists at the start of every coarse step, so a
// captured coarse step stays valid while members adapt.  An autotuner picks
// the workgroup shape, the persistent grid size and whether the groups run as
// concurrent branches of the graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime_internal.h"

namespace {

struct Group {
    int q = 0, storage = 0, lmax = 0, cap_max = 0;
    bool solid = false;        // some member has solid root blocks
    std::vector<int> members;  // indices into amr_batch::sims, in batch order
    std::vector<bool> force_on;  // each member's momentum-exchange switch in the uploaded descriptors
    SimDesc *desc = nullptr;   // device [members]
    uint32_t *items = nullptr; // device [3 lmax][stride]
    int32_t *counts = nullptr; // device [3 lmax]
    int64_t stride = 0;        // sum of the members' capacities
    size_t off_desc = 0, off_items = 0, off_counts = 0;
};

int sim_lmax(const amr_t *h) { return h->lmax; }

// groups in order of first appearance; arena offsets of their buffers
size_t plan_groups(amr_t *const *sims, int n, std::vector<Group> &groups) {
    groups.clear();
    for (int i = 0; i < n; i++) {
        const amr_t *h = sims[i];
        Group *g = nullptr;
        for (auto &x : groups)
            if (x.q == h->c.q && x.storage == h->c.storage) g = &x;
        if (!g) {
            groups.emplace_back();
            g = &groups.back();
            g->q = h->c.q;
            g->storage = h->c.storage;
        }
        g->members.push_back(i);
        g->solid = g->solid || h->c.n_solid > 0;
        g->lmax = std::max(g->lmax, sim_lmax(h));
        g->cap_max = std::max(g->cap_max, h->c.m.cap);
        g->stride += h->c.m.cap;
    }
    size_t t = 0;
    auto take = [&](size_t bytes) {
        size_t o = align256(t);
        t = o + bytes;
        return o;
    };
    for (auto &g : groups) {
        g.off_desc = take(g.members.size() * sizeof(SimDesc));
        g.off_items = take((size_t)3 * g.lmax * g.stride * sizeof(uint32_t));
        g.off_counts = take((size_t)3 * g.lmax * sizeof(int32_t));
    }
    return align256(t);
}

}  // namespace

struct amr_batch {
    std::vector<amr_t *> sims;
    std::vector<Group> groups;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> side;  // one per group after the first (concurrent schedule)
    std::vector<hipEvent_t> ev;     // fork + one join per side stream
    int par0 = 0;                   // level-0 buffer parity shared by every member
    int n_cu = 256;
    amr_batch_tuning tune;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool graph_ok = false;
};

namespace {

amr_status validate_members(amr_t *const *sims, int n, void *stream) {
    if (!sims || n < 1) return fail(AMR_ERR_ARG, "a batch needs at least one simulation");
    for (int i = 0; i < n; i++) {
        const amr_t *h = sims[i];
        if (!h) return fail(AMR_ERR_ARG, "simulation %d is NULL", i);
        if (h->c.coll != AMR_COLLIDE_BGK)
            return fail(AMR_ERR_ARG, "simulation %d uses a moment-space collision; batches advance BGK members only", i);
        for (int j = 0; j < i; j++)
            if (sims[j] == h) return fail(AMR_ERR_ARG, "simulation %d appears twice", i);
        if (h->c.stream != (hipStream_t)stream)
            return fail(AMR_ERR_ARG, "simulation %d was created on another stream", i);
        if ((uint32_t)h->c.m.cap > kItemBlockMask + 1u)
            return fail(AMR_ERR_ARG, "simulation %d: max_blocks above %u", i, kItemBlockMask + 1u);
        if (h->par[0] != sims[0]->par[0])
            return fail(AMR_ERR_STATE, "simulation %d is at another level-0 buffer parity (odd vs even "
                                       "number of coarse steps)", i);
        for (int L = 1; L < h->lmax; L++)
            if (h->par[L] != 0) return fail(AMR_ERR_STATE, "simulation %d is inside a coarse step", i);
    }
    std::vector<Group> groups;
    plan_groups(sims, n, groups);
    for (auto &g : groups)
        if ((int)g.members.size() > kMaxBatchSims)
            return fail(AMR_ERR_ARG, "more than %d simulations of one lattice and storage", kMaxBatchSims);
    return AMR_OK;
}

SimDesc make_desc(const amr_t *h) {
    SimDesc d;
    std::memset(&d, 0, sizeof(d));
    d.m = h->c.m;
    d.f[0] = h->c.f[0];
    d.f[1] = h->c.f[1];
    d.lp = level_params(h);
    d.bc = h->bc;
    d.order = h->c.order;
    d.iface = h->c.iface;
    d.solid = h->c.solidl;
    d.nids = h->c.ctr->nids;
    d.niface = h->c.ctr->niface;
    d.nsolid = h->c.ctr->nsolid;
    d.force_on = h->force_on ? 1 : 0;
    return d;
}

int collide_grid(const amr_batch *b) { return std::max(1, b->tune.wg_per_cu * b->n_cu); }

// one coarse step of one group: step(L) = ghost fill of L+1, collide-stream
// of L, step(L+1) twice, interface averaging of L+1 into L
void group_level(const amr_batch *b, const Group &g, hipStream_t st, int L, int *par) {
    if (L >= g.lmax) return;
    const int grid = collide_grid(b);
    const bool finer = L + 1 < g.lmax;
    const int64_t s = g.stride;
    if (finer)
        launch_interp_batch(st, g.q, g.storage, g.desc, g.items + (3 * L + 1) * s, g.counts + 3 * L + 1, L, par[L],
                            par[L + 1], grid);
    launch_collide_batch(st, g.q, g.storage, g.desc, g.items + (3 * L) * s, g.counts + 3 * L, L, par[L],
                         b->tune.threads, grid);
    par[L] ^= 1;
    if (g.solid)  // momentum exchange with solid blocks, from the buffer just written
        launch_exchange_batch(st, g.q, g.storage, g.desc, g.items + (3 * L + 2) * s, g.counts + 3 * L + 2, par[L],
                              std::max(1, b->n_cu));
    if (finer) {
        group_level(b, g, st, L + 1, par);
        group_level(b, g, st, L + 1, par);
        launch_average_batch(st, g.q, g.storage, g.desc, g.items + (3 * L + 1) * s, g.counts + 3 * L + 1, L, par[L],
                             par[L + 1], grid);
    }
}

void group_step(const amr_batch *b, const Group &g, hipStream_t st, int par0) {
    launch_batch_items(st, g.desc, (int)g.members.size(), g.lmax, g.cap_max, g.items, g.stride, g.counts);
    int par[kMaxLevels] = {0};
    par[0] = par0;
    group_level(b, g, st, 0, par);
}

// one coarse step of the batch on b->stream (eager or under capture)
amr_status batch_coarse_step(amr_batch *b, int par0) {
    const bool concurrent = b->tune.schedule == 1 && b->groups.size() > 1;
    if (!concurrent) {
        for (auto &g : b->groups) group_step(b, g, b->stream, par0);
        return AMR_OK;
    }
    HIP_TRY(hipEventRecord(b->ev[0], b->stream));
    for (size_t k = 1; k < b->groups.size(); k++) {
        HIP_TRY(hipStreamWaitEvent(b->side[k - 1], b->ev[0], 0));
        group_step(b, b->groups[k], b->side[k - 1], par0);
        HIP_TRY(hipEventRecord(b->ev[k], b->side[k - 1]));
    }
    group_step(b, b->groups[0], b->stream, par0);
    for (size_t k = 1; k < b->groups.size(); k++) HIP_TRY(hipStreamWaitEvent(b->stream, b->ev[k], 0));
    return AMR_OK;
}

void drop_batch_graphs(amr_batch *b) {
    for (int i = 0; i < 2; i++)
        if (b->gexec[i]) {
            hipGraphExecDestroy(b->gexec[i]);
            b->gexec[i] = nullptr;
        }
    b->graph_ok = false;
}

void set_member_parity(amr_batch *b) {
    for (auto *h : b->sims) h->par[0] = b->par0;
}

void count_member_sweeps(amr_batch *b, int32_t n) {
    for (auto *h : b->sims)
        if (h->force_on)
            for (int L = 0; L < h->lmax; L++) h->force_sweeps[L] += (double)n * (double)(1 << L);
}

// A member whose momentum-exchange switch changed since its descriptor was
// uploaded gets its group's descriptors again (the work lists are built from
// them on the device, so captured steps stay valid).
amr_status refresh_descs(amr_batch *b) {
    for (auto &g : b->groups) {
        bool stale = false;
        for (size_t k = 0; k < g.members.size(); k++)
            stale = stale || g.force_on[k] != b->sims[g.members[k]]->force_on;
        if (!stale) continue;
        std::vector<SimDesc> host;
        for (size_t k = 0; k < g.members.size(); k++) {
            host.push_back(make_desc(b->sims[g.members[k]]));
            g.force_on[k] = b->sims[g.members[k]]->force_on;
        }
        HIP_TRY(hipMemcpyAsync(g.desc, host.data(), host.size() * sizeof(SimDesc), hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
    }
    return AMR_OK;
}

amr_status run_steps(amr_batch *b, int32_t n, bool use_graph) {
    for (int32_t k = 0; k < n; k++) {
        if (use_graph) {
            if (!b->graph_ok) {
                for (int p = 0; p < 2; p++) {
                    hipGraph_t g;
                    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                    amr_status s = batch_coarse_step(b, p);
                    hipError_t e = hipStreamEndCapture(b->stream, &g);
                    if (s != AMR_OK) return s;
                    if (e != hipSuccess) return fail(AMR_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
                    e = hipGraphInstantiate(&b->gexec[p], g, nullptr, nullptr, 0);
                    hipGraphDestroy(g);
                    if (e != hipSuccess) {
                        drop_batch_graphs(b);
                        return fail(AMR_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
                    }
                }
                b->graph_ok = true;
            }
            HIP_TRY(hipGraphLaunch(b->gexec[b->par0], b->stream));
        } else {
            amr_status s = batch_coarse_step(b, b->par0);
            if (s != AMR_OK) return s;
        }
        b->par0 ^= 1;
    }
    set_member_parity(b);
    count_member_sweeps(b, n);
    HIP_TRY(hipGetLastError());
    return AMR_OK;
}

amr_status check_tuning(const amr_batch_tuning *t) {
    if (!t) return fail(AMR_ERR_ARG, "tuning is NULL");
    if (t->threads != 64 && t->threads != 128 && t->threads != 256)
        return fail(AMR_ERR_ARG, "threads must be 64, 128 or 256");
    if (t->wg_per_cu < 1 || t->wg_per_cu > 64) return fail(AMR_ERR_ARG, "wg_per_cu must be in [1, 64]");
    if (t->schedule != 0 && t->schedule != 1) return fail(AMR_ERR_ARG, "schedule must be 0 or 1");
    return AMR_OK;
}

}  // namespace

extern "C" {

amr_status amr_batch_query_bytes(amr_t *const *sims, int32_t n, uint64_t *arena_bytes) {
    if (!arena_bytes) return fail(AMR_ERR_ARG, "arena_bytes is NULL");
    if (!sims || n < 1) return fail(AMR_ERR_ARG, "a batch needs at least one simulation");
    for (int i = 0; i < n; i++)
        if (!sims[i]) return fail(AMR_ERR_ARG, "simulation %d is NULL", i);
    std::vector<Group> groups;
    *arena_bytes = plan_groups(sims, n, groups);
    return AMR_OK;
}

amr_status amr_batch_create(amr_t *const *sims, int32_t n, void *dev_arena, uint64_t arena_bytes, void *hip_stream,
                            amr_batch_t **out) {
    if (!out) return fail(AMR_ERR_ARG, "out is NULL");
    amr_status s = validate_members(sims, n, hip_stream);
    if (s != AMR_OK) return s;
    if (!dev_arena) return fail(AMR_ERR_ARG, "dev_arena is NULL");
    if (((uintptr_t)dev_arena & 255) != 0) return fail(AMR_ERR_ARG, "dev_arena must be 256-byte aligned");
    amr_batch *b = new amr_batch();
    const size_t need = plan_groups(sims, n, b->groups);
    if (arena_bytes < need) {
        delete b;
        return fail(AMR_ERR_CAPACITY, "arena of %llu bytes is smaller than the %llu bytes required",
                    (unsigned long long)arena_bytes, (unsigned long long)need);
    }
    b->sims.assign(sims, sims + n);
    for (int i = 0; i < n; i++) sims[i]->batches++;
    b->stream = (hipStream_t)hip_stream;
    b->par0 = sims[0]->par[0];
    b->tune.threads = 256;
    b->tune.wg_per_cu = 8;
    b->tune.schedule = 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        b->n_cu = std::max(1, prop.multiProcessorCount);
    char *a = (char *)dev_arena;
    hipError_t e = hipSuccess;
    for (auto &g : b->groups) {
        g.desc = (SimDesc *)(a + g.off_desc);
        g.items = (uint32_t *)(a + g.off_items);
        g.counts = (int32_t *)(a + g.off_counts);
        std::vector<SimDesc> host;
        for (int i : g.members) host.push_back(make_desc(sims[i]));
        for (int i : g.members) g.force_on.push_back(sims[i]->force_on);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g.desc, host.data(), host.size() * sizeof(SimDesc), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    for (size_t k = 0; e == hipSuccess && k < b->groups.size(); k++) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->ev.push_back(ev);
        if (e == hipSuccess && k > 0) {
            hipStream_t st;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e == hipSuccess) b->side.push_back(st);
        }
    }
    if (e != hipSuccess) {
        amr_batch_destroy(b);
        return fail(AMR_ERR_DEVICE, "batch set-up: %s", hipGetErrorString(e));
    }
    *out = b;
    return AMR_OK;
}

amr_status amr_batch_step(amr_batch_t *b, int32_t n, uint32_t flags) {
    if (!b) return fail(AMR_ERR_ARG, "batch is NULL");
    if (n < 0) return fail(AMR_ERR_ARG, "n_coarse_steps must be >= 0");
    if (flags & AMR_PROFILE) return fail(AMR_ERR_ARG, "AMR_PROFILE is not available for batches");
    for (auto *h : b->sims)
        if (h->par[0] != b->par0) return fail(AMR_ERR_STATE, "a member was stepped outside the batch");
    amr_status s = refresh_descs(b);
    if (s != AMR_OK) return s;
    s = run_steps(b, n, (flags & AMR_USE_GRAPH) != 0);
    if (s != AMR_OK) return s;
    if (flags & AMR_CHECK_FINITE) {
        int bad = -1;
        for (size_t i = 0; i < b->sims.size(); i++) {
            amr_t *h = b->sims[i];
            launch_mass(h->c, level_params(h));
            double mass[4];
            HIP_TRY(hipMemcpyAsync(mass, h->c.ctr->mass, sizeof(mass), hipMemcpyDeviceToHost, b->stream));
            HIP_TRY(hipStreamSynchronize(b->stream));
            for (int a = 0; a < 4; a++)
                if (!std::isfinite(mass[a]) && bad < 0) bad = (int)i;
        }
        if (bad >= 0) return fail(AMR_ERR_UNSTABLE, "non-finite mass/momentum in simulation %d", bad);
    }
    return AMR_OK;
}

amr_status amr_batch_set_tuning(amr_batch_t *b, const amr_batch_tuning *t) {
    if (!b) return fail(AMR_ERR_ARG, "batch is NULL");
    amr_status s = check_tuning(t);
    if (s != AMR_OK) return s;
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->tune = *t;
    drop_batch_graphs(b);
    return AMR_OK;
}

amr_status amr_batch_get_tuning(amr_batch_t *b, amr_batch_tuning *t) {
    if (!b || !t) return fail(AMR_ERR_ARG, "NULL argument");
    *t = b->tune;
    return AMR_OK;
}

amr_status amr_batch_autotune(amr_batch_t *b, int32_t trial_steps, amr_batch_tuning *best, double *best_ms) {
    if (!b) return fail(AMR_ERR_ARG, "batch is NULL");
    if (trial_steps < 1) return fail(AMR_ERR_ARG, "trial_steps must be >= 1");
    for (auto *h : b->sims)
        if (h->par[0] != b->par0) return fail(AMR_ERR_STATE, "a member was stepped outside the batch");
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    const int threads[3] = {64, 128, 256};
    const int wpc[4] = {2, 4, 8, 16};
    const int nsched = b->groups.size() > 1 ? 2 : 1;
    amr_batch_tuning top = b->tune;
    double top_ms = -1.0;
    amr_status s = AMR_OK;
    for (int sc = 0; sc < nsched && s == AMR_OK; sc++)
        for (int ti = 0; ti < 3 && s == AMR_OK; ti++)
            for (int wi = 0; wi < 4 && s == AMR_OK; wi++) {
                amr_batch_tuning c;
                c.threads = threads[ti];
                c.wg_per_cu = wpc[wi];
                c.schedule = sc;
                s = amr_batch_set_tuning(b, &c);
                if (s != AMR_OK) break;
                // the first step captures the graphs; time the replays only
                s = run_steps(b, 2, true);
                if (s != AMR_OK) break;
                if (hipEventRecord(t0, b->stream) != hipSuccess) { s = fail(AMR_ERR_DEVICE, "event record"); break; }
                s = run_steps(b, trial_steps, true);
                if (s != AMR_OK) break;
                float ms = 0.f;
                if (hipEventRecord(t1, b->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                    hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
                    s = fail(AMR_ERR_DEVICE, "event timing");
                    break;
                }
                const double per = ms / trial_steps;
                if (top_ms < 0.0 || per < top_ms) {
                    top_ms = per;
                    top = c;
                }
            }
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    if (s != AMR_OK) return s;
    s = amr_batch_set_tuning(b, &top);
    if (s != AMR_OK) return s;
    if (best) *best = top;
    if (best_ms) *best_ms = top_ms;
    return AMR_OK;
}

amr_status amr_batch_destroy(amr_batch_t *b) {
    if (!b) return AMR_OK;
    if (b->stream || !b->sims.empty()) hipStreamSynchronize(b->stream);
    drop_batch_graphs(b);
    for (auto st : b->side) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
    }
    for (auto ev : b->ev) hipEventDestroy(ev);
    for (auto h : b->sims) h->batches--;
    delete b;
    return AMR_OK;
}

}  // extern "C"
