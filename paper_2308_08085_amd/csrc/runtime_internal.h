// runtime_internal.h -- state shared by the host runtime files (single
// simulations in runtime.hip, batches in batch.hip): the handle behind amr_t,
// its arena layout, error reporting.
#pragma once

#include <string>
#include <vector>

#include "../../include/amr_lbm.h"
#include "kernels.h"

namespace amr {

// record a message for amr_last_error() and return `code`
amr_status fail(amr_status code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(AMR_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t f[2], nbr, nbrc, X, level, status, tag, ldes, viol, bflag, gmask, imask;
    size_t ids, ids_tmp, iface, refl, sweep, order, force, solidl, gap, first, rlist, clist, cnt, off, rank, bins, scan_part;
    size_t crit, part4, solid, solid_list, ctr, staging, staging_bytes, total, hid, U, parent, fresh;
};

}  // namespace amr

using namespace amr;

struct amr_handle {
    amr_config cfg;
    Ctx c;
    Layout lay;
    int lmax;
    int device;  // the GPU current at creation
    int nids[kMaxLevels], niface[kMaxLevels], nsolid[kMaxLevels], nref[kMaxLevels], nsweep[kMaxLevels];
    double ghost_w[kMaxLevels], avg_w[kMaxLevels];  // cells the grid communication of each level moves
    int gtop;
    int par[kMaxLevels];
    double force_sweeps[kMaxLevels] = {0};  // collide-stream sweeps per level since the force reset
    bool force_on = true;                   // accumulate the momentum exchange every sweep
    bool sync_velocity = true;              // criterion velocities from the synchronisation's averaging
    bool skip_parents = false;              // sweeps leave out refined blocks without N_SKIP children
    int batches = 0;                        // batches this handle is a member of
    double tau[kMaxLevels];
    BCParams bc;
    std::vector<uint8_t> solid;
    // graph of one coarse step, per level-0 parity
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool graph_ok = false;
    // AMR_PROFILE: events around each solver launch (kind, start, stop, blocks, bytes)
    bool profiling = false;
    struct Timed { int kind; hipEvent_t a, b; double blocks, bytes; };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    double kstats[3][4] = {{0}};
    // device times of the adaptation steps (amr_adapt_step order): events at
    // the step boundaries, read after the stream synchronisations the calls
    // make anyway; the first three are those of the last amr_tag
    hipEvent_t step_ev[11] = {nullptr};  // tag: 0-3; adapt: 4-5 (prep), 6-10 (S2 ... S7)
    double step_ms[AMR_T_STEPS] = {0};
};

namespace amr {

// relaxation and rescaling of every level, with the current buffer parities
LevelParams level_params(const amr_handle *h);


}  // namespace amr
