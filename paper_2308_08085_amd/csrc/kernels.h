// kernels.h -- host-side launchers of the HIP kernels (implemented in
// lbm_kernels.hip and mesh_kernels.hip), called by the runtime.
#pragma once

#include "common.h"

namespace amr {

struct DevCounters {
    int32_t nids[kMaxLevels];
    int32_t niface[kMaxLevels];
    int32_t nsolid[kMaxLevels];
    int32_t nref[kMaxLevels];    // refined blocks per level (list refl)
    int32_t nsweep[kMaxLevels];  // blocks per level in the sweep list
    int32_t gtop;
    int32_t n_ref, n_coa, n_rev;
    int32_t nfreed;
    int32_t n_out;
    int32_t pad[2];
    unsigned long long wmax_bits;
    int32_t totals[kMaxLevels];
    int32_t bases[kMaxLevels];
    double mass[4];
    // cells the solver's grid communication moves from level L, per coarse
    // step of L: ghost cells its interpolation writes into level L+1, parent
    // cells its averaging writes (each from 2^d fine cells)
    unsigned long long ghost_w[kMaxLevels];
    unsigned long long avg_w[kMaxLevels];
};

// everything a launcher needs: device views and scratch carved from the arena
struct Ctx {
    DevMesh m;
    int dim, q, nb, mb, nc, storage;
    int nroot;
    int root[3];
    int periodic[3];
    int face_prio[6];
    int face_kind[6];
    void *f[2];
    int32_t *ids;        // [lmax][cap]
    int32_t *ids_tmp;    // [lmax][cap]
    int32_t *iface;      // [lmax][cap]
    int32_t *refl;       // [lmax][cap]: the refined blocks of each level (parents of the next)
    int32_t *sweep;      // [lmax][cap]: the launch order without refined blocks none of whose
                         // children has an N_SKIP link
    int32_t *order;      // [lmax][cap] solver launch order per level (Morton)
    int32_t *solidl;     // [lmax][cap] leaf blocks next to a solid block, per level
    int32_t *gap;        // [cap]
    int32_t *first;      // [cap]
    int32_t *rank;       // [lmax * cap]
    int32_t *rlist;      // [cap]
    int32_t *clist;      // [cap]
    int8_t *bins;        // [lmax * cap]
    int32_t *scan_part;  // [nwg_max * 8]
    int32_t *cnt;        // [cap]
    int32_t *off;        // [cap]
    double *crit;        // [cap]
    double *U;           // [3][cap * Mb] FP64 cell velocities for the criterion
    double *part4;       // [cap * 4]
    uint8_t *solid;      // [nroot]
    int32_t *solid_list; // [nroot]
    int32_t n_solid;
    DevCounters *ctr;
    void *staging;
    size_t staging_bytes;
    int64_t stream_bytes;  // sweeps writing more than this use non-temporal stores
    int coll;              // enum amr_collision of the collide-stream sweeps
    double s_high;         // moment-space collision: rate of the moments above second order
    hipStream_t stream;
};

// default of Ctx::stream_bytes: half the 256 MB Infinity Cache
constexpr int64_t kStreamingBytes = int64_t(128) << 20;

// ---- LBM kernels (lbm_kernels.hip) ----
// exchange: also add the momentum exchange with solid blocks (BGK sweeps with
// ordinary stores); returns whether it did, else launch_exchange follows
bool launch_collide_stream(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp,
                           const BCParams &bc, bool exchange = false);
// mode 0: ghost cells of children with an N_SKIP link; 1: every cell of every child
void launch_interp(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells);
// after new children (parents in `list`) were interpolated: the populations of
// existing same-level neighbour cells that now stream from the new blocks
void launch_refresh_neighbours(const Ctx &c, const int32_t *list, int n, const LevelParams &lp);
// mode 0: interface parent cells; 1: every parent cell (non-refined entries are skipped)
// U (all_cells = 1): the averaging also writes the criterion velocities of
// the children it reads that have no N_SKIP link
void launch_average(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells,
                    double *U = nullptr);
// ghost interpolation into level L+1 (interface parents ilist) and the
// collide-stream sweep of level L (launch order clist) in one launch; BGK;
// exchange and the result as for launch_collide_stream
bool launch_interp_collide(const Ctx &c, const int32_t *ilist, int ni, const int32_t *clist, int nblk, int L,
                           const LevelParams &lp, const BCParams &bc, bool exchange = false);
void launch_fill_rest(const Ctx &c);
// initial condition on root blocks [b0, b1) from rho_u_dev[((B - b0) Mb + l) 4]
void launch_set_rho_u_root(const Ctx &c, const double *rho_u_dev, int b0, int b1);
// criterion velocities of level L's blocks in `list`; children: `list` holds
// the interface parents of level L-1 and only their children with an N_SKIP
// link are done (the rest came from launch_average with U)
void launch_velocity(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp, bool children = false);
void launch_vorticity(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp);
void launch_block_f(const Ctx &c, int set, int b0, int b1, double *stage, const LevelParams &lp);
void launch_out_gather(const Ctx &c, int kind, int b0, int b1, int32_t off0, void *stage, const LevelParams &lp);
void launch_mass(const Ctx &c, const LevelParams &lp);
// the same sums through the fixed device array of the library (no arena
// scratch): its address on `device` (resolved once, with that device
// current), the largest block capacity it serves, and the launch
constexpr int kMaxDevices = 64;
hipError_t mass_scratch(int device, double **ptr);
int64_t mass_static_max_blocks();
void launch_mass_static(const Ctx &c, const LevelParams &lp, double *chunks, double *out_dev);
// momentum exchange with solid blocks: per-level totals out[lmax][3] (device), reset to zero
void launch_exchange(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp);
void launch_exchange_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                           const int32_t *count, int par, int grid);
void launch_force_sum(const Ctx &c, double *out);
void launch_force_reset(const Ctx &c);

// ---- batched solver launches: one persistent launch per level over every
// simulation of a batch (items = simulation << 24 | block, counts on the device)
void launch_collide_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                          const int32_t *count, int L, int par, int nt, int grid);
void launch_interp_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                         const int32_t *count, int L, int par0, int par1, int grid);
void launch_average_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                          const int32_t *count, int L, int par0, int par1, int grid);
// items[(3 L + kind) * stride + ...], counts[3 L + kind]: kind 0 launch order, 1 interface parents,
// 2 leaf blocks next to a solid block
void launch_batch_items(hipStream_t stream, const SimDesc *sims, int nsims, int lmax, int cap_max, uint32_t *items,
                        int64_t stride, int32_t *counts);

// ---- mesh kernels (mesh_kernels.hip) ----
void launch_init_mesh(const Ctx &c);
void launch_crit_reset(const Ctx &c);
// block desired levels from the vorticity maxima: relative threshold theta,
// or (ladder != nullptr) |w| * scale against the ladder thresholds
// ladder[p] = 2^(n_start - p n_inc), p = 1 .. L_max-1 (+inf when above 2)
struct LadderParams {
    double scale;
    double thr[kMaxLevels];
};
void launch_tag_vorticity(const Ctx &c, double theta, const LadderParams *ladder);
void launch_tag_distance(const Ctx &c, double d_spec, int freeze);
void launch_effective_tags(const Ctx &c);
// adaptation after the counts are known on the host
void launch_adapt_assign(const Ctx &c, int n_ref);                 // S2 + S3
void launch_adapt_build(const Ctx &c, int n_ref);                 // S4 .. S7 (statuses)
void launch_connectivity(const Ctx &c, int id_bound);             // S8 + masks + interface lists
void launch_out_count(const Ctx &c);  // per-block output counts + exclusive offsets, n_out

}  // namespace amr
