/*
 * amr_lbm.h -- C ABI of the MI355X (gfx950) block-based AMR lattice Boltzmann
 * library: BGK collide + stream over D2Q9 / D3Q19 / D3Q27 on a forest of
 * quad/octrees of 4^d-cell blocks, coarse-to-fine interpolation, fine-to-coarse
 * averaging and fully on-device mesh adaptation, after Ahmed, Sakane et al.,
 * "GPU-Native Adaptive Mesh Refinement with Application to Lattice Boltzmann
 * Simulations" (arXiv 2308.08085).
 *
 * General rules
 *   - Every call returns amr_status: AMR_OK (0) or a negative error code; the
 *     message of the last error on the calling thread is amr_last_error().
 *     No C++ exception crosses this interface.
 *   - A handle is not thread-safe.  All device work is enqueued on the HIP
 *     stream given to amr_create; calls that hand data to host memory, and
 *     amr_tag / amr_adapt (which read counters back), synchronise that stream.
 *   - Device memory: the caller allocates ONE device buffer (the arena) of at
 *     least amr_query_bytes() bytes and keeps it alive until amr_destroy; the
 *     library never allocates or frees device memory.  Host memory passed in
 *     is owned by the caller and only read/written during the call.
 *   - Block IDs, neighbour codes and statuses follow the paper's data
 *     structures (Sec. "Data Structures"): cell l = i + 4j + 16k inside a block;
 *     neighbour p uses the D2Q9 (2-D) or D3Q27 (3-D) direction numbering of
 *     the paper's velocity-set figure, p = 0 being the block itself;
 *     link codes: id >= 0, AMR_NONE, AMR_N_SKIP, AMR_FACE(f) for domain face f
 *     (-x,+x,-y,+y,-z,+z = 0..5), AMR_SOLID.
 */
#ifndef AMR_LBM_H
#define AMR_LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t amr_status;
#define AMR_OK 0
#define AMR_ERR_ARG (-1)       /* invalid argument; nothing was changed */
#define AMR_ERR_CAPACITY (-2)  /* arena or block capacity too small; nothing was changed */
#define AMR_ERR_STATE (-3)     /* call not valid in the current state */
#define AMR_ERR_DEVICE (-4)    /* a HIP runtime call or kernel launch failed */
#define AMR_ERR_UNSTABLE (-5)  /* non-finite mass after lbm_step with AMR_CHECK_FINITE */

/* link codes (Sec. "Refinement and Coarsening": N_skip marks a region covered
 * only by a coarser block) */
#define AMR_NONE (-1)
#define AMR_N_SKIP (-2)
#define AMR_FACE(f) (-3 - (f))
#define AMR_SOLID (-9)

/* block status (table of data structures, "cblock_ID_ref") */
enum amr_block_status {
    AMR_ST_UNREFINED = 0, AMR_ST_REFINED = 1, AMR_ST_REFINED_CHILD = 2, AMR_ST_REFINED_PERM = 3,
    AMR_ST_MARK_REFINE = 4, AMR_ST_MARK_COARSEN = 5, AMR_ST_NEW = 6, AMR_ST_REMOVE = 7, AMR_ST_INACTIVE = 8
};

/* storage of the distributions.  The "shifted" forms store g_p = f_p - w_p
 * (the deviation from the fluid at rest); arithmetic is FP64 for AMR_F64 and
 * FP32 otherwise. */
enum amr_storage { AMR_F64 = 0, AMR_F32 = 1, AMR_F32S = 2, AMR_F16S = 3, AMR_BF16S = 4 };

/* boundary kinds of the domain faces (Sec. "Lattice Boltzmann Method"):
 * known velocity (bounce-back with wall velocity) and outflow (anti-bounce-back
 * at rho_w = 1 with the cell's own velocity) */
enum amr_face_kind { AMR_FACE_VELOCITY = 0, AMR_FACE_OUTFLOW = 1 };

typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t q;                /* 9 (dim 2), 19 or 27 (dim 3) */
    int32_t root[3];          /* root blocks per axis (4^d cells each); root[2] = 1 for dim 2 */
    int32_t max_levels;       /* L_max: levels 0 .. L_max-1, 1 <= L_max <= 8 */
    int32_t max_blocks;       /* block capacity (IDs 0 .. max_blocks-1), >= number of root blocks */
    int32_t storage;          /* enum amr_storage */
    double nu0;               /* kinematic viscosity in level-0 lattice units; tau*_0 = 1/2 + 3 nu0 */
    int32_t periodic[3];      /* periodic axes (faces of a periodic axis are ignored) */
    int32_t face_kind[6];     /* enum amr_face_kind per face */
    double face_u[6][3];      /* wall velocity of AMR_FACE_VELOCITY faces */
    int32_t face_prio[6];     /* a link leaving through an edge or corner takes the BC of the
                                 highest-priority face it crosses (ties: lower face index) */
    const uint8_t *solid_root; /* host array, one flag per root block in structured order
                                  (x fastest); solid blocks are walls at rest.  Copied; may be NULL */
    int32_t interp;           /* enum amr_interp: coarse-to-fine interpolation of ghost cells and
                                 new children */
} amr_config;

/* Coarse-to-fine interpolation (Sec. "Linear Interpolation" and "Cubic
 * Interpolation"): the (bi/tri)linear polynomial through the 2^d parent cells
 * of the child's quadrant, or the tensor-product cubic through all 4^d parent
 * cells (positions -1/12 + I/6 + 2 I_c/3 in the unit square/cube spanned by
 * the parent's corner cell centres).  Both act on the rescaled parent cells. */
enum amr_interp { AMR_INTERP_LINEAR = 0, AMR_INTERP_CUBIC = 1 };

/* Refinement criteria (Sec. "Adaptive Mesh Refinement" of the solver) */
enum amr_tag_kind {
    AMR_TAG_VORTICITY_REL = 0, /* refine leaves whose block vorticity maximum exceeds theta * (max over
                                  all leaves); coarsen refined blocks whose children all fall below */
    AMR_TAG_DISTANCE = 1,      /* refine leaves closer than d_spec / 2^L (root cells) to a solid
                                  block or an outflow face; freeze = 1 makes them permanent */
    AMR_TAG_LADDER = 2         /* Alg. 3: desired level from eps = min(1, log2 |w|), |w| the block
                                  vorticity maximum in units of domain length 1 along x
                                  (N_x times the root-lattice value): L_max-1, lowered to
                                  L_max-1-p for every p = 1 .. L_max-1 with eps < n_start - p n_inc.
                                  Leaves below it refine; parents whose children all want at most
                                  the parent's level coarsen */
};

typedef struct {
    int32_t kind;    /* enum amr_tag_kind */
    double theta;    /* AMR_TAG_VORTICITY_REL */
    double d_spec;   /* AMR_TAG_DISTANCE, root-cell units */
    int32_t freeze;  /* AMR_TAG_DISTANCE */
    double n_start;  /* AMR_TAG_LADDER */
    double n_inc;    /* AMR_TAG_LADDER */
} amr_tag_params;

/* tag values (one int8 per block ID) */
#define AMR_TAG_NONE 0
#define AMR_TAG_REFINE 1
#define AMR_TAG_COARSEN (-1)
#define AMR_TAG_REFINE_PERM 2

/* Device time of each adaptation step (the paper's breakdown of the
 * refinement and coarsening routine, Sec. "Refinement and Coarsening" and its
 * timing tables), in amr_adapt_stats.step_ms.  The first three are those of
 * the last amr_tag call on the handle. */
enum amr_adapt_step {
    AMR_T_SYNC_AVERAGE = 0,  /* pre-adaptation averaging of every parent (amr_tag) */
    AMR_T_SYNC_INTERP = 1,   /* pre-adaptation ghost interpolation (amr_tag) */
    AMR_T_CRITERION = 2,     /* velocities, criterion, block maxima, tags (amr_tag) */
    AMR_T_PREP = 3,          /* effective tags and their counts */
    AMR_T_ASSIGN = 4,        /* S2-S3: first-child IDs from the gap stack, 2:1 reversion */
    AMR_T_BUILD = 5,         /* S4-S6: new children, removals, ID-set compaction and append */
    AMR_T_CONNECT = 6,       /* S8: links and neighbour-children, cell masks, work lists */
    AMR_T_FILL = 7,          /* S7: every cell of the new children, neighbours' refreshed slots */
    AMR_T_STEPS = 8
};

typedef struct {
    int32_t n_refine;         /* blocks refined */
    int32_t n_coarsen;        /* blocks whose children were removed */
    int32_t n_reverted;       /* coarsen marks reverted by 2:1 balance */
    int32_t n_free;           /* gap-stack size after the call */
    int32_t level_blocks[8];  /* active blocks per level after the call */
    double step_ms[8];        /* device milliseconds per step, indexed by amr_adapt_step; the
                                 adaptation steps are 0 when nothing was refined or coarsened */
} amr_adapt_stats;

typedef struct amr_handle amr_t;

/* Size of the device arena a configuration needs (distribution buffers, block
 * metadata, ID sets, gap stack and scratch).  Pure host computation.
 * Errors: AMR_ERR_ARG for an invalid configuration. */
amr_status amr_query_bytes(const amr_config *cfg, uint64_t *arena_bytes);

/* Build the root grid (Sec. "Overview": root IDs in structured order, the gap
 * set holds every other ID in reverse) on the caller's device arena and HIP
 * stream, with f = feq(rho = 1, u = 0) everywhere.  `hip_stream` is a
 * hipStream_t (NULL = default stream).  The arena must be 256-byte aligned.
 * Errors: AMR_ERR_ARG, AMR_ERR_CAPACITY (arena smaller than amr_query_bytes),
 * AMR_ERR_DEVICE. */
amr_status amr_create(const amr_config *cfg, void *dev_arena, uint64_t arena_bytes, void *hip_stream,
                      amr_t **out);

/* Pre-adaptation synchronisation (average every parent from level L_max-2 up,
 * then fill every ghost layer from level 0 down) followed by tagging.  With
 * tags_in == NULL the criterion `p` is evaluated on the device; otherwise the
 * host array tags_in[max_blocks] (AMR_TAG_* values) is adopted.  Either way
 * ineligible tags are dropped: refinement only of leaves below level L_max-1
 * with no N_SKIP link (2:1 balance), coarsening only of blocks with status
 * AMR_ST_REFINED.  tags_out (host, max_blocks, nullable) receives the
 * effective tags.  Synchronises the stream.  The device times of the
 * synchronisation and the criterion are kept for the next amr_adapt's stats.
 * Errors: AMR_ERR_ARG, AMR_ERR_DEVICE. */
amr_status amr_tag(amr_t *h, const amr_tag_params *p, const int8_t *tags_in, int8_t *tags_out);

/* Refine and coarsen every tagged block at once (Sec. "Refinement and
 * Coarsening"): gaps are assigned to refined blocks in ascending block ID from
 * the top of the gap stack; coarsen marks that would break 2:1 balance are
 * reverted; freed child groups are pushed back in reverse (parent level,
 * parent ID, child) order; ID sets drop removed IDs stably and append new
 * children in (parent ID, child) order; new children are interpolated from
 * their parents; neighbour and neighbour-child tables are rebuilt.  Consumes
 * the tags of the last amr_tag.  `stats` (host, nullable) receives counts and
 * the device time of each step (amr_adapt_step).
 * Errors: AMR_ERR_CAPACITY when the gap stack cannot hold the new children
 * (nothing changed), AMR_ERR_DEVICE. */
amr_status amr_adapt(amr_t *h, amr_adapt_stats *stats);

/* Advance n coarse time steps (Sec. "Grid Advancement"): step(L) = interpolate
 * to the ghosts of level L+1, collide and stream level L, step(L+1) twice,
 * average the interface cells back.  Asynchronous unless flags has
 * AMR_CHECK_FINITE, which sums the FP64 mass afterwards and returns
 * AMR_ERR_UNSTABLE if it is not finite.
 * Errors: AMR_ERR_ARG (n < 0), AMR_ERR_UNSTABLE, AMR_ERR_DEVICE. */
#define AMR_CHECK_FINITE 1u
#define AMR_USE_GRAPH 2u   /* replay one captured coarse step (HIP graph) instead of eager launches */
#define AMR_PROFILE 4u     /* time every solver launch with HIP events on the stream (eager; see
                              AMR_FIELD_KERNEL_STATS); synchronises the stream */
amr_status lbm_step(amr_t *h, int32_t n_coarse_steps, uint32_t flags);

/* Field and mesh access.  op: AMR_GET copies device data into the host buffer
 * `buf`; AMR_SET copies host data in (only the kinds marked SET).  `sim` must
 * be 0.  `bytes` is the size of `buf`; too small -> AMR_ERR_ARG and
 * amr_last_error() states the required size.  Synchronises the stream.
 *
 * "Output cells" are the leaf (status AMR_ST_UNREFINED), non-ghost cells of
 * active blocks, in (block ID, cell) order.
 *   AMR_FIELD_N_OUT        GET int64[1]: number of output cells
 *   AMR_FIELD_CELLS        GET int32[n][2]: (block ID, cell) of each output cell
 *   AMR_FIELD_RHO_U        GET double[n][4]: rho, ux, uy, uz of each output cell;
 *                          SET double[n_root_blocks*Mb][4] in (root block, cell) order:
 *                          f = feq(rho, u) on the root level (initial condition)
 *   AMR_FIELD_F            GET double[n][q]: unshifted f of each output cell
 *   AMR_FIELD_BLOCK_F      GET/SET double[max_blocks][Mb][q]: unshifted f of every cell of
 *                          every block in its level's current buffer (inactive blocks: any)
 *   AMR_FIELD_LEVEL        GET int8[max_blocks]
 *   AMR_FIELD_STATUS       GET int8[max_blocks]
 *   AMR_FIELD_COORD        GET int32[3][max_blocks]: block origin in finest-cell units
 *   AMR_FIELD_NBR          GET int32[nb][max_blocks]: neighbour links, nb = 9 (2-D) / 27 (3-D)
 *   AMR_FIELD_NBR_CHILD    GET int32[nb][max_blocks]: first child of each neighbour, AMR_NONE
 *                          for a leaf, the link code if negative
 *   AMR_FIELD_IDSET        GET int32[L_max + L_max*max_blocks]: per-level counts, then
 *                          each level's list (padded to max_blocks)
 *   AMR_FIELD_GAP          GET int32[1 + max_blocks]: gap-stack size, then the stack bottom-up
 *   AMR_FIELD_COUNTS       GET int32[L_max]: active blocks per level
 *   AMR_FIELD_MASS_MOM     GET double[4]: FP64 sum over output cells of V rho and V rho u,
 *                          V = 2^(-d L) the cell volume in root cells
 *   AMR_FIELD_CRIT         GET double[max_blocks]: block vorticity maximum of the last
 *                          AMR_TAG_VORTICITY_REL tagging, -1 for non-leaves
 *   AMR_FIELD_PARITY       GET int32[L_max]: buffer (0/1) holding each level's data
 *   AMR_FIELD_FORCE        GET double[L_max][4]: momentum exchange with the solid blocks (Sec.
 *                          "Flow Past a Square Cylinder"): per level, the sum over its sweeps of
 *                          2 f*_q c_q over every post-collision population of a leaf cell whose
 *                          link ends in a solid block (x, y, z, in that level's lattice units),
 *                          then the number of sweeps; since the last reset: SET (any buffer),
 *                          creation, or an amr_adapt that changes the mesh
 *   AMR_FIELD_FORCE_ON     GET/SET int32[1]: 1 (the default) = accumulate the momentum
 *                          exchange in every lbm_step and batch step, 0 = skip its launches
 *                          and sweep counts (for runs that sample the force only part of the
 *                          time); SET accepts 0 or 1 (else AMR_ERR_ARG) and re-captures the
 *                          step graphs when the value changes
 *   AMR_FIELD_STREAM_BYTES GET/SET int64[1]: store policy of the collide-stream sweeps: a
 *                          level whose sweep writes more than this many bytes is written with
 *                          non-temporal stores (its output is read again only by the next sweep,
 *                          after the whole level has passed through the caches); default
 *                          128 MiB (half the 256 MB Infinity Cache), 0 = every level, any
 *                          value >= 0 (else AMR_ERR_ARG).  Results do not depend on it; SET
 *                          re-captures the step graphs when the value changes
 *   AMR_FIELD_SYNC_VELOCITY GET/SET int32[1]: 1 (the default) = the averaging of the
 *                          pre-adaptation synchronisation also computes the
 *                          vorticity criterion's velocities of the children it reads (those
 *                          without an N_SKIP link, whose cells the ghost interpolation that
 *                          follows leaves alone), and the velocity pass covers only the rest;
 *                          0 = the velocity pass computes every velocity.  Criterion values
 *                          and tags do not depend on it; SET accepts 0 or 1 (else AMR_ERR_ARG)
 *   AMR_FIELD_SKIP_PARENTS GET/SET int32[1]: 0 (the default) = every sweep of level L
 *                          advances every block of the level's ID set (Sec. "Grid Advancement");
 *                          1 = it leaves out the refined blocks none of whose children has an
 *                          N_SKIP link (the paper leaves parents out of the advancement, Sec.
 *                          "Streaming", and its MLUPS count excludes them).  Under linear interpolation nothing a leaf reads depends
 *                          on those blocks' cells before the next synchronisation (amr_tag)
 *                          averages them again, so leaf cells, output fields, forces and tags
 *                          are unchanged bit for bit; the skipped blocks' own cells (and cells of
 *                          neighbouring parents away from any coarse leaf) hold stale values
 *                          until then.  SET 1 needs linear interpolation (else AMR_ERR_ARG); SET
 *                          re-captures the step graphs when the value changes.  Batch steps
 *                          always advance every block.
 *   AMR_FIELD_KERNEL_STATS GET double[3][4]: for the collide-stream, interpolation and averaging
 *                          kernels: launches, summed event time (ms), blocks processed, and the
 *                          distribution bytes those blocks must move, accumulated over lbm_step
 *                          calls made with AMR_PROFILE; SET (any buffer) resets the sums
 * Errors: AMR_ERR_ARG, AMR_ERR_DEVICE. */
#define AMR_GET 0
#define AMR_SET 1
enum amr_field_kind {
    AMR_FIELD_N_OUT = 0, AMR_FIELD_CELLS = 1, AMR_FIELD_RHO_U = 2, AMR_FIELD_F = 3, AMR_FIELD_BLOCK_F = 4,
    AMR_FIELD_LEVEL = 5, AMR_FIELD_STATUS = 6, AMR_FIELD_COORD = 7, AMR_FIELD_NBR = 8,
    AMR_FIELD_NBR_CHILD = 9, AMR_FIELD_IDSET = 10, AMR_FIELD_GAP = 11, AMR_FIELD_COUNTS = 12,
    AMR_FIELD_MASS_MOM = 13, AMR_FIELD_CRIT = 14, AMR_FIELD_PARITY = 15, AMR_FIELD_KERNEL_STATS = 16,
    AMR_FIELD_FORCE = 17, AMR_FIELD_FORCE_ON = 18, AMR_FIELD_STREAM_BYTES = 19, AMR_FIELD_SYNC_VELOCITY = 20,
    AMR_FIELD_SKIP_PARENTS = 21
};
amr_status amr_fields(amr_t *h, int32_t op, int32_t kind, int32_t sim, void *buf, uint64_t bytes);

/* Collision operator of the collide-stream sweeps.  The paper's method is BGK
 * (Sec. "Collision"), the default.  It names moment-space (multiple-relaxation-
 * time) collision as the alternative (Sec. "Lattice Boltzmann Method"); this
 * library offers one for D3Q27 only:
 *   AMR_COLLIDE_MRT       moments phi_a(c_x) phi_b(c_y) phi_c(c_z), phi_0 = 1,
 *                         phi_1 = c, phi_2 = 3 c^2 - 1; density, momentum and the
 *                         second-order moments relax at each level's omega, the
 *                         17 higher moments at s_high; transforms on the vector
 *                         ALU in the storage's arithmetic (FP64 or FP32);
 *   AMR_COLLIDE_MRT_MFMA  the same operator with both high-moment transforms on
 *                         the matrix cores (FP16 operands, FP32 accumulation);
 *                         storages with FP32 arithmetic only.
 * s_high = omega gives the BGK result exactly.  The interpolation and averaging
 * rescaling stay those of BGK (Secs. "Linear Interpolation", "Averaging"), whose
 * derivation assumes BGK.  Batches (amr_batch_create) accept BGK members only.
 * kind: enum amr_collision; s_high in (0, 2), ignored for AMR_COLLIDE_BGK.
 * Captured step graphs are re-captured.
 * Errors: AMR_ERR_ARG (unknown kind, lattice other than D3Q27, FP64 storage
 * with AMR_COLLIDE_MRT_MFMA, s_high out of range, handle in a batch). */
enum amr_collision { AMR_COLLIDE_BGK = 0, AMR_COLLIDE_MRT = 1, AMR_COLLIDE_MRT_MFMA = 2 };
amr_status amr_set_collision(amr_t *h, int32_t kind, double s_high);

/* Release the host-side handle.  The arena stays the caller's; the stream is
 * synchronised first.  NULL is accepted. */
amr_status amr_destroy(amr_t *h);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops): the mass and momentum of
 * AMR_FIELD_MASS_MOM, equal to it bit for bit, written to `out_dev` (4 doubles
 * of device memory owned by the caller) and only enqueued on the handle's
 * stream.  It allocates nothing and uses no arena scratch: its partial sums
 * live in one fixed device array of the library (32 KiB per GPU, held until
 * the process ends), so meshes of at most 4,194,304 blocks (max_blocks) are
 * accepted.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams, or other handles' calls on the same GPU not
 * ordered with this one) race.
 * Errors: AMR_ERR_ARG (NULL), AMR_ERR_CAPACITY (max_blocks above the limit),
 * AMR_ERR_DEVICE. */
amr_status amr_mass_mom_static(amr_t *h, double *out_dev);

/* ---------------------------------------------------------------------------
 * Batches: many independent simulations advanced together.  Not part of the
 * paper's method, which advances one forest; each member keeps its own block-ID
 * space, tables and adaptation (amr_tag / amr_adapt / amr_fields on its own
 * handle), and a batch step gives every member exactly the result of the same
 * number of lbm_step calls on it alone.  Members of equal lattice and storage
 * advance each level sweep in one persistent launch (collide-stream, ghost
 * interpolation, interface averaging); the work lists are rebuilt on the
 * device from the members' own lists at the start of every coarse step, so a
 * captured coarse step stays valid while members adapt between batch steps. */
typedef struct amr_batch amr_batch_t;

typedef struct {
    int32_t threads;    /* threads per workgroup of the collide-stream launches: 64, 128 or 256
                           (3-D: 1, 2 or 4 blocks per workgroup; 2-D: 4, 8 or 16) */
    int32_t wg_per_cu;  /* persistent grid = wg_per_cu x compute units, 1 .. 64 */
    int32_t schedule;   /* 0: groups of different lattice/storage one after another;
                           1: each group on its own concurrent branch of the step */
} amr_batch_tuning;

/* Device arena a batch of `n` simulations needs (descriptors and work lists).
 * Errors: AMR_ERR_ARG. */
amr_status amr_batch_query_bytes(amr_t *const *sims, int32_t n, uint64_t *arena_bytes);

/* Group `n` existing simulations (host array of handles, copied) into a batch
 * on the caller's arena (256-byte aligned, at least amr_batch_query_bytes) and
 * stream.  Every member must have been created on `hip_stream` and have made
 * the same number of coarse steps modulo 2; at most 255 members per lattice
 * and storage, each with max_blocks <= 2^24.  The members must outlive the
 * batch.  Default tuning: 256 threads, 8 workgroups per CU, schedule 0.
 * Errors: AMR_ERR_ARG, AMR_ERR_STATE, AMR_ERR_CAPACITY, AMR_ERR_DEVICE. */
amr_status amr_batch_create(amr_t *const *sims, int32_t n, void *dev_arena, uint64_t arena_bytes, void *hip_stream,
                            amr_batch_t **out);

/* Advance every member n coarse steps (flags: AMR_USE_GRAPH, AMR_CHECK_FINITE;
 * AMR_PROFILE is refused).  After a batch step the members must not be stepped
 * alone before the next batch step unless by an even number of coarse steps.
 * Errors: AMR_ERR_ARG, AMR_ERR_STATE, AMR_ERR_UNSTABLE (first non-finite
 * member named in amr_last_error), AMR_ERR_DEVICE. */
amr_status amr_batch_step(amr_batch_t *b, int32_t n_coarse_steps, uint32_t flags);

/* Launch shape of the batch (drops its captured graphs).  Errors: AMR_ERR_ARG. */
amr_status amr_batch_set_tuning(amr_batch_t *b, const amr_batch_tuning *t);
amr_status amr_batch_get_tuning(amr_batch_t *b, amr_batch_tuning *t);

/* Time every launch shape (threads x wg_per_cu x schedule) over `trial_steps`
 * graph-replayed coarse steps each, keep the fastest and return it with its
 * time per coarse step.  The members advance (2 + trial_steps) coarse steps
 * per shape tried; results do not depend on the shape.
 * Errors: AMR_ERR_ARG, AMR_ERR_STATE, AMR_ERR_DEVICE. */
amr_status amr_batch_autotune(amr_batch_t *b, int32_t trial_steps, amr_batch_tuning *best, double *best_ms);

/* Release the batch (members and arena stay the caller's).  NULL is accepted. */
amr_status amr_batch_destroy(amr_batch_t *b);

/* Message of the last error raised on the calling thread ("" if none). */
const char *amr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMR_LBM_H */
