/*
 * amr_oracle.h -- plain, slow, FP64 CPU oracle of the block-based AMR lattice
 * Boltzmann method of Ahmed & Sakane et al., "GPU-Native Adaptive Mesh
 * Refinement with Application to Lattice Boltzmann Simulations"
 * (arXiv 2308.08085).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this code; it exists to check the HIP path.  It shares no code, header,
 * table or constant with the HIP library: every lattice table, index formula
 * and update rule here is written out independently from the paper.
 *
 * Conventions (the paper's notation where it has one):
 *   - cell l = i + 4j + 16k inside a 4^d block (Sec. "Data Structures");
 *   - block neighbour p uses the D2Q9 (2-D) / D3Q27 (3-D) vectors, p = 0 is
 *     the block itself (Sec. "Data Structures", velocity-set figure);
 *   - nbr codes: id >= 0, NONE = -1, N_SKIP = -2, domain face f -> -3-f
 *     (faces -x,+x,-y,+y,-z,+z = 0..5), solid -> -9;
 *   - block origins are integers in units of the finest possible cell.
 */
#ifndef AMR_ORACLE_H
#define AMR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim;            /* 2 or 3 */
    int32_t q;              /* 9 (2-D), 19 or 27 (3-D) */
    int32_t root[3];        /* root blocks per axis; root[2] = 1 in 2-D */
    int32_t lmax;           /* number of grid levels L_max >= 1 */
    int32_t cap;            /* block capacity (IDs 0 .. cap-1) */
    double nu0;             /* kinematic viscosity in level-0 lattice units */
    int32_t periodic[3];
    int32_t face_kind[6];   /* 0 = known velocity (bounce-back), 1 = outflow (anti-bounce-back) */
    double face_u[6][3];    /* wall velocity of velocity faces */
    int32_t face_prio[6];   /* edge/corner links take the BC of the highest-priority face */
    const uint8_t *solid;   /* per root block (structured order), 1 = solid; may be NULL */
    int32_t rescale_mode;   /* 0 = the paper's rescaling; 1 = deliberately wrong ratio (tests only) */
    int32_t interp;         /* coarse-to-fine interpolation: 0 = linear, 1 = cubic */
} orc_config;

typedef struct {
    int32_t kind;           /* 0 = relative vorticity threshold, 1 = distance to solid / outflow,
                               2 = log2 ladder of the vorticity (Alg. 3) */
    double theta;           /* kind 0: refine where block vorticity > theta * max */
    double d_spec;          /* kind 1: distance in root cells, divided by 2^L on level L */
    int32_t freeze;         /* kind 1: refined blocks become refined-permanent */
    double n_start, n_inc;  /* kind 2: the ladder's start and increment */
} orc_tag_params;

typedef struct orc orc_t;

/* lattice tables: c[q*3], w[q], opp[q] */
int orc_lattice(int dim, int q, int32_t *c, double *w, int32_t *opp);
/* equilibrium (single cell) */
int orc_feq(int dim, int q, double rho, const double *u, double *out);
/* BGK collision of a single cell with relaxation rate omega */
int orc_collide(int dim, int q, double omega, const double *f, double *out);
/* moment-space collision of one D3Q27 cell (see orc_set_collision) and its moment matrix [27][27] */
int orc_mrt_collide(double omega, double s_high, const double *f, double *out);
int orc_mrt_matrix(double *m_out);
/* linear interpolation of all cells of child c of a parent block; parent[Mb*q], out[Mb*q] (cell-major) */
int orc_interp_child(int dim, int q, double r, const double *parent, int child, double *out);
/* the same with cubic interpolation (Sec. "Cubic Interpolation") */
int orc_interp_child_cubic(int dim, int q, double r, const double *parent, int child, double *out);
/* averaging of all parent cells from their children; children[Nc*Mb*q], out[Mb*q] */
int orc_average_parent(int dim, int q, double r, const double *children, double *out);

orc_t *orc_create(const orc_config *cfg);
void orc_destroy(orc_t *o);
/* initial condition on the root level: ru[(B*Mb + l)*4 + {rho,ux,uy,uz}] for every root block */
int orc_set_root_rho_u(orc_t *o, const double *ru);
/* copy f of block B (current level buffer), cell-major [Mb*q] */
int orc_get_block_f(orc_t *o, int32_t B, double *out);
int orc_set_block_f(orc_t *o, int32_t B, const double *in);
/* every active block's current data, [cap][Mb][q] cell-major; inactive blocks read 0 */
int orc_get_f_all(orc_t *o, double *out);
/* cell classes of an active block: 0 interior, 1 interface, 2 ghost; out[Mb] */
int orc_cell_classes(orc_t *o, int32_t B, int32_t *out);
/* host threads of the per-block loops (n <= 0: unchanged); returns the count in use */
int orc_set_threads(int n);
/* collision of the sweeps: kind 0 = BGK (default), 1 = moment-space, D3Q27
 * only, moments above second order relaxing at s_high in (0, 2) */
int orc_set_collision(orc_t *o, int kind, double s_high);
int orc_step(orc_t *o, int32_t n_coarse_steps);
/* one collide-stream sweep of level L alone (for timing; leaves the forest mid-step) */
int orc_sweep(orc_t *o, int32_t L);
int orc_sync(orc_t *o);
int orc_tag(orc_t *o, const orc_tag_params *p, const int8_t *tags_in, int8_t *tags_out);
int orc_adapt(orc_t *o, int32_t *stats /* [4]: n_refine, n_coarsen, n_reverted, n_ignored */);
/* momentum exchange with the solid blocks since the last reset (or mesh
 * change), per level: out[L*4 + 0..2] force summed over that level's sweeps
 * in its lattice units, out[L*4 + 3] the number of sweeps */
int orc_force(orc_t *o, double *out /* [lmax][4] */, int reset);
/* per-block criterion of the last orc_tag (kind 0), -1 for non-leaves */
int orc_get_crit(orc_t *o, double *out /* cap */);

/* number of output cells: leaf, non-ghost cells of active blocks */
int64_t orc_n_out(orc_t *o);
int orc_get_out(orc_t *o, int32_t *blk, int32_t *cell, double *rho, double *u3, double *f);
int orc_mass_mom(orc_t *o, double *out4);
int orc_get_mesh(orc_t *o, int8_t *level, int8_t *status, int32_t *X3, int32_t *nbr, int32_t *nbrc,
                 int32_t *n_ids, int32_t *ids, int32_t *gtop, int32_t *gap);
int32_t orc_parity(orc_t *o, int32_t L);
/* rescaling ratios of level L -> L+1: out2[0] coarse-to-fine, out2[1] fine-to-coarse */
int orc_ratios(orc_t *o, int32_t L, double *out2);

#ifdef __cplusplus
}
#endif
#endif
