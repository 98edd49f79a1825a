/*
 * amr_oracle.c -- plain FP64 CPU oracle of block-based AMR for the lattice
 * Boltzmann method (arXiv 2308.08085).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  It shares no code
 * with the HIP library.
 *
 * Each routine names the passage of the paper it follows.  Where the paper is
 * silent or garbled the reading taken is stated at the routine (the list of
 * readings is kept with the design notes of the repository).  The loops are
 * deliberately naive: one cell, one direction at a time, in the order the
 * paper describes, no blocking or fusion.
 *
 * Threads: the per-block loops of a level sweep, of the interpolation, of the
 * averaging and of the criterion may run on several host threads (OpenMP,
 * orc_set_threads).  Every block writes only slots no other block writes in
 * the same loop (a push targets one slot per (cell, direction); the
 * interpolation writes the children of its own parent; the averaging its own
 * parent's cells), and no sum crosses blocks, so the results do not depend on
 * the thread count.
 */
#include "amr_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NONE_ID (-1)
#define N_SKIP (-2)
#define FACE_CODE(f) (-3 - (f))
#define SOLID_CODE (-9)
#define MAXL 16

/* block status values (table of data structures, "cblock_ID_ref") */
enum {
    ST_UNREFINED = 0, ST_REFINED = 1, ST_REFINED_CHILD = 2, ST_REFINED_PERM = 3,
    ST_MARK_REFINE = 4, ST_MARK_COARSEN = 5, ST_NEW = 6, ST_REMOVE = 7, ST_INACTIVE = 8
};
enum { CLS_INTERIOR = 0, CLS_INTERFACE = 1, CLS_GHOST = 2 };
enum { TAG_NONE = 0, TAG_REFINE = 1, TAG_COARSEN = -1, TAG_REFINE_PERM = 2 };

/* ------------------------------------------------------------------------ */
/* Velocity sets (Sec. "Lattice Boltzmann Method" and the velocity-set figure).
 * The numbering follows the figure; the weights are the standard quadrature
 * weights of each set. */
static const int VEC2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int VEC3[27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, 0, 1}, {-1, 0, -1}, {0, 1, 1}, {0, -1, -1},
    {1, -1, 0}, {-1, 1, 0}, {1, 0, -1}, {-1, 0, 1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
    {-1, 1, 1}, {1, -1, -1}};

static int lattice_ok(int dim, int q)
{
    return (dim == 2 && q == 9) || (dim == 3 && (q == 19 || q == 27));
}

static double lattice_weight(int dim, int q, int p)
{
    const int *c = dim == 2 ? VEC2[p] : VEC3[p];
    int n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    if (dim == 2) {
        if (n2 == 0) return 4.0 / 9.0;
        if (n2 == 1) return 1.0 / 9.0;
        return 1.0 / 36.0;
    }
    if (q == 19) {
        if (n2 == 0) return 1.0 / 3.0;
        if (n2 == 1) return 1.0 / 18.0;
        return 1.0 / 36.0;
    }
    if (n2 == 0) return 8.0 / 27.0;
    if (n2 == 1) return 2.0 / 27.0;
    if (n2 == 2) return 1.0 / 54.0;
    return 1.0 / 216.0;
}

static int lattice_opposite(int dim, int p)
{
    const int *c = dim == 2 ? VEC2[p] : VEC3[p];
    int n = dim == 2 ? 9 : 27;
    for (int r = 0; r < n; r++) {
        const int *d = dim == 2 ? VEC2[r] : VEC3[r];
        if (d[0] == -c[0] && d[1] == -c[1] && d[2] == -c[2]) return r;
    }
    return -1;
}

int orc_lattice(int dim, int q, int32_t *c, double *w, int32_t *opp)
{
    if (!lattice_ok(dim, q)) return -1;
    for (int p = 0; p < q; p++) {
        const int *v = dim == 2 ? VEC2[p] : VEC3[p];
        for (int a = 0; a < 3; a++) c[p * 3 + a] = v[a];
        w[p] = lattice_weight(dim, q, p);
        opp[p] = lattice_opposite(dim, p);
    }
    return 0;
}

/* Moments: rho = sum_p f_p, rho*u = sum_p f_p c_p (Sec. "Lattice Boltzmann Method"). */
static void moments(int dim, int q, const double *f, double *rho, double *u)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < q; p++) {
        const int *c = dim == 2 ? VEC2[p] : VEC3[p];
        r += f[p];
        for (int a = 0; a < 3; a++) j[a] += f[p] * c[a];
    }
    *rho = r;
    for (int a = 0; a < 3; a++) u[a] = j[a] / r;
}

/* Second-order equilibrium.  The printed formula swaps the signs of the
 * (u.c)^2 and u.u terms; the standard form is taken:
 * feq_p = w_p rho (1 + u.c/cs^2 + (u.c)^2/(2 cs^4) - u.u/(2 cs^2)), cs^2 = 1/3. */
static void equilibrium(int dim, int q, double rho, const double *u, double *out)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int p = 0; p < q; p++) {
        const int *c = dim == 2 ? VEC2[p] : VEC3[p];
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        out[p] = lattice_weight(dim, q, p) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

int orc_feq(int dim, int q, double rho, const double *u, double *out)
{
    if (!lattice_ok(dim, q)) return -1;
    equilibrium(dim, q, rho, u, out);
    return 0;
}

/* BGK collision f* = (1 - omega) f + omega feq (Sec. "Collision"). */
int orc_collide(int dim, int q, double omega, const double *f, double *out)
{
    if (!lattice_ok(dim, q)) return -1;
    double rho, u[3], feq[27];
    moments(dim, q, f, &rho, u);
    equilibrium(dim, q, rho, u, feq);
    for (int p = 0; p < q; p++) out[p] = (1.0 - omega) * f[p] + omega * feq[p];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Moment-space (multiple-relaxation-time) collision for D3Q27.  The paper
 * uses BGK and names moment-space operators only as an alternative (Sec.
 * "Lattice Boltzmann Method" and its review of collision operators); this is
 * the reference for the library's optional moment-space collision.
 * Moment k = a + 3 b + 9 c (a, b, c in 0..2) is sum_p phi_a(c_px) phi_b(c_py)
 * phi_c(c_pz) f_p with phi_0 = 1, phi_1 = c, phi_2 = 3 c^2 - 1.  Its order
 * counts 1 per phi_1 and 2 per phi_2 factor; moments of order <= 2 (density,
 * momentum, stress) relax at omega, the rest at s_high:
 *   m = M f,  m_eq = M f_eq,  f* = M^-1 (m - S (m - m_eq)),
 * with M^-1 from Gauss-Jordan elimination.  s_high = omega gives BGK. */
static double MRT_M[27][27], MRT_MI[27][27];
static int mrt_ready = 0;

static double mrt_phi(int a, int c)
{
    return a == 0 ? 1.0 : (a == 1 ? (double)c : 3.0 * c * c - 1.0);
}

static int mrt_order(int k)
{
    int o = 0;
    for (int d = 0; d < 3; d++) {
        int a = k % 3;
        k /= 3;
        o += a;
    }
    return o;
}

static int mrt_init(void)
{
    if (mrt_ready) return 0;
    double A[27][54];
    for (int k = 0; k < 27; k++)
        for (int p = 0; p < 27; p++)
            MRT_M[k][p] = mrt_phi(k % 3, VEC3[p][0]) * mrt_phi((k / 3) % 3, VEC3[p][1]) * mrt_phi(k / 9, VEC3[p][2]);
    for (int i = 0; i < 27; i++)
        for (int j = 0; j < 54; j++) A[i][j] = j < 27 ? MRT_M[i][j] : (j - 27 == i ? 1.0 : 0.0);
    for (int col = 0; col < 27; col++) {
        int piv = col;
        for (int r = col + 1; r < 27; r++)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (fabs(A[piv][col]) < 1e-12) return -1;
        if (piv != col)
            for (int j = 0; j < 54; j++) { double t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
        double d = A[col][col];
        for (int j = 0; j < 54; j++) A[col][j] /= d;
        for (int r = 0; r < 27; r++) {
            if (r == col || A[r][col] == 0.0) continue;
            double fct = A[r][col];
            for (int j = 0; j < 54; j++) A[r][j] -= fct * A[col][j];
        }
    }
    for (int i = 0; i < 27; i++)
        for (int j = 0; j < 27; j++) MRT_MI[i][j] = A[i][27 + j];
    mrt_ready = 1;
    return 0;
}

static void mrt_relax(const double *f, const double *feq, double omega, double s_high, double *out)
{
    double ms[27];
    for (int k = 0; k < 27; k++) {
        double m = 0.0, meq = 0.0;
        for (int p = 0; p < 27; p++) {
            m += MRT_M[k][p] * f[p];
            meq += MRT_M[k][p] * feq[p];
        }
        double s = mrt_order(k) <= 2 ? omega : s_high;
        ms[k] = m - s * (m - meq);
    }
    for (int p = 0; p < 27; p++) {
        double v = 0.0;
        for (int k = 0; k < 27; k++) v += MRT_MI[p][k] * ms[k];
        out[p] = v;
    }
}

int orc_mrt_matrix(double *m_out /* [27][27], row = moment */)
{
    if (mrt_init() != 0) return -1;
    memcpy(m_out, MRT_M, sizeof(MRT_M));
    return 0;
}

int orc_mrt_collide(double omega, double s_high, const double *f, double *out)
{
    if (mrt_init() != 0) return -1;
    double rho, u[3], feq[27];
    moments(3, 27, f, &rho, u);
    equilibrium(3, 27, rho, u, feq);
    mrt_relax(f, feq, omega, s_high, out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Coarse-to-fine linear interpolation (Sec. "Linear Interpolation").
 * The parent's cells are rescaled first (g = feq + r (f - feq), Dupuis-Chopard);
 * fine cell (I,J,K) of child c sits at (-1/4 + I/2, -1/4 + J/2, -1/4 + K/2) in
 * the unit square/cube whose corners are the parent cells (2c_x+a, 2c_y+b,
 * 2c_z+e).  The printed 2-D polynomial writes a3*y for a3*x*y and the 3-D
 * coefficient list pairs a5/a6 with the wrong terms; the standard (bi/tri)linear
 * polynomial through the corners is used. */
static void rescale_cell(int dim, int q, double r, const double *f, double *g)
{
    double rho, u[3], feq[27];
    moments(dim, q, f, &rho, u);
    equilibrium(dim, q, rho, u, feq);
    for (int p = 0; p < q; p++) g[p] = feq[p] + r * (f[p] - feq[p]);
}

static double linear_poly(int dim, const double *F /* corners [a + 2b + 4e] */, double x, double y, double z)
{
    if (dim == 2) {
        double a0 = F[0];
        double a1 = F[1] - F[0];
        double a2 = F[2] - F[0];
        double a3 = F[3] - F[2] - F[1] + F[0];
        return a0 + a1 * x + a2 * y + a3 * x * y;
    }
    double a0 = F[0];
    double a1 = F[1] - F[0];
    double a2 = F[2] - F[0];
    double a3 = F[4] - F[0];
    double a4 = F[3] - F[1] - F[2] + F[0];              /* xy */
    double a5 = F[6] - F[2] - F[4] + F[0];              /* yz */
    double a6 = F[5] - F[1] - F[4] + F[0];              /* xz */
    double a7 = F[7] - F[3] - F[5] - F[6] + F[1] + F[2] + F[4] - F[0];
    return a0 + a1 * x + a2 * y + a3 * z + a4 * x * y + a5 * y * z + a6 * x * z + a7 * x * y * z;
}

/* Coarse-to-fine cubic interpolation (Sec. "Cubic Interpolation").  The
 * 4^d rescaled parent cells are the sampling points, at (m/3, n/3, e/3) in the
 * unit square/cube whose corners are the parent's corner cell centres; the
 * interpolant is the tensor-product polynomial of degree 3 per axis through all
 * of them (the one the paper's inverted system of monomials x^i y^j z^k
 * gives), written here as Lagrange interpolation.  Fine cell (I,J,K) of child
 * (cx,cy,cz) sits at -1/12 + I/6 + 2 cx/3 per axis. */
static double lagrange3(int m, double x)
{
    double v = 1.0;
    for (int k = 0; k < 4; k++)
        if (k != m) v *= (x - k / 3.0) / (m / 3.0 - k / 3.0);
    return v;
}

static void interp_child_cells_cubic(int dim, int q, const double *g /* rescaled parent, Mb*q */, int child,
                                     const unsigned char *only, double *out)
{
    int mb = dim == 2 ? 16 : 64;
    int cx = child & 1, cy = (child >> 1) & 1, cz = (child >> 2) & 1;
    for (int l = 0; l < mb; l++) {
        if (only && !only[l]) continue;
        int I = l & 3, J = (l >> 2) & 3, K = l >> 4;
        double x = -1.0 / 12.0 + I / 6.0 + 2.0 * cx / 3.0;
        double y = -1.0 / 12.0 + J / 6.0 + 2.0 * cy / 3.0;
        double z = -1.0 / 12.0 + K / 6.0 + 2.0 * cz / 3.0;
        for (int p = 0; p < q; p++) {
            double sum = 0.0;
            for (int e = 0; e < (dim == 3 ? 4 : 1); e++)
                for (int n = 0; n < 4; n++)
                    for (int m = 0; m < 4; m++) {
                        double wgt = lagrange3(m, x) * lagrange3(n, y) * (dim == 3 ? lagrange3(e, z) : 1.0);
                        sum += wgt * g[(m + 4 * n + 16 * e) * q + p];
                    }
            out[l * q + p] = sum;
        }
    }
}

static void interp_child_cells(int dim, int q, const double *g /* rescaled parent, Mb*q */, int child,
                               const unsigned char *only /* Mb flags or NULL */, double *out)
{
    int mb = dim == 2 ? 16 : 64;
    int cx = child & 1, cy = (child >> 1) & 1, cz = (child >> 2) & 1;
    for (int l = 0; l < mb; l++) {
        if (only && !only[l]) continue;
        int I = l & 3, J = (l >> 2) & 3, K = l >> 4;
        double x = -0.25 + 0.5 * I, y = -0.25 + 0.5 * J, z = -0.25 + 0.5 * K;
        for (int p = 0; p < q; p++) {
            double F[8];
            int ncorner = dim == 2 ? 4 : 8;
            for (int n = 0; n < ncorner; n++) {
                int a = n & 1, b = (n >> 1) & 1, e = (n >> 2) & 1;
                int m = (2 * cx + a) + 4 * (2 * cy + b) + 16 * (2 * cz + e);
                F[n] = g[m * q + p];
            }
            out[l * q + p] = linear_poly(dim, F, x, y, z);
        }
    }
}

static int interp_child_api(int dim, int q, double r, const double *parent, int child, double *out, int cubic)
{
    if (!lattice_ok(dim, q)) return -1;
    int mb = dim == 2 ? 16 : 64;
    double *g = (double *)malloc(sizeof(double) * mb * q);
    for (int m = 0; m < mb; m++) rescale_cell(dim, q, r, parent + m * q, g + m * q);
    if (cubic) interp_child_cells_cubic(dim, q, g, child, NULL, out);
    else interp_child_cells(dim, q, g, child, NULL, out);
    free(g);
    return 0;
}

int orc_interp_child(int dim, int q, double r, const double *parent, int child, double *out)
{
    return interp_child_api(dim, q, r, parent, child, out, 0);
}

int orc_interp_child_cubic(int dim, int q, double r, const double *parent, int child, double *out)
{
    return interp_child_api(dim, q, r, parent, child, out, 1);
}

/* Fine-to-coarse averaging (Sec. "Averaging").  Parent cell (i,j,k) takes the
 * mean of the 2^d rescaled fine cells of child octant (i/2, j/2, k/2) whose
 * first cell is (2(i mod 2), 2(j mod 2), 2(k mod 2)); the printed sum runs to
 * N_c and K' divides twice, both read as typos.  Cells are added in ascending
 * fine index. */
static void average_parent_cell(int dim, int q, double r, const double *child_f /* Mb*q of the child */,
                                int l_parent, double *out)
{
    int i = l_parent & 3, j = (l_parent >> 2) & 3, k = l_parent >> 4;
    int bi = 2 * (i & 1), bj = 2 * (j & 1), bk = 2 * (k & 1);
    int nc = dim == 2 ? 4 : 8;
    double acc[27];
    for (int p = 0; p < q; p++) acc[p] = 0.0;
    for (int n = 0; n < nc; n++) {
        int a = n & 1, b = (n >> 1) & 1, e = (n >> 2) & 1;
        int lf = (bi + a) + 4 * (bj + b) + 16 * (bk + e);
        double g[27];
        rescale_cell(dim, q, r, child_f + lf * q, g);
        for (int p = 0; p < q; p++) acc[p] += g[p];
    }
    for (int p = 0; p < q; p++) out[p] = acc[p] / nc;
}

static int child_of_parent_cell(int l_parent)
{
    int i = l_parent & 3, j = (l_parent >> 2) & 3, k = l_parent >> 4;
    return (i >> 1) + 2 * (j >> 1) + 4 * (k >> 1);
}

int orc_average_parent(int dim, int q, double r, const double *children, double *out)
{
    if (!lattice_ok(dim, q)) return -1;
    int mb = dim == 2 ? 16 : 64;
    for (int l = 0; l < mb; l++) {
        int c = child_of_parent_cell(l);
        average_parent_cell(dim, q, r, children + (size_t)c * mb * q, l, out + l * q);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Forest state (Sec. "Overview" and table of data structures). */
struct orc {
    orc_config cfg;
    uint8_t *solid;
    int dim, q, nb, mb, nc, cap, nroot, lmax;
    int dom[3];             /* domain extent in finest cells */
    int8_t *level, *status, *tag;
    int32_t *X;             /* cap*3 block origins */
    int32_t *nbr, *nbrc;    /* cap*nb */
    int32_t *ids[MAXL];
    int32_t nids[MAXL];
    int32_t *gap;
    int32_t gtop;
    double *f[2];           /* cap*mb*q, cell-major */
    int par[MAXL];          /* buffer holding the current data of each level */
    double tau[MAXL];
    double *crit;
    double *force;          /* cap*3 momentum exchange with solid blocks since the last reset */
    double sweeps[MAXL];    /* collide-stream sweeps of each level since the last reset */
    int coll;               /* 0 = BGK, 1 = moment-space (D3Q27) */
    double s_high;          /* rate of the moments above second order (coll = 1) */
};

static const int *bvec(const orc_t *o, int p) { return o->dim == 2 ? VEC2[p] : VEC3[p]; }

/* index of the neighbour direction with per-axis offsets (rx, ry, rz) */
static int dir_index(const orc_t *o, int rx, int ry, int rz)
{
    for (int p = 0; p < o->nb; p++) {
        const int *v = bvec(o, p);
        if (v[0] == rx && v[1] == ry && v[2] == rz) return p;
    }
    return -1;
}

static int width(const orc_t *o, int L) { return 4 << (o->lmax - 1 - L); }

static double *cellf(orc_t *o, int buf, int32_t B, int l)
{
    return o->f[buf] + ((size_t)B * o->mb + l) * o->q;
}

/* Relaxation per level (Sec. "Collision"): nu = cs^2 (tau - dt/2) with
 * dt_L = dt / 2^L gives tau*_L = 1/2 + 2^L (tau*_0 - 1/2). */
static void set_taus(orc_t *o)
{
    double tau0 = 0.5 + 3.0 * o->cfg.nu0;
    for (int L = 0; L < o->lmax; L++) o->tau[L] = 0.5 + (double)(1 << L) * (tau0 - 0.5);
}

/* rescaling ratios of Sec. "Linear Interpolation" / "Averaging": tau^F/tau^C
 * with the paper's dimensional tau (tau = tau* dt), i.e. tau*_F / (2 tau*_C). */
static double ratio_cf(const orc_t *o, int L)
{
    if (o->cfg.rescale_mode == 1) return o->tau[L + 1] / o->tau[L];
    return o->tau[L + 1] / (2.0 * o->tau[L]);
}
static double ratio_fc(const orc_t *o, int L)
{
    if (o->cfg.rescale_mode == 1) return o->tau[L] / o->tau[L + 1];
    return 2.0 * o->tau[L] / o->tau[L + 1];
}

int orc_ratios(orc_t *o, int32_t L, double *out2)
{
    if (L < 0 || L + 1 >= o->lmax) return -1;
    out2[0] = ratio_cf(o, L);
    out2[1] = ratio_fc(o, L);
    return 0;
}

/* Root-grid neighbour of root block (bi,bj,bk) in direction p (Sec. "Data
 * Structures": the root grid is structured, so its links are known).  Regions
 * outside the domain get the code of the highest-priority face they cross. */
static int32_t root_link(const orc_t *o, int bi, int bj, int bk, int p)
{
    const int *v = bvec(o, p);
    int r[3] = {bi + v[0], bj + v[1], bk + v[2]};
    int crossed[6] = {0, 0, 0, 0, 0, 0}, out = 0;
    for (int a = 0; a < o->dim; a++) {
        if (r[a] < 0) {
            if (o->cfg.periodic[a]) r[a] += o->cfg.root[a];
            else { crossed[2 * a] = 1; out = 1; }
        } else if (r[a] >= o->cfg.root[a]) {
            if (o->cfg.periodic[a]) r[a] -= o->cfg.root[a];
            else { crossed[2 * a + 1] = 1; out = 1; }
        }
    }
    if (out) {
        int best = -1;
        for (int fc = 0; fc < 6; fc++)
            if (crossed[fc] && (best < 0 || o->cfg.face_prio[fc] > o->cfg.face_prio[best])) best = fc;
        return FACE_CODE(best);
    }
    int32_t id = r[0] + o->cfg.root[0] * (r[1] + o->cfg.root[1] * r[2]);
    if (o->solid && o->solid[id]) return SOLID_CODE;
    return id;
}

static int is_refined(int8_t s)
{
    return s == ST_REFINED || s == ST_REFINED_CHILD || s == ST_REFINED_PERM;
}

orc_t *orc_create(const orc_config *cfg)
{
    if (!lattice_ok(cfg->dim, cfg->q) || cfg->lmax < 1 || cfg->lmax > MAXL) return NULL;
    if (cfg->interp != 0 && cfg->interp != 1) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->cfg = *cfg;
    o->dim = cfg->dim;
    o->q = cfg->q;
    o->nb = cfg->dim == 2 ? 9 : 27;
    o->mb = cfg->dim == 2 ? 16 : 64;
    o->nc = cfg->dim == 2 ? 4 : 8;
    o->lmax = cfg->lmax;
    o->nroot = cfg->root[0] * cfg->root[1] * (cfg->dim == 3 ? cfg->root[2] : 1);
    if (cfg->dim == 2) o->cfg.root[2] = 1;
    o->cap = cfg->cap;
    if (o->cap < o->nroot) { free(o); return NULL; }
    if (cfg->solid) {
        o->solid = (uint8_t *)malloc(o->nroot);
        memcpy(o->solid, cfg->solid, o->nroot);
    }
    o->cfg.solid = o->solid;
    for (int a = 0; a < 3; a++) o->dom[a] = o->cfg.root[a] * width(o, 0);
    size_t cap = (size_t)o->cap;
    o->level = (int8_t *)calloc(cap, 1);
    o->status = (int8_t *)calloc(cap, 1);
    o->tag = (int8_t *)calloc(cap, 1);
    o->X = (int32_t *)calloc(cap * 3, sizeof(int32_t));
    o->nbr = (int32_t *)calloc(cap * o->nb, sizeof(int32_t));
    o->nbrc = (int32_t *)calloc(cap * o->nb, sizeof(int32_t));
    for (int L = 0; L < o->lmax; L++) o->ids[L] = (int32_t *)malloc(cap * sizeof(int32_t));
    o->gap = (int32_t *)malloc(cap * sizeof(int32_t));
    o->f[0] = (double *)calloc(cap * o->mb * o->q, sizeof(double));
    o->f[1] = (double *)calloc(cap * o->mb * o->q, sizeof(double));
    o->crit = (double *)malloc(cap * sizeof(double));
    o->force = (double *)calloc((size_t)cap * 3, sizeof(double));
    set_taus(o);

    /* root grid: IDs in structured order, all leaves; the gap set holds
     * every other ID in reverse so that the smallest IDs are used first
     * (Sec. "Overview"). */
    for (int B = 0; B < o->cap; B++) o->status[B] = ST_INACTIVE;
    for (int bk = 0; bk < o->cfg.root[2]; bk++)
        for (int bj = 0; bj < o->cfg.root[1]; bj++)
            for (int bi = 0; bi < o->cfg.root[0]; bi++) {
                int32_t B = bi + o->cfg.root[0] * (bj + o->cfg.root[1] * bk);
                o->level[B] = 0;
                o->X[B * 3 + 0] = bi * width(o, 0);
                o->X[B * 3 + 1] = bj * width(o, 0);
                o->X[B * 3 + 2] = bk * width(o, 0);
                if (o->solid && o->solid[B]) continue;
                o->status[B] = ST_UNREFINED;
                for (int p = 0; p < o->nb; p++) {
                    int32_t n = root_link(o, bi, bj, bk, p);
                    o->nbr[B * o->nb + p] = n;
                    o->nbrc[B * o->nb + p] = n >= 0 ? NONE_ID : n;
                }
                o->ids[0][o->nids[0]++] = B;
            }
    o->gtop = 0;
    for (int32_t id = o->cap - 1; id >= o->nroot; id--) o->gap[o->gtop++] = id;

    /* f = feq(1, 0) everywhere until initial conditions are set */
    double u0[3] = {0, 0, 0}, feq[27];
    equilibrium(o->dim, o->q, 1.0, u0, feq);
    for (int b = 0; b < 2; b++)
        for (size_t n = 0; n < cap * o->mb; n++)
            for (int p = 0; p < o->q; p++) o->f[b][n * o->q + p] = feq[p];
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    free(o->solid); free(o->level); free(o->status); free(o->tag); free(o->X);
    free(o->nbr); free(o->nbrc); free(o->gap); free(o->f[0]); free(o->f[1]); free(o->crit); free(o->force);
    for (int L = 0; L < o->lmax; L++) free(o->ids[L]);
    free(o);
}

int32_t orc_parity(orc_t *o, int32_t L) { return (L >= 0 && L < o->lmax) ? o->par[L] : -1; }

int orc_set_root_rho_u(orc_t *o, const double *ru)
{
    for (int32_t B = 0; B < o->nroot; B++) {
        if (o->status[B] == ST_INACTIVE) continue;
        for (int l = 0; l < o->mb; l++) {
            const double *v = ru + ((size_t)B * o->mb + l) * 4;
            double u[3] = {v[1], v[2], v[3]};
            equilibrium(o->dim, o->q, v[0], u, cellf(o, o->par[0], B, l));
        }
    }
    return 0;
}

int orc_get_block_f(orc_t *o, int32_t B, double *out)
{
    if (B < 0 || B >= o->cap) return -1;
    memcpy(out, cellf(o, o->par[o->level[B]], B, 0), sizeof(double) * o->mb * o->q);
    return 0;
}

/* every active block's current data, [cap][Mb][q]; inactive blocks read 0 */
int orc_get_f_all(orc_t *o, double *out)
{
    size_t n = (size_t)o->mb * o->q;
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] == ST_INACTIVE) memset(out + B * n, 0, sizeof(double) * n);
        else memcpy(out + B * n, cellf(o, o->par[o->level[B]], B, 0), sizeof(double) * n);
    }
    return 0;
}

int orc_set_collision(orc_t *o, int kind, double s_high)
{
    if (kind == 0) {
        o->coll = 0;
        return 0;
    }
    if (kind != 1 || o->dim != 3 || o->q != 27 || !(s_high > 0.0 && s_high < 2.0)) return -1;
    if (mrt_init() != 0) return -1;
    o->coll = 1;
    o->s_high = s_high;
    return 0;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int orc_set_block_f(orc_t *o, int32_t B, const double *in)
{
    if (B < 0 || B >= o->cap) return -1;
    memcpy(cellf(o, o->par[o->level[B]], B, 0), in, sizeof(double) * o->mb * o->q);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cell classes (Sec. "Grid Communication"): the two layers of fine cells next
 * to a coarse-fine interface are ghosts, the next two are interface cells.
 * Reading for corners and edges: the Chebyshev distance from the cell to every
 * neighbour region whose link is N_SKIP, adjacent = 1. */
static int cell_class(const orc_t *o, int32_t B, int l)
{
    if (o->level[B] == 0) return CLS_INTERIOR;
    int ci[3] = {l & 3, (l >> 2) & 3, l >> 4};
    int d = 1 << 20;
    for (int p = 1; p < o->nb; p++) {
        if (o->nbr[B * o->nb + p] != N_SKIP) continue;
        const int *v = bvec(o, p);
        int dist = 0;
        for (int a = 0; a < o->dim; a++) {
            int da = v[a] == 1 ? 4 - ci[a] : (v[a] == -1 ? ci[a] + 1 : 0);
            if (da > dist) dist = da;
        }
        if (dist < d) d = dist;
    }
    if (d <= 2) return CLS_GHOST;
    if (d <= 4) return CLS_INTERFACE;
    return CLS_INTERIOR;
}

/* cell classes of block B (0 interior, 1 interface, 2 ghost), out[Mb] */
int orc_cell_classes(orc_t *o, int32_t B, int32_t *out)
{
    if (B < 0 || B >= o->cap || o->status[B] == ST_INACTIVE) return -1;
    for (int l = 0; l < o->mb; l++) out[l] = cell_class(o, B, l);
    return 0;
}

static int has_nskip(const orc_t *o, int32_t B)
{
    for (int p = 1; p < o->nb; p++)
        if (o->nbr[B * o->nb + p] == N_SKIP) return 1;
    return 0;
}

/* neighbour region of a cell position given in local cell coordinates that may
 * leave the block by one cell (-1 .. 4) */
static int region_of(const orc_t *o, const int *t, int *local_l)
{
    int r[3] = {0, 0, 0}, loc[3] = {0, 0, 0};
    for (int a = 0; a < 3; a++) {
        if (t[a] < 0) { r[a] = -1; loc[a] = t[a] + 4; }
        else if (t[a] > 3) { r[a] = 1; loc[a] = t[a] - 4; }
        else loc[a] = t[a];
    }
    if (local_l) *local_l = loc[0] + 4 * loc[1] + 16 * loc[2];
    return dir_index(o, r[0], r[1], r[2]);
}

/* Boundary conditions (Sec. "Lattice Boltzmann Method"), rho_w = 1:
 * known velocity  f_pbar = f*_p - 2 w_p rho_w (c_p.u_w)/cs^2,
 * outflow         f_pbar = -f*_p + 2 w_p rho_w (1 + (c_p.u_w)^2/(2cs^4) - u_w.u_w/(2cs^2)),
 * where the printed outflow term misses the square.  Solid blocks are walls at
 * rest; the outflow takes u_w as the cell's own velocity (Sec. "Flow Past a
 * Square Cylinder"). */
static double boundary_value(const orc_t *o, int32_t code, int p, double fstar, const double *u)
{
    const int *c = o->dim == 2 ? VEC2[p] : VEC3[p];
    double w = lattice_weight(o->dim, o->q, p);
    if (code == SOLID_CODE) return fstar;
    int face = -3 - code;
    if (o->cfg.face_kind[face] == 0) {
        const double *uw = o->cfg.face_u[face];
        double cu = c[0] * uw[0] + c[1] * uw[1] + c[2] * uw[2];
        return fstar - 6.0 * w * 1.0 * cu;
    }
    double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return -fstar + 2.0 * w * 1.0 * (1.0 + 4.5 * cu * cu - 1.5 * uu);
}

/* One collide-and-stream sweep of level L over every block of id_set_L (Secs.
 * "Grid Advancement", "Streaming", "Collision"), in two-buffer push form:
 * f_p(x + c_p) <- f*_p(x).  Links leaving the fluid get the boundary value in
 * the opposite slot of the same cell; populations that would arrive from a
 * region covered only by a coarser block are not streamed, and the cell keeps
 * its own post-collision value in that slot (such cells are ghosts). */
/* The momentum exchange with solid blocks (Sec. "Flow Past a Square
 * Cylinder"): every post-collision population f*_p of a leaf cell whose link
 * c_p ends in a solid block is reflected, passing 2 f*_p c_p to the solid.
 * Summed per block over the sweeps since the last reset, in lattice units of
 * the block's level. */
static void collide_stream_level(orc_t *o, int L)
{
    int src = o->par[L], dst = 1 - o->par[L];
    double omega = 1.0 / o->tau[L];
    int q = o->q, nb = o->nb;
    o->sweeps[L] += 1.0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t n = 0; n < o->nids[L]; n++) {
        int32_t B = o->ids[L][n];
        int leaf = o->status[B] == ST_UNREFINED;
        for (int l = 0; l < o->mb; l++) {
            int ci[3] = {l & 3, (l >> 2) & 3, l >> 4};
            const double *fc = cellf(o, src, B, l);
            double rho, u[3], feq[27], fs[27];
            moments(o->dim, q, fc, &rho, u);
            equilibrium(o->dim, q, rho, u, feq);
            if (o->coll == 1)
                mrt_relax(fc, feq, omega, o->s_high, fs);
            else
                for (int p = 0; p < q; p++) fs[p] = (1.0 - omega) * fc[p] + omega * feq[p];
            double *own = cellf(o, dst, B, l);
            for (int p = 0; p < q; p++) {
                const int *c = o->dim == 2 ? VEC2[p] : VEC3[p];
                int t[3] = {ci[0] + c[0], ci[1] + c[1], ci[2] + c[2]};
                int lt;
                int reg = region_of(o, t, &lt);
                int32_t code = o->nbr[B * nb + reg];
                if (code >= 0) {
                    cellf(o, dst, code, lt)[p] = fs[p];
                } else if (code != N_SKIP && code != NONE_ID) {
                    int pb = lattice_opposite(o->dim, p);
                    own[pb] = boundary_value(o, code, p, fs[p], u);
                    if (code == SOLID_CODE && leaf)
                        for (int a = 0; a < 3; a++) o->force[(size_t)B * 3 + a] += 2.0 * fs[p] * c[a];
                }
            }
            for (int p = 0; p < q; p++) {
                const int *c = o->dim == 2 ? VEC2[p] : VEC3[p];
                int s[3] = {ci[0] - c[0], ci[1] - c[1], ci[2] - c[2]};
                int reg = region_of(o, s, NULL);
                if (o->nbr[B * nb + reg] == N_SKIP) own[p] = fs[p];
            }
        }
    }
    o->par[L] = dst;
}

/* Interpolation from level L to the children of its refined blocks.
 * all_cells = 0: ghost cells of children with an N_SKIP link (start of each
 * step on level L); the whole child when it is newly created. */
static void interp_parent(orc_t *o, int L, int32_t P, int all_cells)
{
    int q = o->q, mb = o->mb;
    double r = ratio_cf(o, L);
    double *g = (double *)malloc(sizeof(double) * mb * q);
    for (int m = 0; m < mb; m++) rescale_cell(o->dim, q, r, cellf(o, o->par[L], P, m), g + m * q);
    int32_t first = o->nbrc[P * o->nb + 0];
    for (int c = 0; c < o->nc; c++) {
        int32_t ch = first + c;
        unsigned char sel[64];
        if (!all_cells) {
            if (!has_nskip(o, ch)) continue;
            for (int l = 0; l < mb; l++) sel[l] = cell_class(o, ch, l) == CLS_GHOST;
        }
        double *out = (double *)malloc(sizeof(double) * mb * q);
        memcpy(out, cellf(o, o->par[L + 1], ch, 0), sizeof(double) * mb * q);
        if (o->cfg.interp == 1) interp_child_cells_cubic(o->dim, q, g, c, all_cells ? NULL : sel, out);
        else interp_child_cells(o->dim, q, g, c, all_cells ? NULL : sel, out);
        memcpy(cellf(o, o->par[L + 1], ch, 0), out, sizeof(double) * mb * q);
        free(out);
    }
    free(g);
}

static void interp_level(orc_t *o, int L)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t n = 0; n < o->nids[L]; n++) {
        int32_t P = o->ids[L][n];
        if (is_refined(o->status[P])) interp_parent(o, L, P, 0);
    }
}

/* Averaging from level L+1 to the refined blocks of level L: parent cells
 * whose children are interface cells (end of each step on level L), or every
 * parent cell (pre-adaptation synchronisation). */
static void average_level(orc_t *o, int L, int all_cells)
{
    int q = o->q, mb = o->mb;
    double r = ratio_fc(o, L);
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t n = 0; n < o->nids[L]; n++) {
        int32_t P = o->ids[L][n];
        if (!is_refined(o->status[P])) continue;
        int32_t first = o->nbrc[P * o->nb + 0];
        for (int l = 0; l < mb; l++) {
            int c = child_of_parent_cell(l);
            int32_t ch = first + c;
            if (!all_cells) {
                int i = l & 3, j = (l >> 2) & 3, k = l >> 4;
                int lf = 2 * (i & 1) + 4 * 2 * (j & 1) + 16 * 2 * (k & 1);
                if (cell_class(o, ch, lf) != CLS_INTERFACE) continue;
            }
            average_parent_cell(o->dim, q, r, cellf(o, o->par[L + 1], ch, 0), l, cellf(o, o->par[L], P, l));
        }
    }
}

/* Recursive sub-cycled advancement (Sec. "Grid Advancement"): interpolate to
 * the ghosts of level L+1, step level L, two steps of level L+1, average the
 * interface cells back. */
static void step_level(orc_t *o, int L)
{
    if (L == o->lmax - 1) {
        collide_stream_level(o, L);
        return;
    }
    interp_level(o, L);
    collide_stream_level(o, L);
    step_level(o, L + 1);
    step_level(o, L + 1);
    average_level(o, L, 0);
}

/* one collide-and-stream sweep of level L alone (timing of the CPU
 * baseline): the level's buffer advances, the forest is left mid-step */
int orc_sweep(orc_t *o, int32_t L)
{
    if (L < 0 || L >= o->lmax) return -1;
    collide_stream_level(o, L);
    return 0;
}

int orc_step(orc_t *o, int32_t n)
{
    for (int32_t s = 0; s < n; s++) step_level(o, 0);
    return 0;
}

/* Pre-adaptation synchronisation (Sec. "Adaptive Mesh Refinement" of the
 * solver): average every parent cell from level L_max-2 up to 0, then fill the
 * ghosts of every level from level 0 down. */
int orc_sync(orc_t *o)
{
    for (int L = o->lmax - 2; L >= 0; L--) average_level(o, L, 1);
    for (int L = 0; L <= o->lmax - 2; L++) interp_level(o, L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Refinement criterion: vorticity magnitude per cell, block maximum (same
 * section).  Gradients use central differences between same-level neighbour
 * cells and one-sided differences where a neighbour is missing; derivatives
 * are taken in root-cell units (factor 2^L). */
static int cell_velocity(orc_t *o, int32_t B, const int *t, double *u)
{
    int lt;
    int reg = region_of(o, t, &lt);
    int32_t code = o->nbr[B * o->nb + reg];
    if (code < 0) return 0;
    double rho;
    moments(o->dim, o->q, cellf(o, o->par[o->level[code]], code, lt), &rho, u);
    return 1;
}

static double cell_vorticity(orc_t *o, int32_t B, int l)
{
    int ci[3] = {l & 3, (l >> 2) & 3, l >> 4};
    double u0[3], rho;
    moments(o->dim, o->q, cellf(o, o->par[o->level[B]], B, l), &rho, u0);
    double g[3][3] = {{0}}; /* g[a][b] = d u_b / d x_a */
    for (int a = 0; a < o->dim; a++) {
        int tp[3] = {ci[0], ci[1], ci[2]}, tm[3] = {ci[0], ci[1], ci[2]};
        tp[a] += 1;
        tm[a] -= 1;
        double up[3], um[3];
        int hp = cell_velocity(o, B, tp, up);
        int hm = cell_velocity(o, B, tm, um);
        for (int b = 0; b < 3; b++) {
            if (hp && hm) g[a][b] = (up[b] - um[b]) / 2.0;
            else if (hp) g[a][b] = up[b] - u0[b];
            else if (hm) g[a][b] = u0[b] - um[b];
            else g[a][b] = 0.0;
        }
    }
    double scale = (double)(1 << o->level[B]);
    if (o->dim == 2) return fabs(g[0][1] - g[1][0]) * scale;
    double wx = g[1][2] - g[2][1], wy = g[2][0] - g[0][2], wz = g[0][1] - g[1][0];
    return sqrt(wx * wx + wy * wy + wz * wz) * scale;
}

/* squared distance (finest cells) between the box of block B and the nearest
 * solid root block or outflow face */
static double block_wall_distance2(orc_t *o, int32_t B)
{
    int W = width(o, o->level[B]);
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) { lo[a] = o->X[B * 3 + a]; hi[a] = lo[a] + (a < o->dim ? W : 0); }
    double best = -1.0;
    if (o->solid) {
        int W0 = width(o, 0);
        for (int32_t s = 0; s < o->nroot; s++) {
            if (!o->solid[s]) continue;
            int64_t d2 = 0;
            for (int a = 0; a < o->dim; a++) {
                int slo = o->X[s * 3 + a], shi = slo + W0;
                int64_t gap = 0;
                if (hi[a] < slo) gap = slo - hi[a];
                else if (shi < lo[a]) gap = lo[a] - shi;
                d2 += gap * gap;
            }
            if (best < 0 || (double)d2 < best) best = (double)d2;
        }
    }
    for (int fc = 0; fc < 2 * o->dim; fc++) {
        if (o->cfg.face_kind[fc] != 1) continue;
        int a = fc / 2;
        int64_t gap = (fc & 1) ? (int64_t)(o->dom[a] - hi[a]) : (int64_t)lo[a];
        double d2 = (double)(gap * gap);
        if (best < 0 || d2 < best) best = d2;
    }
    return best;
}

/* Eligibility of a tag and the 2:1 refine-cancel (Secs. "Adaptive Mesh
 * Refinement" and "Enforcement of 2:1 Balancing"): refinement only of leaves
 * below L_max-1 with no N_SKIP link; coarsening only of refined blocks whose
 * children are all leaves and that are not permanent. */
static int8_t effective_tag(const orc_t *o, int32_t B, int8_t t)
{
    if (o->status[B] == ST_INACTIVE) return TAG_NONE;
    if (t == TAG_REFINE || t == TAG_REFINE_PERM) {
        if (o->status[B] != ST_UNREFINED || o->level[B] >= o->lmax - 1) return TAG_NONE;
        if (has_nskip(o, B)) return TAG_NONE;
        return t;
    }
    if (t == TAG_COARSEN) return o->status[B] == ST_REFINED ? TAG_COARSEN : TAG_NONE;
    return TAG_NONE;
}

/* Desired level of a block from its maximum vorticity (Sec. "Adaptive Mesh
 * Refinement" of the solver, Alg. 3): epsilon = min(1, log2 |w|); the level
 * starts at L_max - 1 and becomes (L_max - 1) - p for every p = 1 .. L_max - 1
 * (in increasing order) with epsilon < N_start - p N_inc.  Reading: |w| is in
 * the units of the paper's physical set-ups, domain length 1 along x and
 * dx = dt = 1/N_x, i.e. N_x times the root-lattice vorticity. */
static int ladder_level(double w, int lmax, double n_start, double n_inc)
{
    double eps = log2(w);
    if (eps > 1.0) eps = 1.0;
    int ldes = lmax - 1;
    for (int p = 1; p <= lmax - 1; p++)
        if (eps < n_start - p * n_inc) ldes = (lmax - 1) - p;
    return ldes;
}

int orc_tag(orc_t *o, const orc_tag_params *prm, const int8_t *tags_in, int8_t *tags_out)
{
    orc_sync(o);
    int8_t *raw = (int8_t *)calloc(o->cap, 1);
    for (int32_t B = 0; B < o->cap; B++) o->crit[B] = -1.0;
    if (tags_in) {
        memcpy(raw, tags_in, o->cap);
    } else if (prm->kind == 0 || prm->kind == 2) {
        double wmax = 0.0;
        for (int L = 0; L < o->lmax; L++) {
#pragma omp parallel for schedule(dynamic, 16)
            for (int32_t n = 0; n < o->nids[L]; n++) {
                int32_t B = o->ids[L][n];
                if (o->status[B] != ST_UNREFINED) continue;
                double m = 0.0;
                for (int l = 0; l < o->mb; l++) {
                    double w = cell_vorticity(o, B, l);
                    if (w > m) m = w;
                }
                o->crit[B] = m;
            }
        }
        for (int32_t B = 0; B < o->cap; B++)
            if (o->crit[B] > wmax) wmax = o->crit[B];
        double thr = prm->theta * wmax;
        double nx = 4.0 * o->cfg.root[0]; /* domain length along x in root cells */
        int8_t *ldes = (int8_t *)calloc(o->cap, 1);
        for (int32_t B = 0; B < o->cap; B++) {
            if (o->status[B] != ST_UNREFINED) continue;
            if (prm->kind == 0)
                ldes[B] = o->crit[B] > thr ? (int8_t)(o->lmax - 1) : 0;
            else
                ldes[B] = (int8_t)ladder_level(o->crit[B] * nx, o->lmax, prm->n_start, prm->n_inc);
            if (ldes[B] > o->level[B]) raw[B] = TAG_REFINE;
        }
        for (int32_t P = 0; P < o->cap; P++) {
            if (o->status[P] != ST_REFINED) continue;
            int32_t first = o->nbrc[P * o->nb];
            int mx = 0;
            for (int c = 0; c < o->nc; c++)
                if (ldes[first + c] > mx) mx = ldes[first + c];
            if (mx <= o->level[P]) raw[P] = TAG_COARSEN;
        }
        free(ldes);
    } else {
        double dspec = prm->d_spec * (double)(1 << (o->lmax - 1));
        for (int32_t B = 0; B < o->cap; B++) {
            if (o->status[B] != ST_UNREFINED) continue;
            double thr = dspec / (double)(1 << o->level[B]);
            double d2 = block_wall_distance2(o, B);
            if (d2 >= 0.0 && d2 < thr * thr) raw[B] = prm->freeze ? TAG_REFINE_PERM : TAG_REFINE;
        }
    }
    for (int32_t B = 0; B < o->cap; B++) o->tag[B] = effective_tag(o, B, raw[B]);
    if (tags_out) memcpy(tags_out, o->tag, o->cap);
    free(raw);
    return 0;
}

int orc_get_crit(orc_t *o, double *out)
{
    memcpy(out, o->crit, sizeof(double) * o->cap);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Refinement and coarsening (Sec. "Refinement and Coarsening", Algs. 1-2),
 * applied to all levels at once.  Deterministic readings of the ordering the
 * paper leaves open: refine-marked blocks take gaps in ascending block ID from
 * the top of the gap stack; freed children are pushed back in reverse order of
 * (parent level, parent ID, child index); ID sets drop removed IDs stably and
 * append new children in (parent ID, child index) order. */
static void reset_force(orc_t *o)
{
    memset(o->force, 0, sizeof(double) * 3 * (size_t)o->cap);
    for (int L = 0; L < MAXL; L++) o->sweeps[L] = 0.0;
}

/* Per level: force on the solid blocks summed over the active blocks of that
 * level (x, y, z, in that level's lattice units, summed over its sweeps) and
 * the number of sweeps since the last reset. */
int orc_force(orc_t *o, double *out /* [lmax][4] */, int reset)
{
    for (int L = 0; L < o->lmax; L++)
        for (int a = 0; a < 4; a++) out[L * 4 + a] = 0.0;
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] == ST_INACTIVE) continue;
        for (int a = 0; a < 3; a++) out[o->level[B] * 4 + a] += o->force[(size_t)B * 3 + a];
    }
    for (int L = 0; L < o->lmax; L++) out[L * 4 + 3] = o->sweeps[L];
    if (reset) reset_force(o);
    return 0;
}

int orc_adapt(orc_t *o, int32_t *stats)
{
    int nb = o->nb, nc = o->nc;
    int32_t n_ref = 0, n_coa = 0, n_rev = 0;
    /* Preparation: effective tags (idempotent) and counts */
    for (int32_t B = 0; B < o->cap; B++) {
        o->tag[B] = effective_tag(o, B, o->tag[B]);
        if (o->tag[B] == TAG_REFINE || o->tag[B] == TAG_REFINE_PERM) n_ref++;
        if (o->tag[B] == TAG_COARSEN) n_coa++;
    }
    if (stats) { stats[0] = n_ref; stats[1] = n_coa; stats[2] = 0; stats[3] = 0; }
    if (n_ref == 0 && n_coa == 0) return 0;
    if ((int64_t)nc * n_ref > o->gtop) return -2; /* capacity: nothing changed */
    reset_force(o); /* blocks are created and removed: the force sums restart */

    /* S2: map gaps to refine-marked blocks */
    int32_t *first = (int32_t *)malloc(sizeof(int32_t) * o->cap);
    int32_t r = 0;
    for (int32_t B = 0; B < o->cap; B++) {
        first[B] = -1;
        if (o->tag[B] == TAG_REFINE || o->tag[B] == TAG_REFINE_PERM) {
            first[B] = o->gap[o->gtop - 1 - nc * r];
            r++;
        }
    }
    o->gtop -= nc * n_ref;

    /* S3: 2:1 balance.  A leaf is violating if any provisional neighbour-child
     * (including this call's new children, and itself at p = 0) is valid; a
     * coarsen-marked parent with a violating child is reverted. */
    int8_t *viol = (int8_t *)calloc(o->cap, 1);
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] != ST_UNREFINED) continue;
        for (int p = 0; p < nb; p++) {
            int32_t n = o->nbr[B * nb + p];
            int32_t pc = (n >= 0 && first[n] >= 0) ? first[n] : o->nbrc[B * nb + p];
            if (p == 0) pc = first[B] >= 0 ? first[B] : o->nbrc[B * nb];
            if (pc >= 0) { viol[B] = 1; break; }
        }
    }
    for (int32_t P = 0; P < o->cap; P++) {
        if (o->tag[P] != TAG_COARSEN) continue;
        int32_t c0 = o->nbrc[P * nb];
        for (int c = 0; c < nc; c++)
            if (viol[c0 + c]) { o->tag[P] = TAG_NONE; n_rev++; break; }
    }
    n_coa -= n_rev;
    free(viol);

    /* S4: build new children (level, status, coordinates) */
    int8_t *is_new = (int8_t *)calloc(o->cap, 1);
    for (int32_t P = 0; P < o->cap; P++) {
        if (first[P] < 0) continue;
        int L = o->level[P] + 1;
        for (int c = 0; c < nc; c++) {
            int32_t ch = first[P] + c;
            o->level[ch] = (int8_t)L;
            o->status[ch] = ST_NEW;
            o->nbrc[ch * nb] = NONE_ID;
            is_new[ch] = 1;
            int cv[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            for (int a = 0; a < 3; a++) o->X[ch * 3 + a] = o->X[P * 3 + a] + cv[a] * width(o, L);
        }
    }

    /* S5: coarsen in ID sets, push freed groups onto the gap stack */
    int32_t *freed = (int32_t *)malloc(sizeof(int32_t) * o->cap);
    int32_t nfreed = 0;
    int8_t *removed = (int8_t *)calloc(o->cap, 1);
    for (int L = 0; L < o->lmax; L++)
        for (int32_t P = 0; P < o->cap; P++) {
            if (o->tag[P] != TAG_COARSEN || o->level[P] != L) continue;
            int32_t c0 = o->nbrc[P * nb];
            for (int c = 0; c < nc; c++) {
                freed[nfreed++] = c0 + c;
                removed[c0 + c] = 1;
                o->status[c0 + c] = ST_REMOVE;
            }
        }
    for (int L = 1; L < o->lmax; L++) {
        int32_t m = 0;
        for (int32_t n = 0; n < o->nids[L]; n++)
            if (!removed[o->ids[L][n]]) o->ids[L][m++] = o->ids[L][n];
        o->nids[L] = m;
    }
    for (int32_t k = nfreed - 1; k >= 0; k--) o->gap[o->gtop++] = freed[k];

    /* S6: refine in ID sets */
    for (int L = 0; L < o->lmax - 1; L++)
        for (int32_t P = 0; P < o->cap; P++) {
            if (first[P] < 0 || o->level[P] != L) continue;
            for (int c = 0; c < nc; c++) o->ids[L + 1][o->nids[L + 1]++] = first[P] + c;
        }

    /* first-child links of blocks whose status changes (neighbour-child p = 0) */
    for (int32_t P = 0; P < o->cap; P++) {
        if (first[P] >= 0) o->nbrc[P * nb] = first[P];
        if (o->tag[P] == TAG_COARSEN) o->nbrc[P * nb] = NONE_ID;
    }

    /* S7: interpolate to the new children from their parents' data, then
     * finalise statuses and branch/leaf */
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t P = 0; P < o->cap; P++)
        if (first[P] >= 0) interp_parent(o, o->level[P], P, 1);
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->tag[B] == TAG_REFINE) o->status[B] = ST_REFINED;
        else if (o->tag[B] == TAG_REFINE_PERM) o->status[B] = ST_REFINED_PERM;
        else if (o->tag[B] == TAG_COARSEN) o->status[B] = ST_UNREFINED;
        if (o->status[B] == ST_NEW) o->status[B] = ST_UNREFINED;
        else if (o->status[B] == ST_REMOVE) o->status[B] = ST_INACTIVE;
    }
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] != ST_REFINED && o->status[B] != ST_REFINED_CHILD) continue;
        int32_t c0 = o->nbrc[B * nb];
        int any = 0;
        for (int c = 0; c < nc; c++)
            if (is_refined(o->status[c0 + c])) any = 1;
        o->status[B] = any ? ST_REFINED_CHILD : ST_REFINED;
    }

    /* S8: connectivity, level by level from the root.  Neighbour-children of
     * level L come from its links; links of the children of level L follow
     * from their parent's neighbour-children (Alg. 2): for child c and
     * direction p, t = c + p in {-1..2}^d, the parent region q = floor(t/2)
     * and the child index c' = t mod 2 inside that region. */
    for (int L = 0; L < o->lmax; L++) {
        for (int32_t n = 0; n < o->nids[L]; n++) {
            int32_t B = o->ids[L][n];
            for (int p = 1; p < nb; p++) {
                int32_t nn = o->nbr[B * nb + p];
                o->nbrc[B * nb + p] = nn >= 0 ? o->nbrc[nn * nb] : nn;
            }
        }
        if (L == o->lmax - 1) break;
        for (int32_t n = 0; n < o->nids[L]; n++) {
            int32_t P = o->ids[L][n];
            if (!is_refined(o->status[P])) continue;
            int32_t c0 = o->nbrc[P * nb];
            for (int c = 0; c < nc; c++) {
                int cv[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
                int32_t ch = c0 + c;
                for (int p = 0; p < nb; p++) {
                    const int *v = bvec(o, p);
                    int qv[3] = {0, 0, 0}, cc[3] = {0, 0, 0};
                    for (int a = 0; a < o->dim; a++) {
                        int t = cv[a] + v[a];
                        qv[a] = t < 0 ? -1 : t / 2;
                        cc[a] = t - 2 * qv[a];
                    }
                    int qd = dir_index(o, qv[0], qv[1], qv[2]);
                    int32_t X = o->nbrc[P * nb + qd];
                    int32_t link;
                    if (X >= 0) link = X + cc[0] + 2 * cc[1] + 4 * cc[2];
                    else if (X == NONE_ID || X == N_SKIP) link = N_SKIP;
                    else link = X;
                    o->nbr[ch * nb + p] = link;
                }
            }
        }
    }
    for (int32_t B = 0; B < o->cap; B++) o->tag[B] = TAG_NONE;
    free(first); free(is_new); free(freed); free(removed);
    if (stats) { stats[0] = n_ref; stats[1] = n_coa; stats[2] = n_rev; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Output: every leaf, non-ghost cell of an active block, in (block ID, cell)
 * order: rho, u and f. */
int64_t orc_n_out(orc_t *o)
{
    int64_t n = 0;
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] != ST_UNREFINED) continue;
        for (int l = 0; l < o->mb; l++)
            if (cell_class(o, B, l) != CLS_GHOST) n++;
    }
    return n;
}

int orc_get_out(orc_t *o, int32_t *blk, int32_t *cell, double *rho, double *u3, double *f)
{
    int64_t n = 0;
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] != ST_UNREFINED) continue;
        for (int l = 0; l < o->mb; l++) {
            if (cell_class(o, B, l) == CLS_GHOST) continue;
            const double *fc = cellf(o, o->par[o->level[B]], B, l);
            double r, u[3];
            moments(o->dim, o->q, fc, &r, u);
            if (blk) blk[n] = B;
            if (cell) cell[n] = l;
            if (rho) rho[n] = r;
            if (u3) for (int a = 0; a < 3; a++) u3[n * 3 + a] = u[a];
            if (f) memcpy(f + n * o->q, fc, sizeof(double) * o->q);
            n++;
        }
    }
    return 0;
}

/* mass and momentum of the output cells, each weighted by its volume in root
 * cells (2^-dL) */
int orc_mass_mom(orc_t *o, double *out4)
{
    double m = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int32_t B = 0; B < o->cap; B++) {
        if (o->status[B] != ST_UNREFINED) continue;
        double vol = 1.0 / (double)(1 << (o->dim * o->level[B]));
        for (int l = 0; l < o->mb; l++) {
            if (cell_class(o, B, l) == CLS_GHOST) continue;
            double r, u[3];
            moments(o->dim, o->q, cellf(o, o->par[o->level[B]], B, l), &r, u);
            m += vol * r;
            for (int a = 0; a < 3; a++) j[a] += vol * r * u[a];
        }
    }
    out4[0] = m;
    for (int a = 0; a < 3; a++) out4[1 + a] = j[a];
    return 0;
}

int orc_get_mesh(orc_t *o, int8_t *level, int8_t *status, int32_t *X3, int32_t *nbr, int32_t *nbrc,
                 int32_t *n_ids, int32_t *ids, int32_t *gtop, int32_t *gap)
{
    size_t cap = (size_t)o->cap;
    if (level) memcpy(level, o->level, cap);
    if (status) memcpy(status, o->status, cap);
    if (X3) memcpy(X3, o->X, cap * 3 * sizeof(int32_t));
    if (nbr) memcpy(nbr, o->nbr, cap * o->nb * sizeof(int32_t));
    if (nbrc) memcpy(nbrc, o->nbrc, cap * o->nb * sizeof(int32_t));
    for (int L = 0; L < o->lmax; L++) {
        if (n_ids) n_ids[L] = o->nids[L];
        if (ids) memcpy(ids + L * cap, o->ids[L], o->nids[L] * sizeof(int32_t));
    }
    if (gtop) *gtop = o->gtop;
    if (gap) memcpy(gap, o->gap, o->gtop * sizeof(int32_t));
    return 0;
}
