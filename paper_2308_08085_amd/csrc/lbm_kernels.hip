// lbm_kernels.hip -- lattice Boltzmann kernels of the AMR-LBM library for
// gfx950: fused BGK collide + stream per level sweep, coarse-to-fine linear
// interpolation, fine-to-coarse averaging, the vorticity criterion and field
// gathers.  Arithmetic is written in the shifted variables g = f - w for every
// storage format (FP64 storage computes in FP64, the rest in FP32).
//
// Distributions are stored source-indexed in block-major rows (see common.h):
// every kernel finds population p of a cell with entry_slot().
#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace amr {

template <typename Lt>
__device__ __forceinline__ int64_t mslot(int B, int p, int l) {
    return ((int64_t)B * Lt::Q + p) * Lt::MB + l;
}

template <typename Lt>
__device__ __forceinline__ int dir_region(int p) {
    return offset_slot(Lt::cx(p), Lt::cy(p), Lt::cz(p)) - (Lt::D == 2 ? 9 : 0);
}

// slot holding population p of cell l of block B (h = its halo record); link
// is the block's link table in region-slot order
template <typename Lt>
__device__ __forceinline__ int64_t entry_slot(const DevMesh &m, const int32_t *link, int B, int h, int p, int l) {
    const int sx = (l & 3) - Lt::cx(p), sy = ((l >> 2) & 3) - Lt::cy(p), sz = (l >> 4) - Lt::cz(p);
    const int32_t code = link[region_of<Lt>(sx, sy, sz)];
    if (code >= 0 && code < m.cap) return mslot<Lt>(code, p, (sx & 3) + 4 * (sy & 3) + 16 * (sz & 3));
    if (code == kNSkip && h >= 0) return m.halo_base + (int64_t)h * m.nh + kHalo<Lt>.idx[p][l];
    return mslot<Lt>(B, Lt::opp(p), l);
}

template <typename Lt, typename R>
__device__ inline void moments_g(const R *g, R &drho, R &ux, R &uy, R &uz) {
    R d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) {
        d += g[p];
        if (Lt::cx(p) > 0) jx += g[p]; else if (Lt::cx(p) < 0) jx -= g[p];
        if (Lt::cy(p) > 0) jy += g[p]; else if (Lt::cy(p) < 0) jy -= g[p];
        if (Lt::cz(p) > 0) jz += g[p]; else if (Lt::cz(p) < 0) jz -= g[p];
    }
    const R rho = R(1) + d;
    drho = d;
    ux = jx / rho;
    uy = jy / rho;
    uz = jz / rho;
}

// a b + c, rounded once
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// deviation of the second-order equilibrium from the rest state over the
// weight: (rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u), so g_eq = w y.
// Callers fuse the weight into the difference with g (one rounding fewer).
template <typename Lt, typename R>
__device__ inline R geq_y(int p, R drho, R ux, R uy, R uz, R uu) {
    const R cu = R(Lt::cx(p)) * ux + R(Lt::cy(p)) * uy + R(Lt::cz(p)) * uz;
    const R rho = R(1) + drho;
    return drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
}

// g_eq + r (g - g_eq): the non-equilibrium part rescaled by r
template <typename Lt, typename R>
__device__ __forceinline__ R rescale_neq(int p, R g, R r, R drho, R ux, R uy, R uz, R uu) {
    const R w = R(Lt::w(p)), y = geq_y<Lt, R>(p, drho, ux, uy, uz, uu);
    return fmadd(w, y, r * fmadd(-w, y, g));
}

// RAW: the stored value itself, also for unshifted storage
template <typename Lt, typename ST, bool RAW = false>
__device__ __forceinline__ typename ST::R load_g(const typename ST::T *f, int64_t slot, int p) {
    using R = typename ST::R;
    const R v = ST::ld(f + slot);
    return (ST::shift || RAW) ? v : v - R(Lt::w(p));
}

template <typename Lt, typename ST, bool NT = false>
__device__ __forceinline__ void store_g(typename ST::T *f, int64_t slot, int p, typename ST::R g) {
    using R = typename ST::R;
    if constexpr (NT)
        ST::stnt(f + slot, ST::shift ? g : g + R(Lt::w(p)));
    else
        ST::st(f + slot, ST::shift ? g : g + R(Lt::w(p)));
}

// gather / scatter all populations of one cell
template <typename Lt, typename ST, bool RAW = false>
__device__ __forceinline__ void gather_cell(const DevMesh &m, const int32_t *link, int B, int h, int l,
                                            const typename ST::T *f, typename ST::R *g) {
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) g[p] = load_g<Lt, ST, RAW>(f, entry_slot<Lt>(m, link, B, h, p, l), p);
}

// The same for a block whose only links outside the fluid are domain faces or
// solid blocks (no coarser neighbour): each population comes from a same-level
// block or from the cell's own opposite slot, a select between two addresses
// rather than a branch per population.
template <typename Lt, typename ST, bool RAW = false>
__device__ __forceinline__ void gather_cell_nohalo(const DevMesh &m, const int32_t *link, int B, int l,
                                                   const typename ST::T *f, typename ST::R *g) {
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) {
        const int sx = (l & 3) - Lt::cx(p), sy = ((l >> 2) & 3) - Lt::cy(p), sz = (l >> 4) - Lt::cz(p);
        const int32_t code = link[region_of<Lt>(sx, sy, sz)];
        const bool in = code >= 0 && code < m.cap;
        const int blk = in ? code : B;
        const int q = in ? p : Lt::opp(p);
        const int cell = in ? (sx & 3) + 4 * (sy & 3) + 16 * (sz & 3) : l;
        g[p] = load_g<Lt, ST, RAW>(f, mslot<Lt>(blk, q, cell), p);
    }
}

// gather of a cell of a block with flags `flag`: the select form unless the
// block has a coarser neighbour
template <typename Lt, typename ST, bool RAW = false>
__device__ __forceinline__ void gather_cell_flag(const DevMesh &m, const int32_t *link, int B, int h, uint8_t flag,
                                                 int l, const typename ST::T *f, typename ST::R *g) {
    if (flag & BF_NSKIP)
        gather_cell<Lt, ST, RAW>(m, link, B, h, l, f, g);
    else
        gather_cell_nohalo<Lt, ST, RAW>(m, link, B, l, f, g);
}

template <typename Lt, typename ST>
__device__ __forceinline__ void scatter_cell(const DevMesh &m, const int32_t *link, int B, int h, int l,
                                             typename ST::T *f, const typename ST::R *g) {
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) store_g<Lt, ST>(f, entry_slot<Lt>(m, link, B, h, p, l), p, g[p]);
}

// Gather of an interior 3-D block (every region link a same-level block; one
// block per wave) through a per-wave LDS table of its 27 region rows.
//
// Population p of cell (i, j, k) comes from cell s = (i, j, k) - c_p, which
// lies in region r = floor(s / 4) (per axis -1, 0 or +1) at local cell s - 4 r.
// Its address is row(r) + p Mb + (s - 4 r) . (1, 4, 16), i.e.
//     tab[r] + own + (p Mb - c_p . (1, 4, 16))   (in elements)
// with tab[r] = row(r) - 4 r . (1, 4, 16) stored per region, own = the
// lane's cell index, and the last term a constant of p.  The region offset
// along x is -1 only for c_x = +1 on the face i = 0 and +1 only for c_x = -1 on
// i = 3, so each lane keeps one table offset per axis and sign of c.  Per
// population that is one three-way add for the table entry, one LDS read and
// one 64-bit add, with no selects and no 64-bit multiplies.
struct InteriorLane {
    uint32_t xm, x0, xp;  // LDS byte address of tab[13 + r_x] for c_x = -1 / 0 / +1
    uint32_t ym, yp;      // byte offset of the y part of the region for c_y = -1 / +1
    uint32_t zm, zp;      // the same along z
    uint32_t own;         // byte offset of the lane's own cell in a row
};

template <typename T>
__device__ __forceinline__ InteriorLane interior_lane(const uint64_t *tab, int i, int j, int k) {
    InteriorLane u;
    // LDS byte offset of the table (the pointer cast to the local address space)
    const uint32_t t = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint64_t *)tab + 13u * 8u;
    u.x0 = t;
    u.xm = t + (i == 3 ? 8u : 0u);
    u.xp = t - (i == 0 ? 8u : 0u);
    u.ym = j == 3 ? 24u : 0u;
    u.yp = j == 0 ? uint32_t(-24) : 0u;
    u.zm = k == 3 ? 72u : 0u;
    u.zp = k == 0 ? uint32_t(-72) : 0u;
    u.own = (uint32_t)(i + 4 * j + 16 * k) * (uint32_t)sizeof(T);
    return u;
}

// out[p] = conv(stored value of population p, p) for every population
template <typename Lt, typename ST, int P, typename Out, typename Conv>
__device__ __forceinline__ void gather_interior_by(const InteriorLane &u, Out *out, Conv conv) {
    if constexpr (P < Lt::Q) {
        using T = typename ST::T;
        constexpr int cx = Lt::cx(P), cy = Lt::cy(P), cz = Lt::cz(P);
        const uint32_t ex = cx < 0 ? u.xm : (cx > 0 ? u.xp : u.x0);
        const uint32_t ey = cy < 0 ? u.ym : (cy > 0 ? u.yp : 0u);
        const uint32_t ez = cz < 0 ? u.zm : (cz > 0 ? u.zp : 0u);
        const uint64_t row = *(const __attribute__((address_space(3))) uint64_t *)(uintptr_t)(ex + ey + ez);
        constexpr int64_t c = (int64_t)P * Lt::MB - (cx + 4 * cy + 16 * cz);
        // a global-memory pointer, so the load is a global (not flat) load and
        // does not hold up the waits on the LDS table reads
        const T *a = (const T *)(const __attribute__((address_space(1))) T *)(row + u.own) + c;
        out[P] = conv(ST::ld(a), P);
        gather_interior_by<Lt, ST, P + 1>(u, out, conv);
    }
}

// the shifted populations g (as load_g; RAW: the stored values)
template <typename Lt, typename ST, bool RAW = false>
__device__ __forceinline__ void gather_interior(const InteriorLane &u, typename ST::R *g) {
    using R = typename ST::R;
    gather_interior_by<Lt, ST, 0>(u, g, [](R v, int p) { return (ST::shift || RAW) ? v : v - R(Lt::w(p)); });
}

// BGK relaxation of one cell in the shifted variables: moments, then
// g <- g + omega (g_eq - g).  (A form with 1/rho taken once and the
// equilibrium grouped by weight saved no time here, and the reciprocal's
// rounding moved FP32 runs measurably further from FP64.)
template <typename Lt, typename R>
__device__ __forceinline__ void bgk_relax(R *g, R om, R &drho, R &ux, R &uy, R &uz, R &uu) {
    moments_g<Lt, R>(g, drho, ux, uy, uz);
    uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int p = 0; p < Lt::Q; p++)
        g[p] = fmadd(om, fmadd(R(Lt::w(p)), geq_y<Lt, R>(p, drho, ux, uy, uz, uu), -g[p]), g[p]);
}

// ---------------------------------------------------------------------------
// Moment-space (multiple-relaxation-time) collision for D3Q27, optional: the
// paper's method is BGK and it names moment-space operators only as the
// alternative (Sec. "Lattice Boltzmann Method").  Moment k = a + 3 b + 9 c is
// sum_p phi_a(c_x) phi_b(c_y) phi_c(c_z) f_p with phi_0 = 1, phi_1 = c,
// phi_2 = 3 c^2 - 1; the rows are orthogonal under the lattice weights with
// norms N_k = n_a n_b n_c (n = 1, 1/3, 2), so M^-1 = diag(w) M^T diag(1/N).
// Moments of order <= 2 relax at omega, the 17 others at s_high.  With the
// non-equilibrium part n = g - g_eq this is BGK plus a correction in the high
// moments only:
//     g* = g - omega n - w_p sum_{k high} M_kp ((s_high - omega) / N_k) (M n)_k
// so s_high = omega gives the BGK arithmetic exactly.
struct Mrt27 {
    static constexpr int NH = 17;
    int hk[NH];  // the moments of order > 2, ascending
    static constexpr int order(int k) { return k % 3 + k / 3 % 3 + k / 9; }
    static constexpr int phi(int a, int c) { return a == 0 ? 1 : (a == 1 ? c : 3 * c * c - 1); }
    static constexpr int m(int k, int p) { return phi(k % 3, D3::cx(p)) * phi(k / 3 % 3, D3::cy(p)) * phi(k / 9, D3::cz(p)); }
    static constexpr double norm(int k) {
        return (k % 3 == 0 ? 1.0 : (k % 3 == 1 ? 1.0 / 3.0 : 2.0)) *
               (k / 3 % 3 == 0 ? 1.0 : (k / 3 % 3 == 1 ? 1.0 / 3.0 : 2.0)) *
               (k / 9 == 0 ? 1.0 : (k / 9 == 1 ? 1.0 / 3.0 : 2.0));
    }
    constexpr Mrt27() : hk() {
        int n = 0;
        for (int k = 0; k < 27; k++)
            if (order(k) > 2) hk[n++] = k;
    }
};
constexpr Mrt27 kMrt27{};

// g -= w_p sum_k M_kp fac h_k / N_k with h = M n over the high moments, on the
// vector ALU (every coefficient a compile-time constant)
template <typename R, int S = 0>
__device__ __forceinline__ void mrt27_high(const R *n, R fac, R *g) {
    if constexpr (S < Mrt27::NH) {
        constexpr int k = kMrt27.hk[S];
        R h = R(0);
#pragma unroll
        for (int p = 0; p < 27; p++)
            if constexpr (true) {
                const int c = Mrt27::m(k, p);
                if (c == 1) h += n[p];
                else if (c == -1) h -= n[p];
                else if (c != 0) h += R(c) * n[p];
            }
        h *= fac * R(1.0 / Mrt27::norm(k));
#pragma unroll
        for (int p = 0; p < 27; p++) {
            const int c = Mrt27::m(k, p);
            if (c != 0) g[p] -= R(Lat<27>::w(p) * c) * h;
        }
        mrt27_high<R, S + 1>(n, fac, g);
    }
}

// The same correction with both transforms on the matrix cores
// (v_mfma_f32_16x16x32_f16; FP16 operands, FP32 accumulation).  One wave, 64
// cells = four tiles of 16.  Lane layout of the instruction: A[i][k] at lane l
// for i = l % 16, k = 8 (l / 16) + e (e = 0..7); B[k][j] for j = l % 16, the same
// k; D[i][j] in register r of lane l for i = 4 (l / 16) + r, j = l % 16.
//   forward:  H = M_high N   (rows: 32 slots, the 17 high moments first;
//                             K: the 27 populations; columns: cells)
//   scale:    slot s by (s_high - omega) / N_k, to FP16
//   back:     C = M_high^T H' (rows: populations; K in the order in which each
//             lane already holds the forward result: k = 8 g + e is slot
//             4 g + e for e < 4 and 16 + 4 g + e - 4 otherwise, g = l / 16)
// N is scaled by 2^8 before rounding to FP16 (non-equilibrium parts are small)
// and C by 2^-8 after.  The cell-major transposes go through LDS.
typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

struct MrtMfmaOps {
    _Float16 af[2][64][8];  // forward A, row blocks 0 / 1, per lane
    _Float16 ab[2][64][8];  // back A, population blocks 0 / 1, per lane
    float invn[32];         // 1 / N of the slot's moment; 0 past the 17
    static constexpr int slot_of_back_k(int k) { return (k % 8) < 4 ? 4 * (k / 8) + k % 8 : 16 + 4 * (k / 8) + k % 8 - 4; }
    constexpr MrtMfmaOps() : af(), ab(), invn() {
        for (int s = 0; s < 32; s++) invn[s] = s < Mrt27::NH ? float(1.0 / Mrt27::norm(kMrt27.hk[s])) : 0.0f;
        for (int b = 0; b < 2; b++)
            for (int l = 0; l < 64; l++)
                for (int e = 0; e < 8; e++) {
                    const int i = l % 16, k = 8 * (l / 16) + e;
                    const int sf = 16 * b + i;  // forward: row = slot, K = population
                    af[b][l][e] = (_Float16)((sf < Mrt27::NH && k < 27) ? Mrt27::m(kMrt27.hk[sf], k) : 0);
                    const int p = 16 * b + i, sb = slot_of_back_k(k);  // back: row = population
                    ab[b][l][e] = (_Float16)((sb < Mrt27::NH && p < 27) ? Mrt27::m(kMrt27.hk[sb], p) : 0);
                }
    }
};
constexpr MrtMfmaOps kMrtMfma{};

__device__ __forceinline__ void mrt27_high_mfma(const float *n, float fac, float *g) {
    constexpr float kScale = 256.0f;
    // per wave: 64 cells x 36 words (FP16 rows of 32 for the forward pass, FP32 rows of 32 for the back pass)
    __shared__ __attribute__((aligned(16))) float buf[4][64 * 36];
    const int l = threadIdx.x & 63, grp = l >> 4, col = l & 15;
    float *wb = buf[threadIdx.x >> 6];
    _Float16 *hb = (_Float16 *)wb;
    // cell-major FP16 rows of the scaled non-equilibrium parts: [cell][32]
#pragma unroll
    for (int c = 0; c < 4; c++) {
        mf_h8 v;
#pragma unroll
        for (int e = 0; e < 8; e++) v[e] = (_Float16)(8 * c + e < 27 ? n[8 * c + e] * kScale : 0.0f);
        *(mf_h8 *)(hb + l * 72 + 8 * c) = v;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    mf_h8 af0, af1, ab0, ab1;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        af0[e] = kMrtMfma.af[0][l][e];
        af1[e] = kMrtMfma.af[1][l][e];
        ab0[e] = kMrtMfma.ab[0][l][e];
        ab1[e] = kMrtMfma.ab[1][l][e];
    }
    float fs[8];
#pragma unroll
    for (int e = 0; e < 8; e++) fs[e] = fac * kMrtMfma.invn[e < 4 ? 4 * grp + e : 16 + 4 * grp + e - 4];
    const mf_f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    mf_h8 bb[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const mf_h8 b = *(const mf_h8 *)(hb + (16 * t + col) * 72 + 8 * grp);
        const mf_f4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(af0, b, zero, 0, 0, 0);
        const mf_f4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(af1, b, zero, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 8; e++) bb[t][e] = (_Float16)((e < 4 ? d0[e] : d1[e - 4]) * fs[e]);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const mf_f4 c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ab0, bb[t], zero, 0, 0, 0);
        const mf_f4 c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ab1, bb[t], zero, 0, 0, 0);
        // populations 4 grp + r and 16 + 4 grp + r of cell 16 t + col
        *(mf_f4 *)(wb + (16 * t + col) * 36 + 4 * grp) = c0;
        *(mf_f4 *)(wb + (16 * t + col) * 36 + 16 + 4 * grp) = c1;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int p = 0; p < 27; p++) g[p] -= float(Lat<27>::w(p) / 256.0) * wb[l * 36 + p];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Collision of one cell: COLL 0 = BGK, 1 = moment-space on the vector ALU,
// 2 = moment-space with the high-moment transforms on the matrix cores (a
// whole wave, every lane active; mrt27_high_mfma).
template <typename Lt, typename R, int COLL>
__device__ __forceinline__ void relax(R *g, R om, R sh, R &drho, R &ux, R &uy, R &uz, R &uu) {
    if constexpr (COLL == 0 || Lt::Q != 27) {
        bgk_relax<Lt, R>(g, om, drho, ux, uy, uz, uu);
    } else {
        moments_g<Lt, R>(g, drho, ux, uy, uz);
        uu = ux * ux + uy * uy + uz * uz;
        R n[27];
#pragma unroll
        for (int p = 0; p < 27; p++) {
            n[p] = fmadd(-R(Lt::w(p)), geq_y<Lt, R>(p, drho, ux, uy, uz, uu), g[p]);
            g[p] -= om * n[p];
        }
        if constexpr (COLL == 1)
            mrt27_high<R>(n, sh - om, g);
        else if constexpr (sizeof(R) == 4)
            mrt27_high_mfma(n, sh - om, g);
    }
}

// Per-workgroup staging of NBLK block descriptors; links by region slot.
// sim[] names the simulation of each entry in the batched kernels.
template <typename Lt, int NBLK>
struct BlockStage {
    static constexpr int NS = Lt::D == 2 ? 9 : 27;
    int32_t link[NBLK][NS];
    int32_t id[NBLK];
    int32_t hid[NBLK];
    int32_t sim[NBLK];
    uint8_t flag[NBLK];
};

// st.id[] (-1 = none) must be written and synchronised before the call;
// mesh_of(s) gives the mesh of entry s
template <typename Lt, int NBLK, typename MeshOf>
__device__ void stage_blocks_by(MeshOf mesh_of, BlockStage<Lt, NBLK> &st) {
    for (int e = threadIdx.x; e < NBLK * Lt::NB; e += blockDim.x) {
        const int s = e / Lt::NB, p = e - s * Lt::NB;
        const int B = st.id[s];
        int32_t v = 0, h = -1;
        uint8_t fl = 0;
        if (B >= 0) {
            const DevMesh &m = mesh_of(s);
            v = m.nbr[(int64_t)p * m.cap + B];
            if (p == 0) {
                h = m.hid[B];
                fl = m.bflag[B];
            }
        }
        st.link[s][dir_region<Lt>(p)] = v;
        if (p == 0) {
            st.hid[s] = h;
            st.flag[s] = fl;
        }
    }
    __syncthreads();
}

template <typename Lt, int NBLK>
__device__ void stage_blocks(const DevMesh &m, BlockStage<Lt, NBLK> &st) {
    stage_blocks_by<Lt, NBLK>([&](int) -> const DevMesh & { return m; }, st);
}

// Fill the row tables of the NBLK staged blocks (row(r) - 4 r . (1, 4, 16)
// in elements, as addresses; 0 where the link is not a block)
template <typename Lt, int NBLK, typename MeshOf, typename SrcOf>
__device__ __forceinline__ void fill_row_tables(const BlockStage<Lt, NBLK> &st, MeshOf mesh_of, SrcOf src_of,
                                                uint64_t (*tab)[27]) {
    for (int e = threadIdx.x; e < NBLK * 27; e += blockDim.x) {
        const int s = e / 27, r = e - s * 27;
        const int32_t id = st.id[s] >= 0 ? st.link[s][r] : -1;
        uint64_t v = 0;
        if (id >= 0 && id < mesh_of(s).cap) {
            const int rx = r % 3 - 1, ry = (r / 3) % 3 - 1, rz = r / 9 - 1;
            const int64_t el = (int64_t)id * (Lt::Q * Lt::MB) - 4 * (rx + 4 * ry + 16 * rz);
            v = (uint64_t)(uintptr_t)src_of(s) + (uint64_t)(el * (int64_t)sizeof(*src_of(s)));
        }
        tab[s][r] = v;
    }
}

// Contiguous range of work units [u0, u1) of a persistent workgroup: the
// count is read on the device, so one launch shape serves every mesh.
__device__ inline void persistent_range(int units, int &u0, int &u1) {
    const int G = gridDim.x;
    const int wg = xcd_remap(blockIdx.x, G);
    const int per = (units + G - 1) / G;
    u0 = min(units, wg * per);
    u1 = min(units, u0 + per);
}

// Read-only view of the batch descriptors in the constant address space: with
// a wave-uniform index their fields come in through scalar loads.
typedef const __attribute__((address_space(4))) SimDesc CSimDesc;
__device__ inline CSimDesc *const_view(const SimDesc *p) { return (CSimDesc *)p; }

__device__ inline DevMesh load_mesh(CSimDesc *cs) {
    DevMesh m;
    m.cap = cs->m.cap;
    m.capc = cs->m.capc;
    m.lmax = cs->m.lmax;
    m.halo_base = cs->m.halo_base;
    m.nh = cs->m.nh;
    m.interp = cs->m.interp;
    m.force = cs->m.force;
    m.hid = cs->m.hid;
    m.parent = cs->m.parent;
    m.fresh = cs->m.fresh;
    m.nbr = cs->m.nbr;
    m.nbrc = cs->m.nbrc;
    m.X = cs->m.X;
    m.level = cs->m.level;
    m.status = cs->m.status;
    m.tag = cs->m.tag;
    m.ldes = cs->m.ldes;
    m.viol = cs->m.viol;
    m.bflag = cs->m.bflag;
    m.gmask = cs->m.gmask;
    m.imask = cs->m.imask;
    return m;
}

// Thread index hidden from loop-invariant code motion: inside a persistent
// loop the per-cell index arithmetic is then redone per work unit instead of
// being hoisted and kept live across the loop.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// decode a batch work item into (simulation, block)
__device__ inline void decode_item(uint32_t it, int &sim, int &B) {
    sim = (int)(it >> kItemSimShift);
    B = (int)(it & kItemBlockMask);
}

// ---------------------------------------------------------------------------
// Fused collide + stream of one level (Secs. "Streaming", "Collision").  One
// 4^d block per 64-lane group (3-D: one block per wave; 2-D: four blocks per
// wave).  Each cell gathers its populations, collides, and writes its
// outgoing populations to its own slots; an outgoing population that would
// leave the fluid is replaced there by its bounce-back.  A population arriving
// from a region covered only by a coarser block keeps the cell's own
// post-collision value (halo record).  NTS: write with non-temporal stores
// (for levels whose output is too large to stay cached until the next sweep).
// EX: a leaf block next to a solid also adds its momentum exchange of this
// sweep to its total, exactly as the separate pass (exchange_block) would from
// the values just stored.
// Body: the cells of staged block s (this thread: cell l).
template <int Q, int S, int NBLK, bool NTS, int COLL = 0, bool EX = false>
__device__ __forceinline__ void collide_block(const DevMesh &m, const BlockStage<Lat<Q>, NBLK> &st, int s, int l,
                                              const typename Store<S>::T *__restrict__ src,
                                              typename Store<S>::T *__restrict__ dst, typename Store<S>::R om,
                                              const BCParams &bc, const uint64_t *tab,
                                              typename Store<S>::R sh = typename Store<S>::R(0)) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    const int B = st.id[s];
    if (B < 0) return;
    const uint8_t flag = st.flag[s];
    const int h = st.hid[s];
    const int32_t *link = st.link[s];
    const int i = l & 3, j = (l >> 2) & 3, k = l >> 4;

    R g[Q];
    R drho, ux, uy, uz;
    if constexpr (Lt::D == 3) {
        // Interior block (every region link a same-level block): one block per
        // wave; sources through the wave's row table (tab, in LDS).
        if (!(flag & (BF_BOUNDARY | BF_NSKIP))) {
            gather_interior<Lt, ST>(interior_lane<typename ST::T>(tab, i, j, k), g);
            R uu;
            relax<Lt, R, COLL>(g, om, sh, drho, ux, uy, uz, uu);
            const int Bu = __builtin_amdgcn_readfirstlane(B);
#pragma unroll
            for (int p = 0; p < Q; p++) store_g<Lt, ST, NTS>(dst, mslot<Lt>(Bu, p, l), p, g[p]);
            return;
        }
    }
    gather_cell<Lt, ST>(m, link, B, h, l, src, g);
    R uu;
    relax<Lt, R, COLL>(g, om, sh, drho, ux, uy, uz, uu);

    [[maybe_unused]] double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        if (flag & BF_BOUNDARY) {
            const int32_t code = link[region_of<Lt>(i + Lt::cx(q), j + Lt::cy(q), k + Lt::cz(q))];
            if (code < 0 && code != kNSkip) {
                R val;
                if (code == kSolid) {
                    val = g[q];
                    if constexpr (EX) {
                        // 2 f*_q c_q from the value as stored (rounded to the storage type)
                        typename ST::T t;
                        ST::st(&t, ST::shift ? val : val + R(Lt::w(q)));
                        const double two_f = 2.0 * double(ST::ld(&t) + (ST::shift ? Lt::w(q) : 0.0));
                        fx += two_f * Lt::cx(q);
                        fy += two_f * Lt::cy(q);
                        fz += two_f * Lt::cz(q);
                    }
                } else {
                    const int face = -3 - code;
                    const R cx = R(Lt::cx(q)), cy = R(Lt::cy(q)), cz = R(Lt::cz(q));
                    if (bc.kind[face] == AMR_FACE_VELOCITY) {
                        const R cuw = cx * R(bc.u[face][0]) + cy * R(bc.u[face][1]) + cz * R(bc.u[face][2]);
                        val = g[q] - R(6) * R(Lt::w(q)) * cuw;
                    } else {
                        const R cu = cx * ux + cy * uy + cz * uz;
                        val = -g[q] + R(2) * R(Lt::w(q)) * (R(4.5) * cu * cu - R(1.5) * uu);
                    }
                }
                // the slot now holds population opposite(q) of this cell
                store_g<Lt, ST, NTS>(dst, mslot<Lt>(B, q, l), Lt::opp(q), val);
                continue;
            }
        }
        store_g<Lt, ST, NTS>(dst, mslot<Lt>(B, q, l), q, g[q]);
    }
    if constexpr (EX) {
        // uniform over the block's lanes: sum over the block, one lane adds
        if ((flag & BF_SOLID) && m.status[B] == ST_UNREF) {
#pragma unroll
            for (int mask = 1; mask < Lt::MB; mask <<= 1) {
                fx += __shfl_xor(fx, mask, 64);
                fy += __shfl_xor(fy, mask, 64);
                fz += __shfl_xor(fz, mask, 64);
            }
            if (l == 0) {
                m.force[(int64_t)B * 3 + 0] += fx;
                m.force[(int64_t)B * 3 + 1] += fy;
                m.force[(int64_t)B * 3 + 2] += fz;
            }
        }
    }
    if ((flag & BF_NSKIP) && h >= 0) {
#pragma unroll
        for (int p = 1; p < Q; p++) {
            if (link[region_of<Lt>(i - Lt::cx(p), j - Lt::cy(p), k - Lt::cz(p))] == kNSkip)
                store_g<Lt, ST, NTS>(dst, m.halo_base + (int64_t)h * m.nh + kHalo<Lt>.idx[p][l], p, g[p]);
        }
    }
}

// Workgroup size: 256 threads (3-D: four blocks of the Morton launch order)
// for every storage.  Boundary and interface blocks take the slower generic
// path, and a CU can start a new workgroup only when all of its waves fit: with
// 512 threads a slow wave held back seven others (16-bit storage on the
// cylinder set-up: 968 us per launch against 915 us with 256), while 128
// threads lose the neighbour reuse between the blocks of a workgroup.
template <int S>
constexpr int collide_threads() { return 256; }

// blocks per workgroup of k_collide_stream (one per 64-lane group)
template <int Q, int S>
constexpr int collide_blocks_per_wg() { return collide_threads<S>() / Lat<Q>::MB; }

// COLL: 0 = BGK, 1 / 2 = moment-space collision (D3Q27) on the vector ALU /
// with the matrix-core transforms; s_high = its rate above second order
// One workgroup's share of a level sweep: blocks wg * BPW .. of the list
template <int Q, int S, bool NTS, int COLL, bool EX = false>
__device__ __forceinline__ void collide_wg(const int32_t *__restrict__ list, int n, const DevMesh &m,
                                           const typename Store<S>::T *__restrict__ src,
                                           typename Store<S>::T *__restrict__ dst, double omega_d, const BCParams &bc,
                                           double s_high, int wg) {
    using Lt = Lat<Q>;
    using R = typename Store<S>::R;
    constexpr int MB = Lt::MB, BPW = collide_blocks_per_wg<Q, S>();
    __shared__ BlockStage<Lt, BPW> st;
    __shared__ uint64_t tab[Lt::D == 3 ? BPW : 1][27];
    const int base = wg * BPW;
    if ((int)threadIdx.x < BPW) st.id[threadIdx.x] = base + (int)threadIdx.x < n ? list[base + threadIdx.x] : -1;
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    if constexpr (Lt::D == 3) {
        fill_row_tables<Lt, BPW>(st, [&](int) -> const DevMesh & { return m; }, [&](int) { return src; }, tab);
        __syncthreads();
    }
    const int s = threadIdx.x / MB;
    collide_block<Q, S, BPW, NTS, COLL, EX>(m, st, s, threadIdx.x % MB, src, dst, R(omega_d), bc,
                                            tab[Lt::D == 3 ? s : 0], R(s_high));
}

template <int Q, int S, bool NTS, int COLL = 0, bool EX = false>
__global__ __launch_bounds__(collide_threads<S>()) void k_collide_stream(
    const int32_t *__restrict__ list, int n, DevMesh m, const typename Store<S>::T *__restrict__ src,
    typename Store<S>::T *__restrict__ dst, double omega_d, BCParams bc, double s_high) {
    collide_wg<Q, S, NTS, COLL, EX>(list, n, m, src, dst, omega_d, bc, s_high, xcd_remap(blockIdx.x, gridDim.x));
}

// Batched form: level L of every simulation of a batch in one persistent
// launch of NT-thread workgroups (NT / Mb blocks each); all simulations share
// the buffer parity `par` of level L.
template <int Q, int S, int NT>
__global__ __launch_bounds__(NT) void k_collide_stream_batch(const SimDesc *__restrict__ sims,
                                                             const uint32_t *__restrict__ items,
                                                             const int32_t *__restrict__ count, int L, int par) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    using T = typename ST::T;
    constexpr int MB = Lt::MB, BPW = NT / MB;
    __shared__ BlockStage<Lt, BPW> st;
    __shared__ uint64_t tab[Lt::D == 3 ? BPW : 1][27];
    const int n = *count;
    int u0, u1;
    persistent_range((n + BPW - 1) / BPW, u0, u1);
    for (int u = u0; u < u1; u++) {
        if ((int)threadIdx.x < BPW) {
            const int idx = u * BPW + (int)threadIdx.x;
            int sim = 0, B = -1;
            if (idx < n) decode_item(items[idx], sim, B);
            st.id[threadIdx.x] = B;
            st.sim[threadIdx.x] = sim;
        }
        __syncthreads();
        stage_blocks_by<Lt, BPW>([&](int e) -> const DevMesh & { return sims[st.sim[e]].m; }, st);
        if constexpr (Lt::D == 3) {
            fill_row_tables<Lt, BPW>(st, [&](int e) -> const DevMesh & { return sims[st.sim[e]].m; },
                                     [&](int e) { return (const T *)sims[st.sim[e]].f[par]; }, tab);
            __syncthreads();
        }
        const int tid = opaque_tid();
        const int s = tid / MB;
        int sim = st.sim[s];
        if (MB == 64) sim = __builtin_amdgcn_readfirstlane(sim);  // one block per wave
        CSimDesc *cs = const_view(sims) + sim;
        const DevMesh m = load_mesh(cs);
        collide_block<Q, S, BPW, false>(m, st, s, tid % MB, (const T *)cs->f[par], (T *)cs->f[1 - par],
                                 R(cs->lp.omega[L]), sims[sim].bc, tab[Lt::D == 3 ? s : 0]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Coarse-to-fine linear interpolation with Dupuis-Chopard rescaling (Sec.
// "Linear Interpolation").  One parent block per workgroup: its cells are
// rescaled into LDS, then every targeted fine cell evaluates the (bi/tri)linear
// polynomial through the 2^d parent cells of its quadrant at
// (-1/4 + I/2, -1/4 + J/2, -1/4 + K/2).
template <typename R>
__device__ inline R lin2(R F0, R F1, R F2, R F3, R x, R y) {
    const R a0 = F0, a1 = F1 - F0, a2 = F2 - F0, a3 = F3 - F2 - F1 + F0;
    return a0 + a1 * x + a2 * y + a3 * x * y;
}
template <typename R>
__device__ inline R lin3(const R *F, R x, R y, R z) {
    const R a0 = F[0];
    const R a1 = F[1] - F[0];
    const R a2 = F[2] - F[0];
    const R a3 = F[4] - F[0];
    const R a4 = F[3] - F[1] - F[2] + F[0];
    const R a5 = F[6] - F[2] - F[4] + F[0];
    const R a6 = F[5] - F[1] - F[4] + F[0];
    const R a7 = F[7] - F[3] - F[5] - F[6] + F[1] + F[2] + F[4] - F[0];
    return a0 + a1 * x + a2 * y + a3 * z + a4 * x * y + a5 * y * z + a6 * x * z + a7 * x * y * z;
}

// Weights of the cubic Lagrange polynomials through the nodes u = 0, 1, 2, 3 at u.
template <typename R>
__device__ __forceinline__ void lagrange4(R u, R *w) {
    const R a = u, b = u - R(1), c = u - R(2), d = u - R(3);
    w[0] = -(b * c * d) / R(6);
    w[1] = (a * c * d) / R(2);
    w[2] = -(a * b * d) / R(2);
    w[3] = (a * b * c) / R(6);
}

// Interpolated value of fine cell lf of child c from one population of the
// parent's rescaled cells F[Mb].  Linear: the polynomial through the 2^d
// parent cells of the quadrant at (-1/4 + I/2, ...).  Cubic (Sec. "Cubic
// Interpolation"): the tensor product through all 4^d parent cells, nodes at
// parent cell centres u = 0 .. 3, evaluated at u = 3 (-1/12 + I/6 + 2 c/3)
// one axis at a time.
template <typename Lt, typename R>
__device__ __forceinline__ R interp_value(const R *F, int c, int lf, int cubic) {
    const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    const int I = lf & 3, J = (lf >> 2) & 3, K = lf >> 4;
    if (!cubic) {
        const R x = R(-0.25) + R(0.5) * R(I), y = R(-0.25) + R(0.5) * R(J), z = R(-0.25) + R(0.5) * R(K);
        const int m0 = 2 * cx + 4 * (2 * cy) + 16 * (2 * cz);
        if (Lt::D == 2) return lin2<R>(F[m0], F[m0 + 1], F[m0 + 4], F[m0 + 5], x, y);
        R G[8];
#pragma unroll
        for (int nn = 0; nn < 8; nn++) G[nn] = F[m0 + (nn & 1) + 4 * ((nn >> 1) & 1) + 16 * (nn >> 2)];
        return lin3<R>(G, x, y, z);
    }
    R wx[4], wy[4], wz[4];
    lagrange4<R>(R(-0.25) + R(0.5) * R(I) + R(2 * cx), wx);
    lagrange4<R>(R(-0.25) + R(0.5) * R(J) + R(2 * cy), wy);
    lagrange4<R>(R(-0.25) + R(0.5) * R(K) + R(2 * cz), wz);
    R v = R(0);
#pragma unroll
    for (int e = 0; e < (Lt::D == 3 ? 4 : 1); e++) {
        R plane = R(0);
#pragma unroll
        for (int n = 0; n < 4; n++) {
            R row = R(0);
#pragma unroll
            for (int mm = 0; mm < 4; mm++) row += wx[mm] * F[mm + 4 * n + 16 * e];
            plane += wy[n] * row;
        }
        v += (Lt::D == 3 ? wz[e] : R(1)) * plane;
    }
    return v;
}

template <typename Lt, typename R>
struct InterpSmem {
    R g[Lt::Q][Lt::MB];
    uint64_t gm[Lt::NC];
    BlockStage<Lt, Lt::NC + 1> st;  // entry NC = the parent
};

// Body (whole workgroup): targeted cells of the children of refined parent P.
// CUB: 0 linear, 1 cubic, 2 the mesh's choice at run time.
template <int Q, int S, int CUB>
__device__ __forceinline__ void interp_parent(const DevMesh &m, int P, const typename Store<S>::T *src,
                                              typename Store<S>::T *dst, typename Store<S>::R r, int all_cells,
                                              InterpSmem<Lat<Q>, typename Store<S>::R> &sm, int t) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr int MB = Lt::MB, NC = Lt::NC;
    const int first = m.nbrc[P];
    if (t <= NC) sm.st.id[t] = t < NC ? first + t : P;
    if (t < NC) sm.gm[t] = all_cells ? ~0ull : m.gmask[first + t];
    __syncthreads();
    stage_blocks<Lt, NC + 1>(m, sm.st);
    if (t < MB) {
        R g[Q];
        gather_cell_flag<Lt, ST>(m, sm.st.link[NC], P, sm.st.hid[NC], sm.st.flag[NC], t, src, g);
        R drho, ux, uy, uz;
        moments_g<Lt, R>(g, drho, ux, uy, uz);
        const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int p = 0; p < Q; p++) sm.g[p][t] = rescale_neq<Lt, R>(p, g[p], r, drho, ux, uy, uz, uu);
    }
    __syncthreads();
    const int cubic = CUB == 2 ? m.interp : CUB;
    for (int e = t; e < NC * MB; e += blockDim.x) {
        const int c = e / MB, lf = e - c * MB;
        if (!((sm.gm[c] >> lf) & 1ull)) continue;
        const int32_t *link = sm.st.link[c];
        const int hc = sm.st.hid[c];
        if (cubic) {
            // 4^d terms per population: not unrolled over the populations
#pragma unroll 1
            for (int p = 0; p < Q; p++) {
                const R v = interp_value<Lt, R>(sm.g[p], c, lf, 1);
                store_g<Lt, ST>(dst, entry_slot<Lt>(m, link, first + c, hc, p, lf), p, v);
            }
        } else {
#pragma unroll
            for (int p = 0; p < Q; p++) {
                const R v = interp_value<Lt, R>(sm.g[p], c, lf, 0);
                store_g<Lt, ST>(dst, entry_slot<Lt>(m, link, first + c, hc, p, lf), p, v);
            }
        }
    }
}

// refined parents only (a listed block that is not one is skipped)
__device__ inline bool interp_target(const DevMesh &m, int P, int nc) {
    const int first = m.nbrc[P];
    return !(first < 0 || first > m.cap - nc || m.level[P] + 1 >= m.lmax);
}

template <int Q, int S, int CUB>
__device__ __forceinline__ void interp_wg(const int32_t *__restrict__ list, int n, const DevMesh &m,
                                          typename Store<S>::T *f0, typename Store<S>::T *f1, const LevelParams &lp,
                                          int all_cells, int item) {
    using R = typename Store<S>::R;
    __shared__ InterpSmem<Lat<Q>, R> sm;
    if (item >= n) return;
    const int P = list[item];
    if (!interp_target(m, P, Lat<Q>::NC)) return;
    const int L = m.level[P];
    interp_parent<Q, S, CUB>(m, P, lp.par[L] ? f1 : f0, lp.par[L + 1] ? f1 : f0, R(lp.r_cf[L]), all_cells, sm,
                             threadIdx.x);
}

template <int Q, int S, int CUB>
__global__ __launch_bounds__(256) void k_interp(const int32_t *__restrict__ list, int n, DevMesh m,
                                                typename Store<S>::T *f0, typename Store<S>::T *f1, LevelParams lp,
                                                int all_cells) {
    interp_wg<Q, S, CUB>(list, n, m, f0, f1, lp, all_cells, blockIdx.x);
}

// The ghost interpolation into level L+1 and the collide-stream sweep of level
// L in one 256-thread launch: workgroups 0 .. ni-1 interpolate one parent each
// (in 2-D with the first 64 threads; interp_parent strides by the workgroup
// size), the rest sweep the level.  Both read level L's current buffer; one
// writes ghost cells of level L+1, the other level L's other buffer, so they
// need no order, and small levels save a launch gap.  EX: the sweep adds the
// momentum exchange too (collide_block).
template <int Q, int S, bool NTS, int CUB, bool EX = false>
__global__ __launch_bounds__(256) void k_interp_collide(const int32_t *__restrict__ ilist, int ni,
                                                        const int32_t *__restrict__ clist, int nblk, DevMesh m,
                                                        typename Store<S>::T *f0, typename Store<S>::T *f1,
                                                        LevelParams lp, int L, BCParams bc) {
    const int b = blockIdx.x;
    if (b < ni) {
        interp_wg<Q, S, CUB>(ilist, ni, m, f0, f1, lp, 0, b);
    } else {
        const typename Store<S>::T *src = lp.par[L] ? f1 : f0;
        typename Store<S>::T *dst = lp.par[L] ? f0 : f1;
        collide_wg<Q, S, NTS, 0, EX>(clist, nblk, m, src, dst, lp.omega[L], bc, lp.omega[L],
                                     xcd_remap(b - ni, (int)gridDim.x - ni));
    }
}

// Batched ghost fill of level L+1 from level L (interface parents of every
// simulation), persistent workgroups; par0/par1 = buffers of levels L, L+1.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_interp_batch(const SimDesc *__restrict__ sims,
                                                      const uint32_t *__restrict__ items,
                                                      const int32_t *__restrict__ count, int L, int par0, int par1) {
    using ST = Store<S>;
    using R = typename ST::R;
    using T = typename ST::T;
    __shared__ InterpSmem<Lat<Q>, R> sm;
    int u0, u1;
    persistent_range(*count, u0, u1);
    for (int u = u0; u < u1; u++) {
        int sim, P;
        decode_item(items[u], sim, P);
        sim = __builtin_amdgcn_readfirstlane(sim);  // one item per workgroup
        P = __builtin_amdgcn_readfirstlane(P);
        CSimDesc *cs = const_view(sims) + sim;
        const DevMesh m = load_mesh(cs);
        if (interp_target(m, P, Lat<Q>::NC))
            interp_parent<Q, S, 2>(m, P, (const T *)cs->f[par0], (T *)cs->f[par1], R(cs->lp.r_cf[L]), 0, sm,
                                   opaque_tid());
        __syncthreads();
    }
}

// Refresh after refinement.  A cell x of an existing block N next to a new
// same-level block C now receives the populations that stream from C's cells;
// they are stored in C's rows, which the interpolation of C's own cells does
// not write.  Their values are those x already had: the ghost interpolation
// from N's parent (x was adjacent to the region C now covers, which was
// covered only by a coarser block).  One workgroup per refined parent.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_refresh_neighbours(const int32_t *__restrict__ list, int n, DevMesh m,
                                                            typename Store<S>::T *f0, typename Store<S>::T *f1,
                                                            LevelParams lp) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    using T = typename ST::T;
    constexpr int MB = Lt::MB, NC = Lt::NC, NS = Lt::D == 2 ? 9 : 27;
    __shared__ R s_g[Q][MB];
    __shared__ BlockStage<Lt, NC + 1> st;  // the new children, then the neighbour's parent
    __shared__ int s_nb[NC][NS];           // existing same-level neighbour per child and region, -1 none
    if ((int)blockIdx.x >= n) return;
    const int P = list[blockIdx.x];
    const int L = m.level[P];
    const int first = m.nbrc[P];
    if (first < 0 || first > m.cap - NC || L + 1 >= m.lmax) return;
    const T *psrc = lp.par[L] ? f1 : f0;
    T *dst = lp.par[L + 1] ? f1 : f0;
    const R r = R(lp.r_cf[L]);
    const int t = threadIdx.x;
    if (t < NC) st.id[t] = first + t;
    if (t == NC) st.id[NC] = -1;
    __syncthreads();
    stage_blocks<Lt, NC + 1>(m, st);
    for (int e = t; e < NC * NS; e += blockDim.x) {
        const int c = e / NS, rg = e - c * NS;
        const int N = st.link[c][rg];
        s_nb[c][rg] = (rg != kCenterSlot<Lt> && N >= 0 && N < m.cap && !m.fresh[N] && m.parent[N] >= 0) ? N : -1;
    }
    __syncthreads();
    for (int c = 0; c < NC; c++) {
        for (int rg = 0; rg < NS; rg++) {
            const int N = s_nb[c][rg];  // uniform over the workgroup
            if (N < 0) continue;
            const int PN = m.parent[N];
            const int cN = N - m.nbrc[PN];
            if (t == 0) st.id[NC] = PN;
            __syncthreads();
            for (int e = t; e < Lt::NB; e += blockDim.x)
                st.link[NC][dir_region<Lt>(e)] = m.nbr[(int64_t)e * m.cap + PN];
            if (t == 0) st.hid[NC] = m.hid[PN];
            __syncthreads();
            if (t < MB) {
                R g[Q];
                gather_cell<Lt, ST>(m, st.link[NC], PN, st.hid[NC], t, psrc, g);
                R drho, ux, uy, uz;
                moments_g<Lt, R>(g, drho, ux, uy, uz);
                const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
                for (int p = 0; p < Q; p++) s_g[p][t] = rescale_neq<Lt, R>(p, g[p], r, drho, ux, uy, uz, uu);
            }
            __syncthreads();
            if (t < MB) {
                const int si = t & 3, sj = (t >> 2) & 3, sk = t >> 4;
#pragma unroll
                for (int p = 1; p < Q; p++) {
                    const int tx = si + Lt::cx(p), ty = sj + Lt::cy(p), tz = sk + Lt::cz(p);
                    if (region_of<Lt>(tx, ty, tz) != rg) continue;
                    // cell x of N (quadrant cN of N's parent): its ghost-fill value
                    const int lx = (tx & 3) + 4 * (ty & 3) + 16 * (tz & 3);
                    const R v = interp_value<Lt, R>(s_g[p], cN, lx, m.interp);
                    store_g<Lt, ST>(dst, mslot<Lt>(first + c, p, t), p, v);
                }
            }
            __syncthreads();
        }
    }
}

__global__ void k_clear_fresh(const int32_t *__restrict__ list, int n, DevMesh m, int nc) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * nc) return;
    const int P = list[e / nc];
    const int first = m.nbrc[P];
    if (first >= 0 && first + e % nc < m.cap) m.fresh[first + e % nc] = 0;
}

// ---------------------------------------------------------------------------
// Fine-to-coarse averaging with rescaling (Sec. "Averaging"): parent cell
// (i,j,k) takes the mean of the 2^d rescaled cells of child octant
// (i/2, j/2, k/2) starting at fine cell (2(i mod 2), 2(j mod 2), 2(k mod 2)).
// One lane per fine cell of the children (3-D: a wave per child; two
// workgroups of four children per parent, so that children that end early do
// not hold back a workgroup of eight): every lane gathers and rescales its
// cell, the 2^d cells of a parent cell (lanes differing in bits 0, 2, 4 of the
// cell index, all in one wave) are summed with xor shuffles, and the lane of
// the first one writes the parent cell.  Children without a targeted cell are
// skipped whole.

// The vorticity criterion reads velocities of leaf blocks and, across the six
// faces of a leaf, of its same-level neighbours: a refined block none of whose
// face neighbours is a leaf is never read.
template <typename Lt>
__device__ __forceinline__ bool velocity_read(const DevMesh &m, const int32_t *link, int B) {
    if (!is_refined(m.status[B])) return true;
    bool read = false;
#pragma unroll
    for (int a = 0; a < Lt::D; a++)
        for (int sg = -1; sg <= 1; sg += 2) {
            const int32_t code =
                link[region_of<Lt>(a == 0 ? 1 + 3 * sg : 1, a == 1 ? 1 + 3 * sg : 1, a == 2 ? 1 + 3 * sg : 1)];
            if (code >= 0 && code < m.cap && m.status[code] == ST_UNREF) read = true;
        }
    return read;
}

// FP64 velocity j / rho of cell `cell` from its populations fv, into U[3][capc]
template <typename Lt>
__device__ __forceinline__ void cell_velocity(const double *fv, double *U, int64_t capc, int64_t cell) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) {
        rho += fv[p];
        j[0] += fv[p] * Lt::cx(p);
        j[1] += fv[p] * Lt::cy(p);
        j[2] += fv[p] * Lt::cz(p);
    }
    for (int a = 0; a < 3; a++) U[a * capc + cell] = j[a] / rho;
}

// refined parents with children in the next level
__device__ inline bool average_target(const DevMesh &m, int P, int nc) {
    const int c0 = m.nbrc[P];
    return is_refined(m.status[P]) && c0 >= 0 && c0 <= m.cap - nc && m.level[P] + 1 < m.lmax;
}

template <typename R>
__device__ __forceinline__ R xor_sum(R v, int mask) {
    return v + __shfl_xor(v, mask, 64);
}

// children per averaging workgroup
template <int Q>
constexpr int avg_children() { return Lat<Q>::D == 3 ? 4 : Lat<Q>::NC; }

// children c0 .. c0 + NCW - 1 of parent P.  VEL (every cell averaged): also
// the criterion's FP64 velocity of each child cell that it reads
// (velocity_read) and that the ghost interpolation after the averaging does
// not rewrite (no N_SKIP link), from the values as stored, into U: the same
// values and arithmetic as k_velocity, so that pass can skip those blocks.
template <int Q, int S, bool VEL = false>
__device__ __forceinline__ void average_parent(const DevMesh &m, int P, int c0, const typename Store<S>::T *src,
                                               typename Store<S>::T *dst, typename Store<S>::R r, int all_cells,
                                               BlockStage<Lat<Q>, avg_children<Q>() + 1> &st,
                                               uint64_t (*tab)[27], int t, double *U = nullptr) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    // with unshifted storage the velocities need the stored values: gather
    // those, then form g exactly as load_g does
    constexpr bool RAW = VEL && !ST::shift;
    constexpr int MB = Lt::MB, NCW = avg_children<Q>(), NC = Lt::NC;
    const int first = m.nbrc[P];
    if (t <= NCW) st.id[t] = t < NCW ? first + c0 + t : P;
    __syncthreads();
    stage_blocks<Lt, NCW + 1>(m, st);
    if constexpr (Lt::D == 3) {
        fill_row_tables<Lt, NCW + 1>(st, [&](int) -> const DevMesh & { return m; }, [&](int) { return src; }, tab);
        __syncthreads();
    }
    const int cw = t / MB, lf = t - cw * MB;
    if (cw >= NCW) return;
    const int c = c0 + cw;  // octant of the child in its parent
    const int child = first + c;
    const uint64_t im = all_cells ? ~0ull : m.imask[child];
    if (im == 0) return;  // the whole child (a wave in 3-D, a 16-lane group in 2-D)
    // the 2^d lanes of one parent cell (cell-index bits 0, 2 and, in 3-D, 4)
    // are exactly the partners of the sums below: a group whose parent cell
    // is not written loads nothing
    const int lead = lf & ~(Lt::D == 3 ? 0x15 : 0x5);
    R g[Q];
    if ((im >> lead) & 1ull) {
        bool done = false;
        if constexpr (Lt::D == 3) {
            if (!(st.flag[cw] & (BF_BOUNDARY | BF_NSKIP))) {
                gather_interior<Lt, ST, RAW>(interior_lane<typename ST::T>(tab[cw], lf & 3, (lf >> 2) & 3, lf >> 4), g);
                done = true;
            }
        }
        if (!done) gather_cell_flag<Lt, ST, RAW>(m, st.link[cw], child, st.hid[cw], st.flag[cw], lf, src, g);
    } else {
#pragma unroll
        for (int p = 0; p < Q; p++) g[p] = R(0);
    }
    if constexpr (VEL) {
        if (!(st.flag[cw] & BF_NSKIP) && velocity_read<Lt>(m, st.link[cw], child)) {
            double fv[Q];
#pragma unroll
            for (int p = 0; p < Q; p++) fv[p] = double(g[p]) + (ST::shift ? Lt::w(p) : 0.0);
            cell_velocity<Lt>(fv, U, m.capc, (int64_t)child * MB + lf);
        }
        if constexpr (RAW) {
            if ((im >> lead) & 1ull) {
#pragma unroll
                for (int p = 0; p < Q; p++) g[p] = g[p] - R(Lt::w(p));
            }
        }
    }
    R drho, ux, uy, uz;
    moments_g<Lt, R>(g, drho, ux, uy, uz);
    const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int p = 0; p < Q; p++) {
        R v = rescale_neq<Lt, R>(p, g[p], r, drho, ux, uy, uz, uu);
        v = xor_sum(v, 1);
        v = xor_sum(v, 4);
        if (Lt::D == 3) v = xor_sum(v, 16);
        g[p] = v;
    }
    const int i = lf & 3, j = (lf >> 2) & 3, k = lf >> 4;
    if (lf != lead || !((im >> lf) & 1ull)) return;
    const int l = ((c & 1) * 2 + (i >> 1)) + 4 * (((c >> 1) & 1) * 2 + (j >> 1)) + 16 * ((c >> 2) * 2 + (k >> 1));
    const int32_t *plink = st.link[NCW];
    const int ph = st.hid[NCW];
#pragma unroll
    for (int p = 0; p < Q; p++) store_g<Lt, ST>(dst, entry_slot<Lt>(m, plink, P, ph, p, l), p, g[p] / R(NC));
}

// grid: NC / avg_children workgroups per listed parent.  At least 6 waves per
// SIMD: left alone the compiler takes 88 VGPRs (5 waves) for D3Q27 FP32; at 80
// the launch is 9 % shorter on the cylinder set-up (no spills; at 64 it spills
// and is slower).
template <int Q, int S, bool VEL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == AMR_F64 ? 1 : 6))) void k_average(const int32_t *__restrict__ list, int n, DevMesh m,
                                                 typename Store<S>::T *f0, typename Store<S>::T *f1, LevelParams lp,
                                                 int all_cells, double *U) {
    using Lt = Lat<Q>;
    using R = typename Store<S>::R;
    constexpr int SPLIT = Lt::NC / avg_children<Q>();
    __shared__ BlockStage<Lt, avg_children<Q>() + 1> st;
    __shared__ uint64_t tab[Lt::D == 3 ? avg_children<Q>() + 1 : 1][27];
    const int item = blockIdx.x / SPLIT, part = blockIdx.x % SPLIT;
    if (item >= n) return;
    const int P = list[item];
    if (!average_target(m, P, Lt::NC)) return;
    const int L = m.level[P];
    average_parent<Q, S, VEL>(m, P, part * avg_children<Q>(), lp.par[L + 1] ? f1 : f0, lp.par[L] ? f1 : f0,
                              R(lp.r_fc[L]), all_cells, st, tab, threadIdx.x, U);
}

// Batched interface averaging of level L+1 into level L, persistent
// workgroups; par0/par1 = buffers of levels L, L+1.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_average_batch(const SimDesc *__restrict__ sims,
                                                       const uint32_t *__restrict__ items,
                                                       const int32_t *__restrict__ count, int L, int par0, int par1) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    using T = typename ST::T;
    constexpr int SPLIT = Lt::NC / avg_children<Q>();
    __shared__ BlockStage<Lt, avg_children<Q>() + 1> st;
    __shared__ uint64_t tab[Lt::D == 3 ? avg_children<Q>() + 1 : 1][27];
    int u0, u1;
    persistent_range(*count * SPLIT, u0, u1);
    for (int u = u0; u < u1; u++) {
        int sim, P;
        decode_item(items[u / SPLIT], sim, P);
        sim = __builtin_amdgcn_readfirstlane(sim);  // one item per workgroup
        P = __builtin_amdgcn_readfirstlane(P);
        CSimDesc *cs = const_view(sims) + sim;
        const DevMesh m = load_mesh(cs);
        if (average_target(m, P, Lt::NC))
            average_parent<Q, S>(m, P, (u % SPLIT) * avg_children<Q>(), (const T *)cs->f[par1], (T *)cs->f[par0],
                                 R(cs->lp.r_fc[L]), 0, st, tab, opaque_tid());
        __syncthreads();
    }
}

// Work items of a batch for every level: kind 0 = launch order of the level,
// kind 1 = its interface parents, kind 2 = its leaf blocks next to a solid
// block; simulations in batch order.  Grid: x chunks of a list, y =
// simulation, z = 3 * level + kind.  counts[3 L + kind].
__device__ inline int item_count(const SimDesc &d, int L, int kind) {
    if (L >= d.m.lmax) return 0;
    return kind == 0 ? d.nids[L] : (kind == 1 ? d.niface[L] : (d.force_on ? d.nsolid[L] : 0));
}

__global__ void k_batch_items(const SimDesc *__restrict__ sims, int nsims, uint32_t *__restrict__ items,
                              int64_t stride, int32_t *__restrict__ counts) {
    const int s = blockIdx.y, L = blockIdx.z / 3, kind = blockIdx.z % 3;
    __shared__ int s_off, s_n;
    if (threadIdx.x == 0) {
        int off = 0;
        for (int t = 0; t < s; t++) off += item_count(sims[t], L, kind);
        const int n = item_count(sims[s], L, kind);
        s_off = off;
        s_n = n;
        if (s == nsims - 1 && blockIdx.x == 0) counts[blockIdx.z] = off + n;
    }
    __syncthreads();
    const SimDesc &sd = sims[s];
    const int32_t *src = (kind == 0 ? sd.order : (kind == 1 ? sd.iface : sd.solid)) + (int64_t)L * sd.m.cap;
    uint32_t *dst = items + (int64_t)blockIdx.z * stride + s_off;
    const uint32_t tag = (uint32_t)s << kItemSimShift;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s_n; i += gridDim.x * blockDim.x)
        dst[i] = tag | (uint32_t)src[i];
}

// ---------------------------------------------------------------------------
// Momentum exchange with solid blocks (Sec. "Flow Past a Square Cylinder"),
// after a collide-stream sweep: a leaf cell's post-collision population f*_q
// whose link ends in a solid block was reflected into the cell's own slot
// (x, q) of the buffer just written; it passes 2 f*_q c_q to the solid.  One
// block per 64 lanes (2-D: 16), summed over the block, added to its FP64 total
// (each block's total is written by one lane only).
template <int Q, int S>
__device__ __forceinline__ void exchange_block(const DevMesh &m, const BlockStage<Lat<Q>, 256 / Lat<Q>::MB> &st,
                                               int s, int l, const typename Store<S>::T *f) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    const int B = st.id[s];
    if (B < 0) return;
    const int32_t *link = st.link[s];
    const int i = l & 3, j = (l >> 2) & 3, k = l >> 4;
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int q = 1; q < Q; q++) {
        if (link[region_of<Lt>(i + Lt::cx(q), j + Lt::cy(q), k + Lt::cz(q))] != kSolid) continue;
        const double two_f = 2.0 * double(ST::ld(f + mslot<Lt>(B, q, l)) + (ST::shift ? Lt::w(q) : 0.0));
        fx += two_f * Lt::cx(q);
        fy += two_f * Lt::cy(q);
        fz += two_f * Lt::cz(q);
    }
#pragma unroll
    for (int mask = 1; mask < Lt::MB; mask <<= 1) {
        fx += __shfl_xor(fx, mask, 64);
        fy += __shfl_xor(fy, mask, 64);
        fz += __shfl_xor(fz, mask, 64);
    }
    if (l == 0) {
        m.force[(int64_t)B * 3 + 0] += fx;
        m.force[(int64_t)B * 3 + 1] += fy;
        m.force[(int64_t)B * 3 + 2] += fz;
    }
}

template <int Q, int S>
__global__ __launch_bounds__(256) void k_exchange(const int32_t *__restrict__ list, int n, DevMesh m,
                                                  const typename Store<S>::T *__restrict__ f) {
    using Lt = Lat<Q>;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    const int base = blockIdx.x * BPW;
    if ((int)threadIdx.x < BPW) st.id[threadIdx.x] = base + (int)threadIdx.x < n ? list[base + threadIdx.x] : -1;
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    exchange_block<Q, S>(m, st, threadIdx.x / MB, threadIdx.x % MB, f);
}

template <int Q, int S>
__global__ __launch_bounds__(256) void k_exchange_batch(const SimDesc *__restrict__ sims,
                                                        const uint32_t *__restrict__ items,
                                                        const int32_t *__restrict__ count, int par) {
    using Lt = Lat<Q>;
    using T = typename Store<S>::T;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    const int n = *count;
    int u0, u1;
    persistent_range((n + BPW - 1) / BPW, u0, u1);
    for (int u = u0; u < u1; u++) {
        if ((int)threadIdx.x < BPW) {
            const int idx = u * BPW + (int)threadIdx.x;
            int sim = 0, B = -1;
            if (idx < n) decode_item(items[idx], sim, B);
            st.id[threadIdx.x] = B;
            st.sim[threadIdx.x] = sim;
        }
        __syncthreads();
        stage_blocks_by<Lt, BPW>([&](int e) -> const DevMesh & { return sims[st.sim[e]].m; }, st);
        const int tid = opaque_tid();
        const int s = tid / MB;
        int sim = st.sim[s];
        if (MB == 64) sim = __builtin_amdgcn_readfirstlane(sim);
        CSimDesc *cs = const_view(sims) + sim;
        const DevMesh m = load_mesh(cs);
        exchange_block<Q, S>(m, st, s, tid % MB, (const T *)cs->f[par]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Per-level totals of the momentum exchange over the active blocks (one
// workgroup per level, fixed summation order): out[L][0..2].
__global__ __launch_bounds__(256) void k_force_sum(DevMesh m, double *out) {
    __shared__ double s[3][256];
    const int L = blockIdx.x, t = threadIdx.x;
    double a[3] = {0.0, 0.0, 0.0};
    for (int B = t; B < m.cap; B += 256) {
        if (m.status[B] == ST_INACTIVE || m.level[B] != L) continue;
        for (int c = 0; c < 3; c++) a[c] += m.force[(int64_t)B * 3 + c];
    }
    for (int c = 0; c < 3; c++) s[c][t] = a[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 3; c++) s[c][t] += s[c][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int c = 0; c < 3; c++) out[L * 3 + c] = s[c][0];
}

__global__ void k_force_reset(DevMesh m) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)m.cap * 3) m.force[e] = 0.0;
}

void launch_force_sum(const Ctx &c, double *out) { k_force_sum<<<c.m.lmax, 256, 0, c.stream>>>(c.m, out); }

void launch_force_reset(const Ctx &c) {
    const int64_t n = (int64_t)c.m.cap * 3;
    k_force_reset<<<(int)((n + 255) / 256), 256, 0, c.stream>>>(c.m);
}

// ---------------------------------------------------------------------------
// initial states: every slot at rest (g = 0, f = w)
template <int Q, int S>
__global__ void k_fill_rest(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1, int64_t total) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    R v = R(0);
    if (!ST::shift && e < m.halo_base) {
        const int p = (int)((e / Lt::MB) % Q);
        v = R(Lt::w(p));
    }
    ST::st(f0 + e, v);
    ST::st(f1 + e, v);
}

// Block-parallel kernels below run 256/Mb blocks per 256-thread workgroup
// over a contiguous block-ID range [b0, b1).

// f = feq(rho, u) of root cells from (rho, ux, uy, uz), ru[((B - b0) Mb + l) 4]
template <int Q, int S>
__global__ __launch_bounds__(256) void k_set_rho_u(DevMesh m, typename Store<S>::T *f, const double *__restrict__ ru,
                                                   int b0, int b1) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    if ((int)threadIdx.x < BPW) {
        const int B = b0 + blockIdx.x * BPW + threadIdx.x;
        st.id[threadIdx.x] = (B < b1 && m.status[B] != ST_INACTIVE) ? B : -1;
    }
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int B = st.id[s];
    if (B < 0) return;
    const double *v = ru + ((int64_t)(B - b0) * MB + l) * 4;
    const double rho = v[0], ux = v[1], uy = v[2], uz = v[3];
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int p = 0; p < Q; p++) {
        const double cu = Lt::cx(p) * ux + Lt::cy(p) * uy + Lt::cz(p) * uz;
        const double val = ST::shift ? Lt::w(p) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu))
                                     : Lt::w(p) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        ST::st(f + entry_slot<Lt>(m, st.link[s], B, st.hid[s], p, l), R(val));
    }
}

// ---------------------------------------------------------------------------
// Vorticity criterion, FP64 (Sec. "Adaptive Mesh Refinement" of the solver).
// First the FP64 velocity of every cell of a level, then central differences
// over same-level neighbour cells (one-sided where a neighbour is missing),
// scaled to root-cell units; block maximum per leaf and the global maximum
// (atomic max on the bit pattern of a non-negative double).
template <typename Lt, typename ST>
__device__ inline void cell_f64(const DevMesh &m, const int32_t *link, int B, int h, int l,
                                const typename ST::T *f, double *fv) {
#pragma unroll
    for (int p = 0; p < Lt::Q; p++)
        fv[p] = double(ST::ld(f + entry_slot<Lt>(m, link, B, h, p, l))) + (ST::shift ? Lt::w(p) : 0.0);
}

// children = 0: `list` holds the blocks.  children = 1: `list` holds parents
// (the interface parents of the level above) and the kernel takes those of
// their children that have an N_SKIP link: after k_average with VEL, the only
// blocks below level 0 whose velocities are still missing.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_velocity(const int32_t *__restrict__ list, int n, DevMesh m,
                                                  const typename Store<S>::T *__restrict__ f, double *U,
                                                  int children) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    __shared__ int any;
    const int base = blockIdx.x * BPW;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if ((int)threadIdx.x < BPW) {
        const int64_t i = (int64_t)base + threadIdx.x;
        int B = -1;
        if (!children) {
            if (i < n) B = list[i];
        } else if (i < (int64_t)n * Lt::NC) {
            const int c0 = m.nbrc[list[i / Lt::NC]];
            const int C = c0 + (int)(i % Lt::NC);
            if (c0 >= 0 && (m.bflag[C] & BF_NSKIP)) B = C;
        }
        st.id[threadIdx.x] = B;
        if (B >= 0) any = 1;
    }
    __syncthreads();
    if (!any) return;  // the whole workgroup: nothing to stage
    stage_blocks<Lt, BPW>(m, st);
    __shared__ uint64_t tab[Lt::D == 3 ? BPW : 1][27];
    if constexpr (Lt::D == 3) {
        fill_row_tables<Lt, BPW>(st, [&](int) -> const DevMesh & { return m; }, [&](int) { return f; }, tab);
        __syncthreads();
    }
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int B = st.id[s];
    if (B < 0) return;
    if (!velocity_read<Lt>(m, st.link[s], B)) return;
    double fv[Q];
    bool done = false;
    if constexpr (Lt::D == 3) {
        if (!(st.flag[s] & (BF_BOUNDARY | BF_NSKIP))) {
            // the same values as cell_f64, through the row table
            gather_interior_by<Lt, ST, 0>(interior_lane<typename ST::T>(tab[s], l & 3, (l >> 2) & 3, l >> 4), fv,
                                          [](typename ST::R v, int p) {
                                              return double(v) + (ST::shift ? Lt::w(p) : 0.0);
                                          });
            done = true;
        }
    }
    if (!done) cell_f64<Lt, ST>(m, st.link[s], B, st.hid[s], l, f, fv);
    cell_velocity<Lt>(fv, U, m.capc, (int64_t)B * MB + l);
}

template <int Q>
__global__ __launch_bounds__(256) void k_vorticity(const int32_t *__restrict__ list, int n, DevMesh m,
                                                   const double *__restrict__ U, double scale, double *crit,
                                                   unsigned long long *wmax_bits) {
    using Lt = Lat<Q>;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    const int base = blockIdx.x * BPW;
    if ((int)threadIdx.x < BPW) st.id[threadIdx.x] = base + (int)threadIdx.x < n ? list[base + threadIdx.x] : -1;
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int B = st.id[s];
    const bool leaf = B >= 0 && m.status[B] == ST_UNREF;
    const int ci[3] = {l & 3, (l >> 2) & 3, l >> 4};
    // the neighbour cells along +-x, +-y (+-z): those in other blocks are read
    // here, all loads at once and before the barrier; those inside the block
    // come from the block's own velocities in LDS below
    double nv[3][2][3] = {};
    int nlc[3][2];
    bool nhas[3][2], nin[3][2];
#pragma unroll
    for (int a = 0; a < Lt::D; a++)
#pragma unroll
        for (int sg = 0; sg < 2; sg++) {
            int t[3] = {ci[0], ci[1], ci[2]};
            t[a] += sg == 0 ? 1 : -1;
            const int rg = region_of<Lt>(t[0], t[1], t[2]);
            const int32_t code = leaf ? st.link[s][rg] : -1;
            nhas[a][sg] = code >= 0 && code < m.cap;
            nin[a][sg] = rg == kCenterSlot<Lt>;
            nlc[a][sg] = (t[0] & 3) + 4 * (t[1] & 3) + 16 * (t[2] & 3);
            if (nhas[a][sg] && !nin[a][sg]) {
                const int64_t nc = (int64_t)code * MB + nlc[a][sg];
#pragma unroll
                for (int b = 0; b < 3; b++) nv[a][sg][b] = U[b * m.capc + nc];
            }
        }
    // the velocities of the block's own cells, for the neighbours inside it
    __shared__ double us[BPW][3][MB];
    if (leaf)
        for (int b = 0; b < 3; b++) us[s][b][l] = U[b * m.capc + (int64_t)B * MB + l];
    __syncthreads();
    double w = 0.0;
    if (leaf) {
        double u0[3];
        for (int b = 0; b < 3; b++) u0[b] = us[s][b][l];
        double gr[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) gr[a][b] = 0.0;
#pragma unroll
        for (int a = 0; a < Lt::D; a++) {
            double up[3], um[3];
            bool hp = false, hm = false;
#pragma unroll
            for (int sg = 0; sg < 2; sg++) {
                if (!nhas[a][sg]) continue;
                double *dstv = sg == 0 ? up : um;
#pragma unroll
                for (int b = 0; b < 3; b++) dstv[b] = nin[a][sg] ? us[s][b][nlc[a][sg]] : nv[a][sg][b];
                if (sg == 0) hp = true; else hm = true;
            }
#pragma unroll
            for (int b = 0; b < 3; b++) {
                if (hp && hm) gr[a][b] = (up[b] - um[b]) / 2.0;
                else if (hp) gr[a][b] = up[b] - u0[b];
                else if (hm) gr[a][b] = u0[b] - um[b];
            }
        }
        if (Lt::D == 2) {
            w = fabs(gr[0][1] - gr[1][0]) * scale;
        } else {
            const double wx = gr[1][2] - gr[2][1], wy = gr[2][0] - gr[0][2], wz = gr[0][1] - gr[1][0];
            w = sqrt(wx * wx + wy * wy + wz * wz) * scale;
        }
    }
    // block maximum over the MB lanes of the block
#pragma unroll
    for (int off = MB / 2; off > 0; off >>= 1) w = fmax(w, __shfl_xor(w, off, 64));
    if (leaf && l == 0) {
        crit[B] = w;
        // the running maximum rarely grows: compare first, so that most blocks
        // skip the atomic on the one shared address
        const unsigned long long bits = (unsigned long long)__double_as_longlong(w);
        if (bits > __hip_atomic_load(wmax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(wmax_bits, bits);
    }
}

// ---------------------------------------------------------------------------
// Gathers / scatters of unshifted FP64 data through the staging buffer.
// Every cell of every active block, [B - b0][l][q]; inactive blocks read 0.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_block_f(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1,
                                                 LevelParams lp, int set, int b0, int b1, double *stage) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    if ((int)threadIdx.x < BPW) {
        const int B = b0 + blockIdx.x * BPW + threadIdx.x;
        st.id[threadIdx.x] = (B < b1 && m.status[B] != ST_INACTIVE) ? B : -1;
    }
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int Braw = b0 + blockIdx.x * BPW + s;
    if (Braw >= b1) return;
    double *row = stage + ((int64_t)(Braw - b0) * MB + l) * Q;
    const int B = st.id[s];
    if (B < 0) {
        if (!set)
            for (int p = 0; p < Q; p++) row[p] = 0.0;
        return;
    }
    typename ST::T *f = lp.par[m.level[B]] ? f1 : f0;
    if (set) {
#pragma unroll
        for (int p = 0; p < Q; p++)
            ST::st(f + entry_slot<Lt>(m, st.link[s], B, st.hid[s], p, l), R(row[p] - (ST::shift ? Lt::w(p) : 0.0)));
    } else {
        cell_f64<Lt, ST>(m, st.link[s], B, st.hid[s], l, f, row);
    }
}

// output cells: leaf, non-ghost cells in (block ID, cell) order; kind: cells,
// rho/u, or f
template <int Q, int S>
__global__ __launch_bounds__(256) void k_out_gather(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1,
                                                    LevelParams lp, int kind, int b0, int b1,
                                                    const int32_t *__restrict__ off, int32_t off0, void *stage) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lt, BPW> st;
    if ((int)threadIdx.x < BPW) {
        const int B = b0 + blockIdx.x * BPW + threadIdx.x;
        st.id[threadIdx.x] = (B < b1 && m.status[B] == ST_UNREF) ? B : -1;
    }
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int B = st.id[s];
    if (B < 0) return;
    const uint64_t full = MB == 64 ? ~0ull : ((1ull << MB) - 1);
    const uint64_t outm = ~m.gmask[B] & full;
    if (!((outm >> l) & 1ull)) return;
    const int64_t pos = (int64_t)off[B] - off0 + __popcll(outm & ((1ull << l) - 1));
    if (kind == AMR_FIELD_CELLS) {
        int32_t *o = (int32_t *)stage + 2 * pos;
        o[0] = B;
        o[1] = l;
        return;
    }
    const typename ST::T *f = lp.par[m.level[B]] ? f1 : f0;
    double fv[Q];
    cell_f64<Lt, ST>(m, st.link[s], B, st.hid[s], l, f, fv);
    if (kind == AMR_FIELD_RHO_U) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < Q; p++) {
            rho += fv[p];
            j[0] += fv[p] * Lt::cx(p);
            j[1] += fv[p] * Lt::cy(p);
            j[2] += fv[p] * Lt::cz(p);
        }
        double *o = (double *)stage + 4 * pos;
        o[0] = rho;
        o[1] = j[0] / rho;
        o[2] = j[1] / rho;
        o[3] = j[2] / rho;
    } else {
        double *o = (double *)stage + Q * pos;
#pragma unroll
        for (int p = 0; p < Q; p++) o[p] = fv[p];
    }
}

// FP64 mass and momentum of the output cells: fixed-order per-block partials,
// then a single-workgroup fixed-order sum.
//
// Body: the partial of the staged blocks with first ID b (256 threads, Mb per
// block); lane 0 of each block's group returns it in v.
template <int Q, int S>
__device__ __forceinline__ void mass_block_partial(const DevMesh &m, typename Store<S>::T *f0,
                                                   typename Store<S>::T *f1, const LevelParams &lp,
                                                   BlockStage<Lat<Q>, 256 / Lat<Q>::MB> &st, int64_t b, double *v) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    constexpr int MB = Lt::MB, BPW = 256 / MB;
    if ((int)threadIdx.x < BPW) {
        const int64_t B = b + threadIdx.x;
        st.id[threadIdx.x] = (B < m.cap && m.status[B] == ST_UNREF) ? (int)B : -1;
    }
    __syncthreads();
    stage_blocks<Lt, BPW>(m, st);
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int B = st.id[s];
    for (int a = 0; a < 4; a++) v[a] = 0.0;
    if (B >= 0 && !((m.gmask[B] >> l) & 1ull)) {
        const int L = m.level[B];
        const typename ST::T *f = lp.par[L] ? f1 : f0;
        double fv[Q];
        cell_f64<Lt, ST>(m, st.link[s], B, st.hid[s], l, f, fv);
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < Q; p++) {
            rho += fv[p];
            j[0] += fv[p] * Lt::cx(p);
            j[1] += fv[p] * Lt::cy(p);
            j[2] += fv[p] * Lt::cz(p);
        }
        const double vol = 1.0 / double(1 << (Lt::D * L));
        v[0] = vol * rho;
        for (int a = 0; a < 3; a++) v[1 + a] = vol * rho * (j[a] / rho);
    }
#pragma unroll
    for (int off = MB / 2; off > 0; off >>= 1)
        for (int a = 0; a < 4; a++) v[a] += __shfl_xor(v[a], off, 64);
}

template <int Q, int S>
__global__ __launch_bounds__(256) void k_mass_blocks(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1,
                                                     LevelParams lp, double *part4) {
    constexpr int MB = Lat<Q>::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lat<Q>, BPW> st;
    double v[4];
    mass_block_partial<Q, S>(m, f0, f1, lp, st, (int64_t)blockIdx.x * BPW, v);
    const int64_t Braw = (int64_t)blockIdx.x * BPW + threadIdx.x / MB;
    if (Braw < m.cap && threadIdx.x % MB == 0)
        for (int a = 0; a < 4; a++) part4[Braw * 4 + a] = v[a];
}

// Fixed-order sums of the per-block partials: each workgroup reduces one chunk
// of kMassChunk blocks and leaves the result in the chunk's first entry (which
// no other workgroup reads); one workgroup then reduces the chunk results.
constexpr int kMassChunk = 4096;

__device__ inline void tree_sum4(double (*s)[256], double *v) {
    for (int a = 0; a < 4; a++) s[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 4; a++) s[a][threadIdx.x] += s[a][threadIdx.x + w];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_mass_chunks(double *part4, int cap) {
    __shared__ double s[4][256];
    const int64_t b0 = (int64_t)blockIdx.x * kMassChunk;
    const int64_t b1 = b0 + kMassChunk < cap ? b0 + kMassChunk : cap;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t B = b0 + threadIdx.x; B < b1; B += 256)
        for (int a = 0; a < 4; a++) v[a] += part4[B * 4 + a];
    tree_sum4(s, v);  // ends with a barrier: every read of the chunk is done
    if (threadIdx.x < 4) part4[b0 * 4 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_mass_final(const double *part4, int cap, double *out) {
    __shared__ double s[4][256];
    const int nchunk = (cap + kMassChunk - 1) / kMassChunk;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < nchunk; c += 256)
        for (int a = 0; a < 4; a++) v[a] += part4[(int64_t)c * kMassChunk * 4 + a];
    tree_sum4(s, v);
    if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

// The same sums without the arena's per-block partials, for callers that cannot
// allocate: one workgroup per chunk of kMassChunk blocks forms the block
// partials itself, BPW blocks at a time, and adds them in the order the
// per-chunk pass above does (thread t: blocks b0 + t, b0 + t + 256, ...); the
// chunk sums go to `chunks` (kMassStaticChunks entries at most), and the final
// pass is the same as above.  The result equals the arena form bit for bit.
constexpr int kMassStaticChunks = 1024;  // blocks up to 1024 * kMassChunk = 4,194,304

template <int Q, int S>
__global__ __launch_bounds__(256) void k_mass_chunks_direct(DevMesh m, typename Store<S>::T *f0,
                                                            typename Store<S>::T *f1, LevelParams lp,
                                                            double *chunks) {
    constexpr int MB = Lat<Q>::MB, BPW = 256 / MB;
    __shared__ BlockStage<Lat<Q>, BPW> st;
    __shared__ double s_part[256][4];
    __shared__ double s[4][256];
    const int64_t b0 = (int64_t)blockIdx.x * kMassChunk;
    const int t = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < kMassChunk / 256; r++) {
        for (int i = 0; i < 256 / BPW; i++) {
            double v[4];
            mass_block_partial<Q, S>(m, f0, f1, lp, st, b0 + 256 * r + BPW * i, v);
            if (t % MB == 0)
                for (int a = 0; a < 4; a++) s_part[BPW * i + t / MB][a] = v[a];
            __syncthreads();  // the stage is rewritten by the next group
        }
        if (b0 + 256 * r + t < m.cap)
            for (int a = 0; a < 4; a++) acc[a] += s_part[t][a];
        __syncthreads();
    }
    tree_sum4(s, acc);
    if (t < 4) chunks[(int64_t)blockIdx.x * 4 + t] = s[t][0];
}

__global__ __launch_bounds__(256) void k_mass_final_direct(const double *chunks, int cap, double *out) {
    __shared__ double s[4][256];
    const int nchunk = (cap + kMassChunk - 1) / kMassChunk;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < nchunk; c += 256)
        for (int a = 0; a < 4; a++) v[a] += chunks[(int64_t)c * 4 + a];
    tree_sum4(s, v);
    if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

// The chunk sums' storage: a fixed array in device memory, one copy per GPU
// for the life of the process.  Host code uses the address resolved once per
// device with hipGetSymbolAddress (mass_scratch), never the array's name.
static __device__ __align__(256) double scratch[kMassStaticChunks * 4];

// ---------------------------------------------------------------------------
// dispatch over (lattice, storage)
#define AMR_DISPATCH(qv, sv, BODY)                                                \
    do {                                                                          \
        switch ((qv) * 8 + (sv)) {                                                \
        case 9 * 8 + AMR_F64: { constexpr int Qc = 9, Sc = AMR_F64; BODY; } break;   \
        case 9 * 8 + AMR_F32: { constexpr int Qc = 9, Sc = AMR_F32; BODY; } break;   \
        case 9 * 8 + AMR_F32S: { constexpr int Qc = 9, Sc = AMR_F32S; BODY; } break; \
        case 9 * 8 + AMR_F16S: { constexpr int Qc = 9, Sc = AMR_F16S; BODY; } break; \
        case 9 * 8 + AMR_BF16S: { constexpr int Qc = 9, Sc = AMR_BF16S; BODY; } break; \
        case 19 * 8 + AMR_F64: { constexpr int Qc = 19, Sc = AMR_F64; BODY; } break;   \
        case 19 * 8 + AMR_F32: { constexpr int Qc = 19, Sc = AMR_F32; BODY; } break;   \
        case 19 * 8 + AMR_F32S: { constexpr int Qc = 19, Sc = AMR_F32S; BODY; } break; \
        case 19 * 8 + AMR_F16S: { constexpr int Qc = 19, Sc = AMR_F16S; BODY; } break; \
        case 19 * 8 + AMR_BF16S: { constexpr int Qc = 19, Sc = AMR_BF16S; BODY; } break; \
        case 27 * 8 + AMR_F64: { constexpr int Qc = 27, Sc = AMR_F64; BODY; } break;   \
        case 27 * 8 + AMR_F32: { constexpr int Qc = 27, Sc = AMR_F32; BODY; } break;   \
        case 27 * 8 + AMR_F32S: { constexpr int Qc = 27, Sc = AMR_F32S; BODY; } break; \
        case 27 * 8 + AMR_F16S: { constexpr int Qc = 27, Sc = AMR_F16S; BODY; } break; \
        case 27 * 8 + AMR_BF16S: { constexpr int Qc = 27, Sc = AMR_BF16S; BODY; } break; \
        default: break;                                                           \
        }                                                                         \
    } while (0)

#define TPTR(Sc, p) ((typename Store<Sc>::T *)(p))

static inline int grid_blocks(int64_t nblocks, int mb) {
    const int bpw = 256 / mb;
    return (int)((nblocks + bpw - 1) / bpw);
}

// A level sweep whose output exceeds c.stream_bytes (by default half the 256 MB
// Infinity Cache) stores with non-temporal writes.  Smaller levels are still
// cached when the next sweep (or the interpolation and averaging) reads them.
template <int Q, int S>
static bool collide_stream_nts(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp,
                               const BCParams &bc, bool exchange) {
    using T = typename Store<S>::T;
    const int sp = lp.par[L];
    constexpr int bpw = collide_blocks_per_wg<Q, S>();
    const int grid = (n + bpw - 1) / bpw;
    const T *src = (const T *)c.f[sp];
    T *dst = (T *)c.f[1 - sp];
    const bool nts = (int64_t)n * Q * c.mb * (int64_t)sizeof(T) > c.stream_bytes;
    const int tpb = collide_threads<S>();
    const double om = lp.omega[L];
    if constexpr (Q == 27) {
        if (c.coll == AMR_COLLIDE_MRT) {
            if (nts) k_collide_stream<Q, S, true, 1><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, c.s_high);
            else k_collide_stream<Q, S, false, 1><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, c.s_high);
            return false;
        }
        if constexpr (S != AMR_F64) {
            if (c.coll == AMR_COLLIDE_MRT_MFMA) {
                if (nts) k_collide_stream<Q, S, true, 2><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, c.s_high);
                else k_collide_stream<Q, S, false, 2><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, c.s_high);
                return false;
            }
        }
    }
    if (exchange && !nts) {
        k_collide_stream<Q, S, false, 0, true><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, om);
        return true;
    }
    if (nts) k_collide_stream<Q, S, true><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, om);
    else k_collide_stream<Q, S, false><<<grid, tpb, 0, c.stream>>>(list, n, c.m, src, dst, om, bc, om);
    return false;
}

bool launch_collide_stream(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp, const BCParams &bc,
                           bool exchange) {
    if (n <= 0) return false;
    bool done = false;
    AMR_DISPATCH(c.q, c.storage, (done = collide_stream_nts<Qc, Sc>(c, list, n, L, lp, bc, exchange)));
    return done;
}

template <int Q, int S>
static bool interp_collide(const Ctx &c, const int32_t *ilist, int ni, const int32_t *clist, int nblk, int L,
                           const LevelParams &lp, const BCParams &bc, bool exchange) {
    using T = typename Store<S>::T;
    constexpr int bpw = collide_blocks_per_wg<Q, S>();
    const int grid = ni + (nblk + bpw - 1) / bpw;
    const bool nts = (int64_t)nblk * Q * c.mb * (int64_t)sizeof(T) > c.stream_bytes;
    T *f0 = (T *)c.f[0], *f1 = (T *)c.f[1];
    if (exchange && !nts) {
        if (c.m.interp == AMR_INTERP_CUBIC)
            k_interp_collide<Q, S, false, 1, true><<<grid, 256, 0, c.stream>>>(ilist, ni, clist, nblk, c.m, f0, f1, lp, L, bc);
        else
            k_interp_collide<Q, S, false, 0, true><<<grid, 256, 0, c.stream>>>(ilist, ni, clist, nblk, c.m, f0, f1, lp, L, bc);
        return true;
    }
    if (c.m.interp == AMR_INTERP_CUBIC) {
        if (nts) k_interp_collide<Q, S, true, 1><<<grid, 256, 0, c.stream>>>(ilist, ni, clist, nblk, c.m, f0, f1, lp, L, bc);
        else k_interp_collide<Q, S, false, 1><<<grid, 256, 0, c.stream>>>(ilist, ni, clist, nblk, c.m, f0, f1, lp, L, bc);
    } else {
        if (nts) k_interp_collide<Q, S, true, 0><<<grid, 256, 0, c.stream>>>(ilist, ni, clist, nblk, c.m, f0, f1, lp, L, bc);
        else k_interp_collide<Q, S, false, 0><<<grid, 256, 0, c.stream>>>(ilist, ni, clist, nblk, c.m, f0, f1, lp, L, bc);
    }
    return false;
}

bool launch_interp_collide(const Ctx &c, const int32_t *ilist, int ni, const int32_t *clist, int nblk, int L,
                           const LevelParams &lp, const BCParams &bc, bool exchange) {
    bool done = false;
    AMR_DISPATCH(c.q, c.storage, (done = interp_collide<Qc, Sc>(c, ilist, ni, clist, nblk, L, lp, bc, exchange)));
    return done;
}

void launch_interp(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells) {
    if (n <= 0) return;
    const int threads = c.dim == 2 ? 64 : 256;
    if (c.m.interp == AMR_INTERP_CUBIC)
        AMR_DISPATCH(c.q, c.storage,
                     (k_interp<Qc, Sc, 1><<<n, threads, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[0]),
                                                                        TPTR(Sc, c.f[1]), lp, all_cells)));
    else
        AMR_DISPATCH(c.q, c.storage,
                     (k_interp<Qc, Sc, 0><<<n, threads, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[0]),
                                                                        TPTR(Sc, c.f[1]), lp, all_cells)));
}

void launch_exchange(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp) {
    if (n <= 0) return;
    const int bpw = 256 / c.mb;
    AMR_DISPATCH(c.q, c.storage,
                 (k_exchange<Qc, Sc><<<(n + bpw - 1) / bpw, 256, 0, c.stream>>>(list, n, c.m,
                                                                               TPTR(Sc, c.f[lp.par[L]]))));
}

void launch_exchange_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                           const int32_t *count, int par, int grid) {
    AMR_DISPATCH(q, storage, (k_exchange_batch<Qc, Sc><<<grid, 256, 0, stream>>>(sims, items, count, par)));
}

template <int Q, int S>
static void collide_batch_shape(hipStream_t stream, const SimDesc *sims, const uint32_t *items, const int32_t *count,
                                int L, int par, int nt, int grid) {
    if (nt == 64)
        k_collide_stream_batch<Q, S, 64><<<grid, 64, 0, stream>>>(sims, items, count, L, par);
    else if (nt == 128)
        k_collide_stream_batch<Q, S, 128><<<grid, 128, 0, stream>>>(sims, items, count, L, par);
    else
        k_collide_stream_batch<Q, S, 256><<<grid, 256, 0, stream>>>(sims, items, count, L, par);
}

void launch_collide_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                          const int32_t *count, int L, int par, int nt, int grid) {
    AMR_DISPATCH(q, storage, (collide_batch_shape<Qc, Sc>(stream, sims, items, count, L, par, nt, grid)));
}

void launch_interp_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                         const int32_t *count, int L, int par0, int par1, int grid) {
    const int threads = q == 9 ? 64 : 256;
    AMR_DISPATCH(q, storage,
                 (k_interp_batch<Qc, Sc><<<grid, threads, 0, stream>>>(sims, items, count, L, par0, par1)));
}

void launch_average_batch(hipStream_t stream, int q, int storage, const SimDesc *sims, const uint32_t *items,
                          const int32_t *count, int L, int par0, int par1, int grid) {
    const int threads = q == 9 ? 64 : 256;  // one lane per fine cell of the workgroup's children
    AMR_DISPATCH(q, storage,
                 (k_average_batch<Qc, Sc><<<grid, threads, 0, stream>>>(sims, items, count, L, par0, par1)));
}

void launch_batch_items(hipStream_t stream, const SimDesc *sims, int nsims, int lmax, int cap_max, uint32_t *items,
                        int64_t stride, int32_t *counts) {
    if (nsims <= 0 || lmax <= 0) return;
    const int chunks = std::min(64, (cap_max + 255) / 256);
    k_batch_items<<<dim3(chunks, nsims, 3 * lmax), 256, 0, stream>>>(sims, nsims, items, stride, counts);
}

void launch_refresh_neighbours(const Ctx &c, const int32_t *list, int n, const LevelParams &lp) {
    if (n <= 0) return;
    const int threads = c.dim == 2 ? 64 : 256;
    AMR_DISPATCH(c.q, c.storage,
                 (k_refresh_neighbours<Qc, Sc><<<n, threads, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[0]),
                                                                             TPTR(Sc, c.f[1]), lp)));
    k_clear_fresh<<<(n * c.nc + 255) / 256, 256, 0, c.stream>>>(list, n, c.m, c.nc);
}

template <int Q, int S>
static void average(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells, double *U) {
    using T = typename Store<S>::T;
    // one lane per fine cell of the workgroup's children; 3-D: two workgroups per parent
    const int split = c.dim == 3 ? 2 : 1;
    const int threads = c.nc / split * c.mb;
    T *f0 = (T *)c.f[0], *f1 = (T *)c.f[1];
    if (U) k_average<Q, S, true><<<n * split, threads, 0, c.stream>>>(list, n, c.m, f0, f1, lp, 1, U);
    else k_average<Q, S><<<n * split, threads, 0, c.stream>>>(list, n, c.m, f0, f1, lp, all_cells, nullptr);
}

void launch_average(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells, double *U) {
    if (n <= 0) return;
    AMR_DISPATCH(c.q, c.storage, (average<Qc, Sc>(c, list, n, lp, all_cells, U)));
}

void launch_fill_rest(const Ctx &c) {
    const int64_t total = c.m.halo_base + (int64_t)c.m.cap * c.m.nh;
    const int grid = (int)((total + 255) / 256);
    AMR_DISPATCH(c.q, c.storage,
                 (k_fill_rest<Qc, Sc><<<grid, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), total)));
}

void launch_set_rho_u_root(const Ctx &c, const double *ru, int b0, int b1) {
    if (b1 <= b0) return;
    AMR_DISPATCH(c.q, c.storage,
                 (k_set_rho_u<Qc, Sc><<<grid_blocks(b1 - b0, c.mb), 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), ru,
                                                                                         b0, b1)));
}

void launch_velocity(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp, bool children) {
    if (n <= 0) return;
    const int64_t items = children ? (int64_t)n * c.nc : n;
    AMR_DISPATCH(c.q, c.storage,
                 (k_velocity<Qc, Sc><<<grid_blocks(items, c.mb), 256, 0, c.stream>>>(
                     list, n, c.m, TPTR(Sc, c.f[lp.par[L]]), c.U, children ? 1 : 0)));
}

void launch_vorticity(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &) {
    if (n <= 0) return;
    const double scale = double(1 << L);
    const int grid = grid_blocks(n, c.mb);
    if (c.q == 9) k_vorticity<9><<<grid, 256, 0, c.stream>>>(list, n, c.m, c.U, scale, c.crit, &c.ctr->wmax_bits);
    else if (c.q == 19) k_vorticity<19><<<grid, 256, 0, c.stream>>>(list, n, c.m, c.U, scale, c.crit, &c.ctr->wmax_bits);
    else k_vorticity<27><<<grid, 256, 0, c.stream>>>(list, n, c.m, c.U, scale, c.crit, &c.ctr->wmax_bits);
}

void launch_block_f(const Ctx &c, int set, int b0, int b1, double *stage, const LevelParams &lp) {
    if (b1 <= b0) return;
    AMR_DISPATCH(c.q, c.storage,
                 (k_block_f<Qc, Sc><<<grid_blocks(b1 - b0, c.mb), 256, 0, c.stream>>>(
                     c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), lp, set, b0, b1, stage)));
}

void launch_out_gather(const Ctx &c, int kind, int b0, int b1, int32_t off0, void *stage, const LevelParams &lp) {
    if (b1 <= b0) return;
    AMR_DISPATCH(c.q, c.storage,
                 (k_out_gather<Qc, Sc><<<grid_blocks(b1 - b0, c.mb), 256, 0, c.stream>>>(
                     c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), lp, kind, b0, b1, c.off, off0, stage)));
}

int64_t mass_static_max_blocks() { return (int64_t)kMassStaticChunks * kMassChunk; }

hipError_t mass_scratch(int device, double **ptr) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {nullptr};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // resolved with its device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

void launch_mass_static(const Ctx &c, const LevelParams &lp, double *chunks, double *out_dev) {
    const int nchunk = (c.m.cap + kMassChunk - 1) / kMassChunk;
    AMR_DISPATCH(c.q, c.storage,
                 (k_mass_chunks_direct<Qc, Sc><<<nchunk, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]),
                                                                            TPTR(Sc, c.f[1]), lp, chunks)));
    k_mass_final_direct<<<1, 256, 0, c.stream>>>(chunks, c.m.cap, out_dev);
}

void launch_mass(const Ctx &c, const LevelParams &lp) {
    AMR_DISPATCH(c.q, c.storage,
                 (k_mass_blocks<Qc, Sc><<<grid_blocks(c.m.cap, c.mb), 256, 0, c.stream>>>(
                     c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), lp, c.part4)));
    k_mass_chunks<<<(c.m.cap + kMassChunk - 1) / kMassChunk, 256, 0, c.stream>>>(c.part4, c.m.cap);
    k_mass_final<<<1, 256, 0, c.stream>>>(c.part4, c.m.cap, c.ctr->mass);
}

}  // namespace amr
