// lbm_kernels.hip -- lattice Boltzmann kernels of the AMR-LBM library for
// gfx950: fused BGK collide + push stream per level sweep, coarse-to-fine
// linear interpolation, fine-to-coarse averaging, the vorticity criterion and
// field gathers.  Arithmetic is written in the "shifted" variables g = f - w
// for every storage format (FP64 storage computes in FP64, the rest in FP32).
#include "kernels.h"

namespace amr {

#define HIP_LAUNCH_CHECK() (void)hipGetLastError()

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

// deviation of the second-order equilibrium from the rest state, w (rho - 1) +
// w rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
template <typename Lt, typename R>
__device__ inline R geq(int p, R drho, R ux, R uy, R uz, R uu) {
    const R cu = R(Lt::cx(p)) * ux + R(Lt::cy(p)) * uy + R(Lt::cz(p)) * uz;
    const R rho = R(1) + drho;
    return R(Lt::w(p)) * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
}

template <typename Lt, typename ST>
__device__ inline void load_g(const typename ST::T *__restrict__ f, int64_t capc, int64_t cell, typename ST::R *g) {
    using R = typename ST::R;
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) {
        const R v = ST::ld(f + p * capc + cell);
        g[p] = ST::shift ? v : v - R(Lt::w(p));
    }
}

template <typename Lt, typename ST>
__device__ inline void store_g(typename ST::T *__restrict__ f, int64_t capc, int64_t cell, int p, typename ST::R g) {
    using R = typename ST::R;
    ST::st(f + p * capc + cell, ST::shift ? g : g + R(Lt::w(p)));
}

// ---------------------------------------------------------------------------
// Fused collide + push stream of one level (Secs. "Streaming", "Collision").
// One 4^d block per 64-lane group (3-D: one block per wave; 2-D: four blocks
// per wave); each workgroup stages the link tables of its blocks in LDS,
// indexed by neighbour-offset slot.  Pushes that leave the fluid turn into the
// boundary value in the opposite slot of the same cell; slots whose source is
// an N_SKIP region keep the cell's own post-collision value.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_collide_stream(const int32_t *__restrict__ list, int n, DevMesh m,
                                                        const typename Store<S>::T *__restrict__ src,
                                                        typename Store<S>::T *__restrict__ dst, double omega_d,
                                                        BCParams bc) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr int MB = Lt::MB, BPW = 256 / MB, NS = Lt::D == 2 ? 9 : 27;
    __shared__ int32_t s_link[BPW][NS];
    __shared__ int32_t s_id[BPW];
    __shared__ uint8_t s_flag[BPW];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int base = wg * BPW;
    for (int e = threadIdx.x; e < BPW * Lt::NB; e += 256) {
        const int s = e / Lt::NB, p = e - s * Lt::NB;
        const int idx = base + s;
        int32_t v = 0;
        if (idx < n) {
            const int B = list[idx];
            v = m.nbr[(int64_t)p * m.cap + B];
            if (p == 0) {
                s_id[s] = B;
                s_flag[s] = m.bflag[B];
            }
        }
        s_link[s][offset_slot(Lt::cx(p), Lt::cy(p), Lt::cz(p)) - (Lt::D == 2 ? 9 : 0)] = v;
    }
    __syncthreads();
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    if (base + s >= n) return;
    const int B = s_id[s];
    const uint8_t flag = s_flag[s];
    const int i = l & 3, j = (l >> 2) & 3, k = l >> 4;
    const int64_t cell = (int64_t)B * MB + l;
    const int64_t capc = m.capc;

    R g[Q];
    load_g<Lt, ST>(src, capc, cell, g);
    R drho, ux, uy, uz;
    moments_g<Lt, R>(g, drho, ux, uy, uz);
    const R uu = ux * ux + uy * uy + uz * uz;
    const R om = R(omega_d);
#pragma unroll
    for (int p = 0; p < Q; p++) g[p] += om * (geq<Lt, R>(p, drho, ux, uy, uz, uu) - g[p]);

#pragma unroll
    for (int p = 0; p < Q; p++) {
        const int tx = i + Lt::cx(p), ty = j + Lt::cy(p), tz = k + Lt::cz(p);
        const int rx = tx < 0 ? -1 : (tx > 3 ? 1 : 0);
        const int ry = ty < 0 ? -1 : (ty > 3 ? 1 : 0);
        const int rz = tz < 0 ? -1 : (tz > 3 ? 1 : 0);
        const int32_t code = s_link[s][offset_slot(rx, ry, rz) - (Lt::D == 2 ? 9 : 0)];
        if (code >= 0) {
            if (code >= m.cap) continue;  // never taken for a consistent forest
            const int lt = (tx & 3) + 4 * (ty & 3) + 16 * (tz & 3);
            store_g<Lt, ST>(dst, capc, (int64_t)code * MB + lt, p, g[p]);
        } else if ((flag & BF_BOUNDARY) && code != kNSkip) {
            R val;
            if (code == kSolid) {
                val = g[p];
            } else {
                const int face = -3 - code;
                const R cx = R(Lt::cx(p)), cy = R(Lt::cy(p)), cz = R(Lt::cz(p));
                if (bc.kind[face] == AMR_FACE_VELOCITY) {
                    const R cuw = cx * R(bc.u[face][0]) + cy * R(bc.u[face][1]) + cz * R(bc.u[face][2]);
                    val = g[p] - R(6) * R(Lt::w(p)) * cuw;
                } else {
                    const R cu = cx * ux + cy * uy + cz * uz;
                    val = -g[p] + R(2) * R(Lt::w(p)) * (R(4.5) * cu * cu - R(1.5) * uu);
                }
            }
            store_g<Lt, ST>(dst, capc, cell, Lt::opp(p), val);
        }
    }
    if (flag & BF_NSKIP) {
#pragma unroll
        for (int p = 1; p < Q; p++) {
            const int sx = i - Lt::cx(p), sy = j - Lt::cy(p), sz = k - Lt::cz(p);
            const int rx = sx < 0 ? -1 : (sx > 3 ? 1 : 0);
            const int ry = sy < 0 ? -1 : (sy > 3 ? 1 : 0);
            const int rz = sz < 0 ? -1 : (sz > 3 ? 1 : 0);
            if (s_link[s][offset_slot(rx, ry, rz) - (Lt::D == 2 ? 9 : 0)] == kNSkip)
                store_g<Lt, ST>(dst, capc, cell, p, g[p]);
        }
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

template <int Q, int S>
__global__ __launch_bounds__(256) void k_interp(const int32_t *__restrict__ list, int n, DevMesh m,
                                                typename Store<S>::T *f0, typename Store<S>::T *f1, LevelParams lp,
                                                int all_cells) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    using T = typename ST::T;
    constexpr int MB = Lt::MB, NC = Lt::NC;
    __shared__ R s_g[Q][MB];
    __shared__ uint64_t s_gm[NC];
    if ((int)blockIdx.x >= n) return;
    const int P = list[blockIdx.x];
    const int L = m.level[P];
    const int first = m.nbrc[P];
    if (first < 0 || first > m.cap - NC || L + 1 >= m.lmax) return;  // only refined parents are listed
    const T *src = lp.par[L] ? f1 : f0;
    T *dst = lp.par[L + 1] ? f1 : f0;
    const R r = R(lp.r_cf[L]);
    const int t = threadIdx.x;
    if (t < NC) s_gm[t] = all_cells ? ~0ull : m.gmask[first + t];
    if (t < MB) {
        R g[Q];
        load_g<Lt, ST>(src, m.capc, (int64_t)P * MB + t, g);
        R drho, ux, uy, uz;
        moments_g<Lt, R>(g, drho, ux, uy, uz);
        const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int p = 0; p < Q; p++) {
            const R ge = geq<Lt, R>(p, drho, ux, uy, uz, uu);
            s_g[p][t] = ge + r * (g[p] - ge);
        }
    }
    __syncthreads();
    for (int e = t; e < NC * MB; e += blockDim.x) {
        const int c = e / MB, lf = e - c * MB;
        if (!((s_gm[c] >> lf) & 1ull)) continue;
        const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        const int I = lf & 3, J = (lf >> 2) & 3, K = lf >> 4;
        const R x = R(-0.25) + R(0.5) * R(I), y = R(-0.25) + R(0.5) * R(J), z = R(-0.25) + R(0.5) * R(K);
        const int m0 = 2 * cx + 4 * (2 * cy) + 16 * (2 * cz);
        const int64_t cell = (int64_t)(first + c) * MB + lf;
#pragma unroll
        for (int p = 0; p < Q; p++) {
            R v;
            if (Lt::D == 2) {
                v = lin2<R>(s_g[p][m0], s_g[p][m0 + 1], s_g[p][m0 + 4], s_g[p][m0 + 5], x, y);
            } else {
                R F[8];
#pragma unroll
                for (int nn = 0; nn < 8; nn++) F[nn] = s_g[p][m0 + (nn & 1) + 4 * ((nn >> 1) & 1) + 16 * (nn >> 2)];
                v = lin3<R>(F, x, y, z);
            }
            store_g<Lt, ST>(dst, m.capc, cell, p, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Fine-to-coarse averaging with rescaling (Sec. "Averaging"): parent cell
// (i,j,k) takes the mean of the 2^d rescaled cells of child octant
// (i/2, j/2, k/2) starting at fine cell (2(i mod 2), 2(j mod 2), 2(k mod 2)).
// One thread per parent cell; 64-thread workgroups (one 3-D parent, four 2-D).
template <int Q, int S>
__global__ __launch_bounds__(64) void k_average(const int32_t *__restrict__ list, int n, DevMesh m,
                                                typename Store<S>::T *f0, typename Store<S>::T *f1, LevelParams lp,
                                                int all_cells) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    using T = typename ST::T;
    constexpr int MB = Lt::MB, NC = Lt::NC, PPW = 64 / MB;
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const int idx = blockIdx.x * PPW + s;
    if (idx >= n) return;
    const int P = list[idx];
    if (!is_refined(m.status[P])) return;
    const int L = m.level[P];
    const int c0 = m.nbrc[P];
    if (c0 < 0 || c0 > m.cap - NC || L + 1 >= m.lmax) return;
    const int i = l & 3, j = (l >> 2) & 3, k = l >> 4;
    const int child = c0 + (i >> 1) + 2 * (j >> 1) + 4 * (k >> 1);
    const int fb = 2 * (i & 1) + 8 * (j & 1) + 32 * (k & 1);
    if (!all_cells && !((m.imask[child] >> fb) & 1ull)) return;
    const T *src = lp.par[L + 1] ? f1 : f0;
    T *dst = lp.par[L] ? f1 : f0;
    const R r = R(lp.r_fc[L]);
    R acc[Q];
#pragma unroll
    for (int p = 0; p < Q; p++) acc[p] = R(0);
#pragma unroll
    for (int nn = 0; nn < NC; nn++) {
        const int lf = fb + (nn & 1) + 4 * ((nn >> 1) & 1) + 16 * (nn >> 2);
        R g[Q];
        load_g<Lt, ST>(src, m.capc, (int64_t)child * MB + lf, g);
        R drho, ux, uy, uz;
        moments_g<Lt, R>(g, drho, ux, uy, uz);
        const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int p = 0; p < Q; p++) {
            const R ge = geq<Lt, R>(p, drho, ux, uy, uz, uu);
            acc[p] += ge + r * (g[p] - ge);
        }
    }
    const int64_t cell = (int64_t)P * MB + l;
#pragma unroll
    for (int p = 0; p < Q; p++) store_g<Lt, ST>(dst, m.capc, cell, p, acc[p] / R(NC));
}

// ---------------------------------------------------------------------------
// initial states
template <int Q, int S>
__global__ void k_fill_rest(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.capc) return;
#pragma unroll
    for (int p = 0; p < Q; p++) {
        store_g<Lt, ST>(f0, m.capc, e, p, typename ST::R(0));
        store_g<Lt, ST>(f1, m.capc, e, p, typename ST::R(0));
    }
}

// f = feq(rho, u) on root cells, from (rho, ux, uy, uz) in (root block, cell) order
template <int Q, int S>
__global__ void k_set_rho_u(DevMesh m, typename Store<S>::T *f, const double *__restrict__ ru, int cell0, int ncells) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    const int el = blockIdx.x * blockDim.x + threadIdx.x;
    if (el >= ncells) return;
    const int e = cell0 + el;
    const int B = e / Lt::MB;
    if (m.status[B] == ST_INACTIVE) return;
    const double rho = ru[4 * el], ux = ru[4 * el + 1], uy = ru[4 * el + 2], uz = ru[4 * el + 3];
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int p = 0; p < Q; p++) {
        const double cu = Lt::cx(p) * ux + Lt::cy(p) * uy + Lt::cz(p) * uz;
        if (ST::shift) {
            const double gv = Lt::w(p) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
            ST::st(f + p * m.capc + e, R(gv));
        } else {
            const double fv = Lt::w(p) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            ST::st(f + p * m.capc + e, R(fv));
        }
    }
}

// ---------------------------------------------------------------------------
// Vorticity criterion, FP64 (Sec. "Adaptive Mesh Refinement" of the solver):
// central differences over same-level neighbour cells, one-sided where a
// neighbour is missing, scaled to root-cell units; block maximum per leaf and
// the global maximum (atomic max on the bit pattern of a non-negative double).
template <typename Lt, typename ST>
__device__ inline void velocity_f64(const typename ST::T *__restrict__ f, int64_t capc, int64_t cell, double *u) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < Lt::Q; p++) {
        const double v = double(ST::ld(f + p * capc + cell)) + (ST::shift ? Lt::w(p) : 0.0);
        rho += v;
        j[0] += v * Lt::cx(p);
        j[1] += v * Lt::cy(p);
        j[2] += v * Lt::cz(p);
    }
    u[0] = j[0] / rho;
    u[1] = j[1] / rho;
    u[2] = j[2] / rho;
}

template <int Q, int S>
__global__ __launch_bounds__(256) void k_vorticity(const int32_t *__restrict__ list, int n, DevMesh m,
                                                   const typename Store<S>::T *__restrict__ f, double scale,
                                                   double *crit, unsigned long long *wmax_bits) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    constexpr int MB = Lt::MB, BPW = 256 / MB, NS = Lt::D == 2 ? 9 : 27;
    __shared__ int32_t s_link[BPW][NS];
    __shared__ int32_t s_id[BPW];
    const int base = blockIdx.x * BPW;
    for (int e = threadIdx.x; e < BPW * Lt::NB; e += 256) {
        const int s = e / Lt::NB, p = e - s * Lt::NB;
        const int idx = base + s;
        int32_t v = 0;
        if (idx < n) {
            const int B = list[idx];
            v = m.nbr[(int64_t)p * m.cap + B];
            if (p == 0) s_id[s] = B;
        }
        s_link[s][offset_slot(Lt::cx(p), Lt::cy(p), Lt::cz(p)) - (Lt::D == 2 ? 9 : 0)] = v;
    }
    __syncthreads();
    const int s = threadIdx.x / MB, l = threadIdx.x % MB;
    const bool valid = base + s < n;
    const int B = valid ? s_id[s] : 0;
    const bool leaf = valid && m.status[B] == ST_UNREF;
    double w = 0.0;
    if (leaf) {
        const int ci[3] = {l & 3, (l >> 2) & 3, l >> 4};
        double u0[3];
        velocity_f64<Lt, ST>(f, m.capc, (int64_t)B * MB + l, u0);
        double gr[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) gr[a][b] = 0.0;
        for (int a = 0; a < Lt::D; a++) {
            double up[3], um[3];
            bool hp = false, hm = false;
            for (int sg = 0; sg < 2; sg++) {
                int t[3] = {ci[0], ci[1], ci[2]};
                t[a] += sg == 0 ? 1 : -1;
                const int rx = t[0] < 0 ? -1 : (t[0] > 3 ? 1 : 0);
                const int ry = t[1] < 0 ? -1 : (t[1] > 3 ? 1 : 0);
                const int rz = t[2] < 0 ? -1 : (t[2] > 3 ? 1 : 0);
                const int32_t code = s_link[s][offset_slot(rx, ry, rz) - (Lt::D == 2 ? 9 : 0)];
                if (code < 0 || code >= m.cap) continue;
                const int lt = (t[0] & 3) + 4 * (t[1] & 3) + 16 * (t[2] & 3);
                if (sg == 0) { velocity_f64<Lt, ST>(f, m.capc, (int64_t)code * MB + lt, up); hp = true; }
                else { velocity_f64<Lt, ST>(f, m.capc, (int64_t)code * MB + lt, um); hm = true; }
            }
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
        atomicMax(wmax_bits, (unsigned long long)__double_as_longlong(w));
    }
}

// ---------------------------------------------------------------------------
// Gathers / scatters of unshifted FP64 data through the staging buffer.
template <int Q, int S>
__global__ void k_block_f(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1, LevelParams lp, int set,
                          int b0, int b1, double *stage) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    using R = typename ST::R;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncell = (int64_t)(b1 - b0) * Lt::MB;
    if (e >= ncell) return;
    const int B = b0 + (int)(e / Lt::MB), l = (int)(e % Lt::MB);
    const int L = m.level[B];
    typename ST::T *f = lp.par[L] ? f1 : f0;
    const int64_t cell = (int64_t)B * Lt::MB + l;
    double *row = stage + e * Q;
#pragma unroll
    for (int p = 0; p < Q; p++) {
        if (set) {
            const double v = row[p] - (ST::shift ? Lt::w(p) : 0.0);
            ST::st(f + p * m.capc + cell, R(v));
        } else {
            row[p] = double(ST::ld(f + p * m.capc + cell)) + (ST::shift ? Lt::w(p) : 0.0);
        }
    }
}

// output cells: leaf, non-ghost cells in (block ID, cell) order; kind: 1 cells,
// 2 rho/u, 3 f
template <int Q, int S>
__global__ void k_out_gather(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1, LevelParams lp,
                             int kind, int b0, int b1, const int32_t *__restrict__ off, int32_t off0, void *stage) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    constexpr int MB = Lt::MB;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)(b1 - b0) * MB) return;
    const int B = b0 + (int)(e / MB), l = (int)(e % MB);
    if (m.status[B] != ST_UNREF) return;
    const uint64_t full = MB == 64 ? ~0ull : ((1ull << MB) - 1);
    const uint64_t outm = ~m.gmask[B] & full;
    if (!((outm >> l) & 1ull)) return;
    const int64_t pos = (int64_t)off[B] - off0 + __popcll(outm & ((1ull << l) - 1));
    const int L = m.level[B];
    const typename ST::T *f = lp.par[L] ? f1 : f0;
    const int64_t cell = (int64_t)B * MB + l;
    if (kind == AMR_FIELD_CELLS) {
        int32_t *o = (int32_t *)stage + 2 * pos;
        o[0] = B;
        o[1] = l;
    } else if (kind == AMR_FIELD_RHO_U) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < Q; p++) {
            const double v = double(ST::ld(f + p * m.capc + cell)) + (ST::shift ? Lt::w(p) : 0.0);
            rho += v;
            j[0] += v * Lt::cx(p);
            j[1] += v * Lt::cy(p);
            j[2] += v * Lt::cz(p);
        }
        double *o = (double *)stage + 4 * pos;
        o[0] = rho;
        o[1] = j[0] / rho;
        o[2] = j[1] / rho;
        o[3] = j[2] / rho;
    } else {
        double *o = (double *)stage + Q * pos;
#pragma unroll
        for (int p = 0; p < Q; p++) o[p] = double(ST::ld(f + p * m.capc + cell)) + (ST::shift ? Lt::w(p) : 0.0);
    }
}

// FP64 mass and momentum of the output cells: fixed-order per-block partials,
// then a single-workgroup fixed-order sum.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_mass_blocks(DevMesh m, typename Store<S>::T *f0, typename Store<S>::T *f1,
                                                     LevelParams lp, double *part4) {
    using Lt = Lat<Q>;
    using ST = Store<S>;
    constexpr int MB = Lt::MB;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int B = (int)(e / MB), l = (int)(e % MB);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const bool inb = B < m.cap;
    if (inb && m.status[B] == ST_UNREF && !((m.gmask[B] >> l) & 1ull)) {
        const int L = m.level[B];
        const typename ST::T *f = lp.par[L] ? f1 : f0;
        const int64_t cell = (int64_t)B * MB + l;
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < Q; p++) {
            const double x = double(ST::ld(f + p * m.capc + cell)) + (ST::shift ? Lt::w(p) : 0.0);
            rho += x;
            j[0] += x * Lt::cx(p);
            j[1] += x * Lt::cy(p);
            j[2] += x * Lt::cz(p);
        }
        const double vol = 1.0 / double(1 << (Lt::D * L));
        v[0] = vol * rho;
        for (int a = 0; a < 3; a++) v[1 + a] = vol * rho * (j[a] / rho);
    }
#pragma unroll
    for (int off = MB / 2; off > 0; off >>= 1)
        for (int a = 0; a < 4; a++) v[a] += __shfl_xor(v[a], off, 64);
    if (inb && l == 0)
        for (int a = 0; a < 4; a++) part4[(int64_t)B * 4 + a] = v[a];
}

__global__ __launch_bounds__(256) void k_mass_final(const double *part4, int cap, double *out) {
    __shared__ double s[4][256];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int B = threadIdx.x; B < cap; B += 256)
        for (int a = 0; a < 4; a++) v[a] += part4[(int64_t)B * 4 + a];
    for (int a = 0; a < 4; a++) s[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 4; a++) s[a][threadIdx.x] += s[a][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

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

void launch_collide_stream(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp, const BCParams &bc) {
    if (n <= 0) return;
    const int bpw = 256 / c.mb;
    const int grid = (n + bpw - 1) / bpw;
    const int sp = lp.par[L];
    AMR_DISPATCH(c.q, c.storage,
                 (k_collide_stream<Qc, Sc><<<grid, 256, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[sp]),
                                                                       TPTR(Sc, c.f[1 - sp]), lp.omega[L], bc)));
}

void launch_interp(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells) {
    if (n <= 0) return;
    const int threads = c.dim == 2 ? 64 : 256;
    AMR_DISPATCH(c.q, c.storage,
                 (k_interp<Qc, Sc><<<n, threads, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]),
                                                                 lp, all_cells)));
}

void launch_average(const Ctx &c, const int32_t *list, int n, const LevelParams &lp, int all_cells) {
    if (n <= 0) return;
    const int ppw = 64 / c.mb;
    const int grid = (n + ppw - 1) / ppw;
    AMR_DISPATCH(c.q, c.storage,
                 (k_average<Qc, Sc><<<grid, 64, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]),
                                                               lp, all_cells)));
}

void launch_fill_rest(const Ctx &c) {
    const int grid = (int)((c.m.capc + 255) / 256);
    AMR_DISPATCH(c.q, c.storage,
                 (k_fill_rest<Qc, Sc><<<grid, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]))));
}

void launch_set_rho_u_root(const Ctx &c, const double *ru, int cell0, int ncells) {
    if (ncells <= 0) return;
    const int grid = (ncells + 255) / 256;
    AMR_DISPATCH(c.q, c.storage,
                 (k_set_rho_u<Qc, Sc><<<grid, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), ru, cell0, ncells)));
}

void launch_vorticity(const Ctx &c, const int32_t *list, int n, int L, const LevelParams &lp) {
    if (n <= 0) return;
    const int bpw = 256 / c.mb;
    const int grid = (n + bpw - 1) / bpw;
    const double scale = double(1 << L);
    AMR_DISPATCH(c.q, c.storage,
                 (k_vorticity<Qc, Sc><<<grid, 256, 0, c.stream>>>(list, n, c.m, TPTR(Sc, c.f[lp.par[L]]), scale,
                                                                  c.crit, &c.ctr->wmax_bits)));
}

void launch_block_f(const Ctx &c, int set, int b0, int b1, double *stage, const LevelParams &lp) {
    const int64_t n = (int64_t)(b1 - b0) * c.mb;
    if (n <= 0) return;
    const int grid = (int)((n + 255) / 256);
    AMR_DISPATCH(c.q, c.storage,
                 (k_block_f<Qc, Sc><<<grid, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), lp, set, b0,
                                                                b1, stage)));
}

void launch_out_gather(const Ctx &c, int kind, int b0, int b1, int32_t off0, void *stage, const LevelParams &lp) {
    const int64_t n = (int64_t)(b1 - b0) * c.mb;
    if (n <= 0) return;
    const int grid = (int)((n + 255) / 256);
    AMR_DISPATCH(c.q, c.storage,
                 (k_out_gather<Qc, Sc><<<grid, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), lp, kind,
                                                                   b0, b1, c.off, off0, stage)));
}

void launch_mass(const Ctx &c, const LevelParams &lp) {
    const int64_t n = (int64_t)c.m.cap * c.mb;
    const int grid = (int)((n + 255) / 256);
    AMR_DISPATCH(c.q, c.storage,
                 (k_mass_blocks<Qc, Sc><<<grid, 256, 0, c.stream>>>(c.m, TPTR(Sc, c.f[0]), TPTR(Sc, c.f[1]), lp,
                                                                    c.part4)));
    k_mass_final<<<1, 256, 0, c.stream>>>(c.part4, c.m.cap, c.ctr->mass);
}

}  // namespace amr
