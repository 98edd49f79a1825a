// mesh_kernels.hip -- on-device mesh management of the AMR-LBM library:
// root-grid construction, refinement criteria to tags, the refine/coarsen
// routine (Sec. "Refinement and Coarsening": gap assignment, 2:1 reversion,
// child construction, ID-set updates, connectivity rebuild) and the ordered
// scans it is built on.  Order-dependent results come from ballot/popcount
// scans, never from atomics, so tables are deterministic.
#include "kernels.h"

namespace amr {

namespace {

constexpr int kScanTPB = 256;
constexpr int kScanPer = 4;
constexpr int kScanItems = kScanTPB * kScanPer;

inline int grid_for(int64_t n, int tpb = 256) { return (int)((n + tpb - 1) / tpb); }

// ---------------------------------------------------------------------------
// Binned exclusive scan: for every element with bin b >= 0, rank = number of
// earlier elements (in index order) with the same bin.  Three passes: per-
// workgroup counts (wave ballots), a single-workgroup scan of the counts, then
// per-element ranks (ballot + popcount of the lanes below).
__global__ __launch_bounds__(256) void k_scan_count(const int8_t *__restrict__ bins, int64_t n, int K,
                                                    int32_t *__restrict__ part) {
    __shared__ int32_t s_cnt[kMaxLevels];
    if ((int)threadIdx.x < K) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int r = 0; r < kScanPer; r++) {
        const int64_t idx = (int64_t)blockIdx.x * kScanItems + r * kScanTPB + threadIdx.x;
        const int b = idx < n ? bins[idx] : -1;
        for (int k = 0; k < K; k++) {
            const uint64_t msk = __ballot(b == k);
            if (lane == 0 && msk) atomicAdd(&s_cnt[k], (int)__popcll(msk));
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < K) part[(int64_t)blockIdx.x * K + threadIdx.x] = s_cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_scan_part(int32_t *__restrict__ part, int nwg, int K, DevCounters *ctr) {
    __shared__ int32_t s[256];
    __shared__ int32_t s_tot[kMaxLevels];
    const int t = threadIdx.x;
    const int chunk = (nwg + 255) / 256;
    for (int k = 0; k < K; k++) {
        const int lo = min(nwg, t * chunk), hi = min(nwg, lo + chunk);
        int sum = 0;
        for (int i = lo; i < hi; i++) sum += part[(int64_t)i * K + k];
        s[t] = sum;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int v = t >= off ? s[t - off] : 0;
            __syncthreads();
            s[t] += v;
            __syncthreads();
        }
        int run = s[t] - sum;
        for (int i = lo; i < hi; i++) {
            const int v = part[(int64_t)i * K + k];
            part[(int64_t)i * K + k] = run;
            run += v;
        }
        if (t == 255) s_tot[k] = s[255];
        __syncthreads();
    }
    if (t == 0) {
        int acc = 0;
        for (int k = 0; k < kMaxLevels; k++) {
            const int v = k < K ? s_tot[k] : 0;
            ctr->totals[k] = v;
            ctr->bases[k] = acc;
            acc += v;
        }
    }
}

__global__ __launch_bounds__(256) void k_scan_rank(const int8_t *__restrict__ bins, int64_t n, int K,
                                                   const int32_t *__restrict__ part, int32_t *__restrict__ rank) {
    __shared__ int32_t s_run[kMaxLevels];
    __shared__ int32_t s_wt[4][kMaxLevels];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((int)threadIdx.x < K) s_run[threadIdx.x] = part[(int64_t)blockIdx.x * K + threadIdx.x];
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    for (int r = 0; r < kScanPer; r++) {
        const int64_t idx = (int64_t)blockIdx.x * kScanItems + r * kScanTPB + threadIdx.x;
        const int b = idx < n ? bins[idx] : -1;
        int my = 0;
        for (int k = 0; k < K; k++) {
            const uint64_t msk = __ballot(b == k);
            if (b == k) my = (int)__popcll(msk & below);
            if (lane == 0) s_wt[wave][k] = (int)__popcll(msk);
        }
        __syncthreads();
        if (b >= 0) {
            int pre = s_run[b];
            for (int w = 0; w < wave; w++) pre += s_wt[w][b];
            rank[idx] = pre + my;
        }
        __syncthreads();
        if ((int)threadIdx.x < K) {
            const int k = threadIdx.x;
            s_run[k] += s_wt[0][k] + s_wt[1][k] + s_wt[2][k] + s_wt[3][k];
        }
        __syncthreads();
    }
}

void run_scan(const Ctx &c, const int8_t *bins, int64_t n, int K) {
    const int nwg = (int)((n + kScanItems - 1) / kScanItems);
    k_scan_count<<<nwg, kScanTPB, 0, c.stream>>>(bins, n, K, c.scan_part);
    k_scan_part<<<1, 256, 0, c.stream>>>(c.scan_part, nwg, K, c.ctr);
    k_scan_rank<<<nwg, kScanTPB, 0, c.stream>>>(bins, n, K, c.scan_part, c.rank);
}

// exclusive prefix sum of non-negative int32 values (output-cell offsets)
__global__ __launch_bounds__(256) void k_wscan_count(const int32_t *__restrict__ v, int64_t n,
                                                     int32_t *__restrict__ part) {
    __shared__ int32_t s[256];
    int sum = 0;
    for (int e = 0; e < kScanPer; e++) {
        const int64_t idx = (int64_t)blockIdx.x * kScanItems + threadIdx.x * kScanPer + e;
        if (idx < n) sum += v[idx];
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_wscan_apply(const int32_t *__restrict__ v, int64_t n,
                                                     const int32_t *__restrict__ part, int32_t *__restrict__ out) {
    __shared__ int32_t s[256];
    const int t = threadIdx.x;
    int loc[kScanPer];
    int sum = 0;
    for (int e = 0; e < kScanPer; e++) {
        const int64_t idx = (int64_t)blockIdx.x * kScanItems + t * kScanPer + e;
        loc[e] = idx < n ? v[idx] : 0;
        sum += loc[e];
    }
    s[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int x = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    int run = part[blockIdx.x] + s[t] - sum;
    for (int e = 0; e < kScanPer; e++) {
        const int64_t idx = (int64_t)blockIdx.x * kScanItems + t * kScanPer + e;
        if (idx < n) out[idx] = run;
        run += loc[e];
    }
}

// ---------------------------------------------------------------------------
struct RootParams {
    int dim, nroot, lmax;
    int root[3];
    int periodic[3];
    int prio[6];
};

template <typename Dd>
__device__ int32_t root_link(const RootParams &rp, const uint8_t *solid, int bi, int bj, int bk, int p) {
    int r[3] = {bi + Dd::cx(p), bj + Dd::cy(p), bk + Dd::cz(p)};
    bool crossed[6] = {false, false, false, false, false, false};
    bool out = false;
    for (int a = 0; a < rp.dim; a++) {
        if (r[a] < 0) {
            if (rp.periodic[a]) r[a] += rp.root[a];
            else { crossed[2 * a] = true; out = true; }
        } else if (r[a] >= rp.root[a]) {
            if (rp.periodic[a]) r[a] -= rp.root[a];
            else { crossed[2 * a + 1] = true; out = true; }
        }
    }
    if (out) {
        int best = -1;
        for (int fc = 0; fc < 6; fc++)
            if (crossed[fc] && (best < 0 || rp.prio[fc] > rp.prio[best])) best = fc;
        return -3 - best;
    }
    const int id = r[0] + rp.root[0] * (r[1] + rp.root[1] * r[2]);
    if (solid && solid[id]) return kSolid;
    return id;
}

template <typename Dd>
__global__ void k_init_blocks(DevMesh m, RootParams rp, const uint8_t *solid, int8_t *bins) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    m.tag[B] = 0;
    m.ldes[B] = 0;
    m.viol[B] = 0;
    m.bflag[B] = 0;
    m.gmask[B] = 0;
    m.imask[B] = 0;
    m.level[B] = 0;
    m.parent[B] = -1;
    m.fresh[B] = 0;
    if (B >= rp.nroot) {
        m.status[B] = ST_INACTIVE;
        for (int a = 0; a < 3; a++) m.X[(int64_t)a * m.cap + B] = 0;
        bins[B] = -1;
        return;
    }
    const int bi = B % rp.root[0], bj = (B / rp.root[0]) % rp.root[1], bk = B / (rp.root[0] * rp.root[1]);
    const int W0 = 4 << (rp.lmax - 1);
    m.X[B] = bi * W0;
    m.X[(int64_t)m.cap + B] = bj * W0;
    m.X[(int64_t)2 * m.cap + B] = bk * W0;
    const bool sol = solid && solid[B];
    m.status[B] = sol ? ST_INACTIVE : ST_UNREF;
    bins[B] = sol ? -1 : 0;
    for (int p = 0; p < Dd::NB; p++) {
        const int32_t n = sol ? 0 : root_link<Dd>(rp, solid, bi, bj, bk, p);
        m.nbr[(int64_t)p * m.cap + B] = n;
        m.nbrc[(int64_t)p * m.cap + B] = n >= 0 ? kNone : n;
    }
}

__global__ void k_init_gap(int32_t *gap, int cap, int nroot) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < cap - nroot) gap[g] = cap - 1 - g;
}

__global__ void k_init_ids(const int8_t *bins, const int32_t *rank, int cap, int32_t *ids, DevCounters *ctr, int nroot) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B < cap && bins[B] == 0) ids[rank[B]] = B;
    if (B == 0) {
        ctr->nids[0] = ctr->totals[0];
        for (int L = 1; L < kMaxLevels; L++) ctr->nids[L] = 0;
        for (int L = 0; L < kMaxLevels; L++) ctr->niface[L] = ctr->nref[L] = ctr->nsweep[L] = 0;
        ctr->gtop = cap - nroot;
        ctr->n_ref = ctr->n_coa = ctr->n_rev = ctr->nfreed = 0;
        ctr->wmax_bits = 0;
    }
}

// ---------------------------------------------------------------------------
// Cell classes (Sec. "Grid Communication"): a cell of a block on level > 0 is a
// ghost if its Chebyshev distance (adjacent = 1) to some N_SKIP neighbour
// region is at most 2, an interface cell at 3 or 4.  Also the per-block flags
// used by the solver kernels.
template <typename Dd>
__global__ void k_block_masks(DevMesh m) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    if (m.status[B] == ST_INACTIVE) {
        m.bflag[B] = 0;
        m.gmask[B] = 0;
        m.imask[B] = 0;
        return;
    }
    uint8_t fl = 0;
    uint32_t skipset = 0;
    for (int p = 1; p < Dd::NB; p++) {
        const int32_t n = m.nbr[(int64_t)p * m.cap + B];
        if (n == kNSkip) { fl |= BF_NSKIP; skipset |= 1u << p; }
        else if (n < 0) fl |= n == kSolid ? (BF_BOUNDARY | BF_SOLID) : BF_BOUNDARY;
    }
    uint64_t gm = 0, im = 0;
    if (m.level[B] > 0 && skipset) {
        for (int l = 0; l < Dd::MB; l++) {
            const int ci[3] = {l & 3, (l >> 2) & 3, l >> 4};
            int d = 1 << 20;
            for (int p = 1; p < Dd::NB; p++) {
                if (!((skipset >> p) & 1u)) continue;
                const int v[3] = {Dd::cx(p), Dd::cy(p), Dd::cz(p)};
                int dist = 0;
                for (int a = 0; a < Dd::D; a++) {
                    const int da = v[a] == 1 ? 4 - ci[a] : (v[a] == -1 ? ci[a] + 1 : 0);
                    dist = da > dist ? da : dist;
                }
                d = dist < d ? dist : d;
            }
            if (d <= 2) gm |= 1ull << l;
            else if (d <= 4) im |= 1ull << l;
        }
    }
    m.bflag[B] = fl;
    m.gmask[B] = gm;
    m.imask[B] = im;
}

template <typename Dd>
__global__ void k_parent_mask(DevMesh m) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap || !is_refined(m.status[B])) return;
    const int c0 = m.nbrc[B];
    bool any = false;
    for (int c = 0; c < Dd::NC; c++) any = any || (m.bflag[c0 + c] & BF_NSKIP);
    if (any) m.bflag[B] = m.bflag[B] | BF_PARENT_MASK;
}

// ---------------------------------------------------------------------------
// Tagging.
__global__ void k_crit_reset(double *crit, int cap, DevCounters *ctr) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B < cap) crit[B] = -1.0;
    if (B == 0) ctr->wmax_bits = 0ull;
}

// leaves: desired level L_max-1 above theta * max, else 0; refine when above the own level
// Desired level of each leaf (Sec. "Adaptive Mesh Refinement" of the
// solver).  Relative threshold: the finest level where the block maximum
// exceeds theta times the maximum over all leaves, else level 0.  Ladder
// (Alg. 3): with eps = min(1, log2 |w|), the level L_max-1 is lowered to
// (L_max-1) - p for every p with eps < n_start - p n_inc; evaluated as
// |w| < 2^(n_start - p n_inc) against thresholds made on the host (a
// threshold above 2 always holds, as eps <= 1).
__global__ void k_tag_vort_leaf(DevMesh m, const double *crit, const DevCounters *ctr, double theta, int ladder,
                                LadderParams lad) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    if (m.status[B] != ST_UNREF) {
        m.tag[B] = 0;
        return;
    }
    int ldes;
    if (ladder) {
        const double w = crit[B] * lad.scale;
        ldes = m.lmax - 1;
        for (int p = 1; p <= m.lmax - 1; p++)
            if (w < lad.thr[p]) ldes = (m.lmax - 1) - p;
    } else {
        const double wmax = __longlong_as_double((long long)ctr->wmax_bits);
        ldes = crit[B] > theta * wmax ? m.lmax - 1 : 0;
    }
    m.ldes[B] = (int8_t)ldes;
    m.tag[B] = ldes > m.level[B] ? 1 : 0;
}

// refined blocks whose children are all leaves: coarsen when no child wants to
// be finer than the parent's level
template <typename Dd>
__global__ void k_tag_vort_parent(DevMesh m) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap || m.status[B] != ST_REF) return;
    const int c0 = m.nbrc[B];
    int mx = 0;
    for (int c = 0; c < Dd::NC; c++) mx = m.ldes[c0 + c] > mx ? m.ldes[c0 + c] : mx;
    if (mx <= m.level[B]) m.tag[B] = -1;
}

struct DistParams {
    int dim, lmax, n_solid;
    int dom[3];
    int face_kind[6];
    double dspec_f;
    int freeze;
};

__global__ void k_tag_distance(DevMesh m, const int32_t *solid_list, DistParams dp) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    if (m.status[B] != ST_UNREF) {
        m.tag[B] = 0;
        return;
    }
    const int L = m.level[B];
    const int W = 4 << (dp.lmax - 1 - L), W0 = 4 << (dp.lmax - 1);
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = m.X[(int64_t)a * m.cap + B];
        hi[a] = lo[a] + (a < dp.dim ? W : 0);
    }
    double best = -1.0;
    for (int s = 0; s < dp.n_solid; s++) {
        const int S = solid_list[s];
        long long d2 = 0;
        for (int a = 0; a < dp.dim; a++) {
            const int slo = m.X[(int64_t)a * m.cap + S], shi = slo + W0;
            long long g = 0;
            if (hi[a] < slo) g = slo - hi[a];
            else if (shi < lo[a]) g = lo[a] - shi;
            d2 += g * g;
        }
        if (best < 0 || (double)d2 < best) best = (double)d2;
    }
    for (int fc = 0; fc < 2 * dp.dim; fc++) {
        if (dp.face_kind[fc] != AMR_FACE_OUTFLOW) continue;
        const int a = fc / 2;
        const long long g = (fc & 1) ? (long long)(dp.dom[a] - hi[a]) : (long long)lo[a];
        const double d2 = (double)(g * g);
        if (best < 0 || d2 < best) best = d2;
    }
    const double thr = dp.dspec_f / (double)(1 << L);
    m.tag[B] = (best >= 0.0 && best < thr * thr) ? (dp.freeze ? 2 : 1) : 0;
}

// eligibility and the 2:1 refine-cancel; counts of refine / coarsen marks
__global__ void k_effective_tags(DevMesh m, DevCounters *ctr) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    int out = 0;
    if (B < m.cap) {
        const int t = m.tag[B], st = m.status[B];
        if (st != ST_INACTIVE) {
            if (t == 1 || t == 2) {
                if (st == ST_UNREF && m.level[B] < m.lmax - 1 && !(m.bflag[B] & BF_NSKIP)) out = t;
            } else if (t == -1) {
                if (st == ST_REF) out = -1;
            }
        }
        m.tag[B] = (int8_t)out;
    }
    const uint64_t r = __ballot(out > 0), c = __ballot(out < 0);
    if ((threadIdx.x & 63) == 0) {
        if (r) atomicAdd(&ctr->n_ref, (int)__popcll(r));
        if (c) atomicAdd(&ctr->n_coa, (int)__popcll(c));
    }
}

// ---------------------------------------------------------------------------
// Adaptation.
__global__ void k_bins_refine(const DevMesh m, int8_t *bins, int by_level) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    const int t = m.tag[B];
    bins[B] = (t == 1 || t == 2) ? (int8_t)(by_level ? m.level[B] : 0) : (int8_t)-1;
}

__global__ void k_bins_coarsen(const DevMesh m, int8_t *bins) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    bins[B] = m.tag[B] == -1 ? m.level[B] : (int8_t)-1;
}

// S2: the r-th refine-marked block (ascending ID) takes the N_c gaps below
// the top of the gap stack; its first child is gap[top - 1 - N_c r]
__global__ void k_assign_first(DevMesh m, const int32_t *rank, const int32_t *gap, const DevCounters *ctr,
                               int32_t *first, int32_t *rlist, int nc) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    const int t = m.tag[B];
    if (t == 1 || t == 2) {
        const int r = rank[B];
        first[B] = gap[ctr->gtop - 1 - nc * r];
        rlist[r] = B;
    } else {
        first[B] = -1;
    }
}

__global__ void k_gtop_add(DevCounters *ctr, int delta_const, int use_freed) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr->gtop += use_freed ? ctr->nfreed : delta_const;
}

// S3: a leaf is violating if any provisional neighbour-child (this call's new
// children included, and its own at p = 0) is a valid ID
template <typename Dd>
__global__ void k_violating(DevMesh m, const int32_t *first) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    int8_t v = 0;
    if (m.status[B] == ST_UNREF) {
        for (int p = 0; p < Dd::NB && !v; p++) {
            int32_t pc;
            if (p == 0) {
                pc = first[B] >= 0 ? first[B] : m.nbrc[B];
            } else {
                const int32_t n = m.nbr[(int64_t)p * m.cap + B];
                pc = (n >= 0 && first[n] >= 0) ? first[n] : m.nbrc[(int64_t)p * m.cap + B];
            }
            if (pc >= 0) v = 1;
        }
    }
    m.viol[B] = v;
}

template <typename Dd>
__global__ void k_revert(DevMesh m, DevCounters *ctr) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    bool rev = false;
    if (B < m.cap && m.tag[B] == -1) {
        const int c0 = m.nbrc[B];
        for (int c = 0; c < Dd::NC && c0 >= 0; c++) rev = rev || m.viol[c0 + c];
        if (rev) m.tag[B] = 0;
    }
    const uint64_t msk = __ballot(rev);
    if ((threadIdx.x & 63) == 0 && msk) atomicAdd(&ctr->n_rev, (int)__popcll(msk));
}

// S4: new children get level + 1, status NEW and their origin; the parent's
// neighbour-child p = 0 becomes its first child
template <typename Dd>
__global__ void k_build_children(DevMesh m, const int32_t *rlist, const int32_t *first, int n_ref) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_ref * Dd::NC) return;
    const int r = e / Dd::NC, c = e - r * Dd::NC;
    const int P = rlist[r];
    const int ch = first[P] + c;
    const int L = m.level[P] + 1;
    const int W = 4 << (m.lmax - 1 - L);
    m.level[ch] = (int8_t)L;
    m.status[ch] = ST_NEW;
    m.tag[ch] = 0;
    const int cv[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    for (int a = 0; a < 3; a++) m.X[(int64_t)a * m.cap + ch] = m.X[(int64_t)a * m.cap + P] + cv[a] * W;
    m.nbrc[ch] = kNone;
    m.parent[ch] = P;
    m.fresh[ch] = 1;
    if (c == 0) m.nbrc[P] = first[P];
}

// S5: freed children in (parent level, parent ID, child) order F; the gap
// stack receives reverse(F) on top
template <typename Dd>
__global__ void k_coarsen(DevMesh m, const int32_t *rank, int32_t *gap, DevCounters *ctr) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap || m.tag[B] != -1) return;
    const int lm = m.lmax - 1;
    const int nF = Dd::NC * (ctr->bases[lm] + ctr->totals[lm]);
    const int pos = ctr->bases[m.level[B]] + rank[B];
    const int c0 = m.nbrc[B];
    for (int c = 0; c < Dd::NC; c++) {
        const int k = pos * Dd::NC + c;
        gap[ctr->gtop + nF - 1 - k] = c0 + c;
        m.status[c0 + c] = ST_REMOVE;
    }
    m.nbrc[B] = kNone;
    if (pos == 0) {
        ctr->nfreed = nF;
        ctr->n_coa = nF / Dd::NC;
    }
}

__global__ void k_zero_freed(DevCounters *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr->nfreed = 0;
        ctr->n_coa = 0;
    }
}

// virtual concatenation of the per-level ID lists: element e = L*cap + i
__global__ void k_bins_keep(const DevMesh m, const int32_t *ids, const DevCounters *ctr, int8_t *bins, int mode) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)m.lmax * m.cap;
    if (e >= tot) return;
    const int L = (int)(e / m.cap), i = (int)(e - (int64_t)L * m.cap);
    int8_t b = -1;
    if (i < ctr->nids[L]) {
        const int B = ids[e];
        if (mode == 0) b = m.status[B] != ST_REMOVE ? (int8_t)L : (int8_t)-1;
        else if (mode == 1) b = (m.bflag[B] & BF_PARENT_MASK) ? (int8_t)L : (int8_t)-1;
        else if (mode == 2) b = is_refined(m.status[B]) ? (int8_t)L : (int8_t)-1;
        else b = (is_refined(m.status[B]) && !(m.bflag[B] & BF_PARENT_MASK)) ? (int8_t)-1 : (int8_t)L;
    }
    bins[e] = b;
}

__global__ void k_compact(const int8_t *bins, const int32_t *rank, const int32_t *src, int32_t *dst, int cap,
                          int64_t tot) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int b = bins[e];
    if (b >= 0) dst[(int64_t)b * cap + rank[e]] = src[e];
}

// copy back the compacted lists; the new sizes are the scan totals
// which: 0 = interface parents (niface), 1 = ID sets (nids), 2 = refined blocks (nref),
// 3 = sweep lists (nsweep)
__global__ void k_copy_lists(const int32_t *src, int32_t *dst, int cap, int lmax, DevCounters *ctr, int which) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)lmax * cap;
    if (e < tot) {
        const int L = (int)(e / cap), i = (int)(e - (int64_t)L * cap);
        if (i < ctr->totals[L]) dst[e] = src[e];
    }
    if (e == 0) {
        for (int L = 0; L < lmax; L++) {
            if (which == 1) ctr->nids[L] = ctr->totals[L];
            else if (which == 2) ctr->nref[L] = ctr->totals[L];
            else if (which == 3) ctr->nsweep[L] = ctr->totals[L];
            else ctr->niface[L] = ctr->totals[L];
        }
    }
}

// S6: append new children to id_set_{L+1} in (parent ID, child) order
template <typename Dd>
__global__ void k_append(DevMesh m, const int32_t *rank, const int32_t *first, int32_t *ids, const DevCounters *ctr) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    const int t = m.tag[B];
    if (t != 1 && t != 2) return;
    const int L = m.level[B];
    const int base = ctr->nids[L + 1] + Dd::NC * rank[B];
    for (int c = 0; c < Dd::NC; c++) ids[(int64_t)(L + 1) * m.cap + base + c] = first[B] + c;
}

template <typename Dd>
__global__ void k_nids_after_append(DevCounters *ctr, int lmax) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int L = lmax - 2; L >= 0; L--) ctr->nids[L + 1] += Dd::NC * ctr->totals[L];
}

// S7: finalise statuses, then branch / leaf
__global__ void k_finalize_status(DevMesh m) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    const int t = m.tag[B];
    int st = m.status[B];
    if (t == 1) st = ST_REF;
    else if (t == 2) st = ST_REF_PERM;
    else if (t == -1) st = ST_UNREF;
    if (st == ST_NEW) st = ST_UNREF;
    else if (st == ST_REMOVE) st = ST_INACTIVE;
    m.status[B] = (int8_t)st;
    m.tag[B] = 0;
}

template <typename Dd>
__global__ void k_branch_leaf(DevMesh m) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    const int st = m.status[B];
    if (st != ST_REF && st != ST_REF_CHILD) return;
    const int c0 = m.nbrc[B];
    bool any = false;
    for (int c = 0; c < Dd::NC; c++) any = any || is_refined(m.status[c0 + c]);
    m.status[B] = any ? ST_REF_CHILD : ST_REF;
}

// S8: neighbour-children of level L from its links ...
template <typename Dd>
__global__ void k_nbrc_level(DevMesh m, const int32_t *ids, const DevCounters *ctr, int L) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ctr->nids[L]) return;
    const int B = ids[(int64_t)L * m.cap + i];
    for (int p = 1; p < Dd::NB; p++) {
        const int32_t n = m.nbr[(int64_t)p * m.cap + B];
        m.nbrc[(int64_t)p * m.cap + B] = n >= 0 ? m.nbrc[n] : n;
    }
}

// ... and links of the children of level L from their parent's
// neighbour-children (Alg. 2 in closed form): for child c and direction p,
// t = c + p in {-1..2}^d, parent region q = floor(t/2), child index t mod 2
template <typename Dd>
__global__ void k_child_links(DevMesh m, const int32_t *ids, const DevCounters *ctr, int L) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = e / Dd::NC, c = e - i * Dd::NC;
    if (i >= ctr->nids[L]) return;
    const int P = ids[(int64_t)L * m.cap + i];
    if (!is_refined(m.status[P])) return;
    const int ch = m.nbrc[P] + c;
    const int cv[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    int32_t pn[27];
    for (int p = 0; p < Dd::NB; p++) pn[p] = m.nbrc[(int64_t)p * m.cap + P];
    for (int p = 0; p < Dd::NB; p++) {
        const int v[3] = {Dd::cx(p), Dd::cy(p), Dd::cz(p)};
        int qv[3] = {0, 0, 0}, cc[3] = {0, 0, 0};
        for (int a = 0; a < Dd::D; a++) {
            const int t = cv[a] + v[a];
            qv[a] = t < 0 ? -1 : t / 2;
            cc[a] = t - 2 * qv[a];
        }
        // direction index of the parent region
        int qd = 0;
        for (int r = 0; r < Dd::NB; r++)
            if (Dd::cx(r) == qv[0] && Dd::cy(r) == qv[1] && Dd::cz(r) == qv[2]) qd = r;
        const int32_t X = pn[qd];
        int32_t link;
        if (X >= 0) link = X + cc[0] + 2 * cc[1] + 4 * cc[2];
        else if (X == kNone || X == kNSkip) link = kNSkip;
        else link = X;
        m.nbr[(int64_t)p * m.cap + ch] = link;
    }
}

__global__ void k_out_count(DevMesh m, int32_t *cnt, int mb) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    const uint64_t full = mb == 64 ? ~0ull : ((1ull << mb) - 1);
    cnt[B] = m.status[B] == ST_UNREF ? (int)__popcll(~m.gmask[B] & full) : 0;
}

__global__ void k_out_total(const int32_t *cnt, const int32_t *off, int cap, DevCounters *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr->n_out = cap > 0 ? off[cap - 1] + cnt[cap - 1] : 0;
}

RootParams root_params(const Ctx &c) {
    RootParams rp;
    rp.dim = c.dim;
    rp.nroot = c.nroot;
    rp.lmax = c.m.lmax;
    for (int a = 0; a < 3; a++) {
        rp.root[a] = c.root[a];
        rp.periodic[a] = c.periodic[a];
    }
    for (int f = 0; f < 6; f++) rp.prio[f] = c.face_prio[f];
    return rp;
}

// halo records: one per active block with an N_SKIP link, numbered in block-ID order
__global__ void k_bins_halo(const DevMesh m, int8_t *bins) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    bins[B] = (m.status[B] != ST_INACTIVE && (m.bflag[B] & BF_NSKIP)) ? 0 : -1;
}

__global__ void k_set_hid(DevMesh m, const int8_t *bins, const int32_t *rank) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    m.hid[B] = bins[B] == 0 ? rank[B] : -1;
}

// Launch order of level L+1 from that of level L: the children of every
// refined block, in its order (children are numbered as Morton digits).
__global__ void k_bins_order(const DevMesh m, const int32_t *order, const DevCounters *ctr, int L, int8_t *bins) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= m.cap) return;
    int8_t b = -1;
    if (n < ctr->nids[L]) {
        const int32_t first = m.nbrc[order[n]];
        if (first >= 0 && first < m.cap) b = 0;
    }
    bins[n] = b;
}

template <typename Dd>
__global__ void k_expand_order(const DevMesh m, const int32_t *order, const int8_t *bins, const int32_t *rank,
                               int32_t *next) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m.cap * Dd::NC) return;
    const int n = (int)(e / Dd::NC), c = (int)(e - (int64_t)n * Dd::NC);
    if (bins[n] != 0) return;
    const int64_t at = (int64_t)rank[n] * Dd::NC + c;
    if (at < m.cap) next[at] = m.nbrc[order[n]] + c;
}

template <typename Dd>
void build_order(const Ctx &c) {
    const int cap = c.m.cap;
    for (int L = 0; L + 1 < c.m.lmax; L++) {
        const int32_t *cur = c.order + (size_t)L * cap;
        k_bins_order<<<grid_for(cap), 256, 0, c.stream>>>(c.m, cur, c.ctr, L, c.bins);
        run_scan(c, c.bins, cap, 1);
        k_expand_order<Dd><<<grid_for((int64_t)cap * Dd::NC), 256, 0, c.stream>>>(c.m, cur, c.bins, c.rank,
                                                                                  c.order + (size_t)(L + 1) * cap);
    }
}

// leaf blocks with a link into a solid block, per level in ID order (the
// blocks whose momentum exchange is summed after each sweep)
__global__ void k_bins_solid(const DevMesh m, int8_t *bins) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= m.cap) return;
    bins[B] = (m.status[B] == ST_UNREF && (m.bflag[B] & BF_SOLID)) ? m.level[B] : int8_t(-1);
}

__global__ void k_solid_lists(const DevMesh m, const int8_t *bins, const int32_t *rank, int32_t *solidl,
                              DevCounters *ctr) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B < m.cap && bins[B] >= 0) solidl[(int64_t)bins[B] * m.cap + rank[B]] = B;
    if (B == 0)
        for (int L = 0; L < kMaxLevels; L++) ctr->nsolid[L] = L < m.lmax ? ctr->totals[L] : 0;
}

// Cells the interpolation and the averaging of each level move (for the
// byte counts of the solver's kernel statistics): over the interface parents
// of level L, the ghost cells of their children and the parent cells whose
// first fine cell (even i, j, k) is an interface cell.
__global__ void k_target_reset(DevCounters *ctr) {
    if (threadIdx.x < kMaxLevels) {
        ctr->ghost_w[threadIdx.x] = 0;
        ctr->avg_w[threadIdx.x] = 0;
    }
}

// One thread per interface parent of one level (grid y = level); the sums
// are reduced over the wave before one atomic per wave.
template <typename Dd>
__global__ __launch_bounds__(256) void k_target_cells(DevMesh m, const int32_t *__restrict__ iface,
                                                      DevCounters *ctr) {
    const int L = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long g = 0, a = 0;
    if (i < ctr->niface[L]) {
        const int P = iface[(int64_t)L * m.cap + i];
        const int first = m.nbrc[P];
        // fine cells with even coordinates: the first of each parent cell's 2^d
        const uint64_t lead = Dd::D == 3 ? 0x0000050500000505ull : 0x0505ull;
        if (first >= 0 && first <= m.cap - Dd::NC)
            for (int c = 0; c < Dd::NC; c++) {
                g += __popcll(m.gmask[first + c]);
                a += __popcll(m.imask[first + c] & lead);
            }
    }
    for (int off = 32; off > 0; off >>= 1) {
        g += __shfl_xor(g, off, 64);
        a += __shfl_xor(a, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (g) atomicAdd(&ctr->ghost_w[L], g);
        if (a) atomicAdd(&ctr->avg_w[L], a);
    }
}

template <typename Dd>
void masks_and_lists(const Ctx &c) {
    const int cap = c.m.cap;
    k_block_masks<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m);
    k_bins_halo<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins);
    run_scan(c, c.bins, cap, 1);
    k_set_hid<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins, c.rank);
    k_parent_mask<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m);
    const int64_t tot = (int64_t)c.m.lmax * cap;
    k_bins_keep<<<grid_for(tot), 256, 0, c.stream>>>(c.m, c.ids, c.ctr, c.bins, 1);
    run_scan(c, c.bins, tot, c.m.lmax);
    k_compact<<<grid_for(tot), 256, 0, c.stream>>>(c.bins, c.rank, c.ids, c.ids_tmp, cap, tot);
    k_copy_lists<<<grid_for(tot), 256, 0, c.stream>>>(c.ids_tmp, c.iface, cap, c.m.lmax, c.ctr, 0);
    k_bins_keep<<<grid_for(tot), 256, 0, c.stream>>>(c.m, c.ids, c.ctr, c.bins, 2);
    run_scan(c, c.bins, tot, c.m.lmax);
    k_compact<<<grid_for(tot), 256, 0, c.stream>>>(c.bins, c.rank, c.ids, c.ids_tmp, cap, tot);
    k_copy_lists<<<grid_for(tot), 256, 0, c.stream>>>(c.ids_tmp, c.refl, cap, c.m.lmax, c.ctr, 2);
    k_bins_solid<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins);
    run_scan(c, c.bins, cap, c.m.lmax);
    k_solid_lists<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins, c.rank, c.solidl, c.ctr);
    build_order<Dd>(c);
    // sweep lists: the launch order of each level without the refined blocks
    // none of whose children has an N_SKIP link (bins over the order lists,
    // which hold the same blocks as the ID sets)
    k_bins_keep<<<grid_for(tot), 256, 0, c.stream>>>(c.m, c.order, c.ctr, c.bins, 3);
    run_scan(c, c.bins, tot, c.m.lmax);
    k_compact<<<grid_for(tot), 256, 0, c.stream>>>(c.bins, c.rank, c.order, c.ids_tmp, cap, tot);
    k_copy_lists<<<grid_for(tot), 256, 0, c.stream>>>(c.ids_tmp, c.sweep, cap, c.m.lmax, c.ctr, 3);
    k_target_reset<<<1, 64, 0, c.stream>>>(c.ctr);
    k_target_cells<Dd><<<dim3(grid_for(cap), c.m.lmax), 256, 0, c.stream>>>(c.m, c.iface, c.ctr);
}

template <typename Dd>
void init_mesh_t(const Ctx &c) {
    const int cap = c.m.cap;
    k_init_blocks<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m, root_params(c), c.solid, c.bins);
    if (cap > c.nroot) k_init_gap<<<grid_for(cap - c.nroot), 256, 0, c.stream>>>(c.gap, cap, c.nroot);
    run_scan(c, c.bins, cap, 1);
    k_init_ids<<<grid_for(cap), 256, 0, c.stream>>>(c.bins, c.rank, cap, c.ids, c.ctr, c.nroot);
    masks_and_lists<Dd>(c);
}

template <typename Dd>
void adapt_assign_t(const Ctx &c, int n_ref) {
    const int cap = c.m.cap;
    k_bins_refine<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins, 0);
    run_scan(c, c.bins, cap, 1);
    k_assign_first<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.rank, c.gap, c.ctr, c.first, c.rlist, Dd::NC);
    k_gtop_add<<<1, 64, 0, c.stream>>>(c.ctr, -Dd::NC * n_ref, 0);
    k_violating<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.first);
    k_revert<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.ctr);
}

template <typename Dd>
void adapt_build_t(const Ctx &c, int n_ref) {
    const int cap = c.m.cap;
    const int64_t tot = (int64_t)c.m.lmax * cap;
    // S4
    if (n_ref > 0) k_build_children<Dd><<<grid_for((int64_t)n_ref * Dd::NC), 256, 0, c.stream>>>(c.m, c.rlist, c.first, n_ref);
    // S5
    k_zero_freed<<<1, 64, 0, c.stream>>>(c.ctr);
    k_bins_coarsen<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins);
    run_scan(c, c.bins, cap, c.m.lmax);
    k_coarsen<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.rank, c.gap, c.ctr);
    k_gtop_add<<<1, 64, 0, c.stream>>>(c.ctr, 0, 1);
    k_bins_keep<<<grid_for(tot), 256, 0, c.stream>>>(c.m, c.ids, c.ctr, c.bins, 0);
    run_scan(c, c.bins, tot, c.m.lmax);
    k_compact<<<grid_for(tot), 256, 0, c.stream>>>(c.bins, c.rank, c.ids, c.ids_tmp, cap, tot);
    k_copy_lists<<<grid_for(tot), 256, 0, c.stream>>>(c.ids_tmp, c.ids, cap, c.m.lmax, c.ctr, 1);
    // S6
    if (n_ref > 0) {
        k_bins_refine<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.bins, 1);
        run_scan(c, c.bins, cap, c.m.lmax);
        k_append<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.rank, c.first, c.ids, c.ctr);
        k_nids_after_append<Dd><<<1, 64, 0, c.stream>>>(c.ctr, c.m.lmax);
    }
    k_finalize_status<<<grid_for(cap), 256, 0, c.stream>>>(c.m);
    k_branch_leaf<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m);
}

template <typename Dd>
void connectivity_t(const Ctx &c) {
    const int cap = c.m.cap;
    for (int L = 0; L < c.m.lmax; L++) {
        k_nbrc_level<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.ids, c.ctr, L);
        if (L < c.m.lmax - 1)
            k_child_links<Dd><<<grid_for((int64_t)cap * Dd::NC), 256, 0, c.stream>>>(c.m, c.ids, c.ctr, L);
    }
    masks_and_lists<Dd>(c);
}

template <typename Dd>
void tag_vorticity_t(const Ctx &c, double theta, const LadderParams *ladder) {
    const int cap = c.m.cap;
    LadderParams lad{};
    if (ladder) lad = *ladder;
    k_tag_vort_leaf<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.crit, c.ctr, theta, ladder ? 1 : 0, lad);
    k_tag_vort_parent<Dd><<<grid_for(cap), 256, 0, c.stream>>>(c.m);
}

}  // namespace

#define AMR_DIM_DISPATCH(dim, CALL) \
    do {                            \
        if ((dim) == 2) { using Dd = D2; CALL; } else { using Dd = D3; CALL; } \
    } while (0)

void launch_init_mesh(const Ctx &c) { AMR_DIM_DISPATCH(c.dim, init_mesh_t<Dd>(c)); }

void launch_crit_reset(const Ctx &c) {
    k_crit_reset<<<grid_for(c.m.cap), 256, 0, c.stream>>>(c.crit, c.m.cap, c.ctr);
}

void launch_tag_vorticity(const Ctx &c, double theta, const LadderParams *ladder) {
    AMR_DIM_DISPATCH(c.dim, tag_vorticity_t<Dd>(c, theta, ladder));
}

void launch_tag_distance(const Ctx &c, double d_spec, int freeze) {
    DistParams dp;
    dp.dim = c.dim;
    dp.lmax = c.m.lmax;
    dp.n_solid = c.n_solid;
    const int W0 = 4 << (c.m.lmax - 1);
    for (int a = 0; a < 3; a++) dp.dom[a] = c.root[a] * W0;
    for (int f = 0; f < 6; f++) dp.face_kind[f] = c.periodic[f / 2] ? -1 : c.face_kind[f];
    dp.dspec_f = d_spec * (double)(1 << (c.m.lmax - 1));
    dp.freeze = freeze;
    k_tag_distance<<<grid_for(c.m.cap), 256, 0, c.stream>>>(c.m, c.solid_list, dp);
}

__global__ void k_zero_counts(DevCounters *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr->n_ref = ctr->n_coa = ctr->n_rev = 0;
}

void launch_effective_tags(const Ctx &c) {
    k_zero_counts<<<1, 64, 0, c.stream>>>(c.ctr);
    k_effective_tags<<<grid_for(c.m.cap), 256, 0, c.stream>>>(c.m, c.ctr);
}

void launch_adapt_assign(const Ctx &c, int n_ref) { AMR_DIM_DISPATCH(c.dim, adapt_assign_t<Dd>(c, n_ref)); }

void launch_adapt_build(const Ctx &c, int n_ref) { AMR_DIM_DISPATCH(c.dim, adapt_build_t<Dd>(c, n_ref)); }

void launch_connectivity(const Ctx &c, int) { AMR_DIM_DISPATCH(c.dim, connectivity_t<Dd>(c)); }

void launch_out_count(const Ctx &c) {
    const int cap = c.m.cap;
    k_out_count<<<grid_for(cap), 256, 0, c.stream>>>(c.m, c.cnt, c.mb);
    const int nwg = (int)((cap + kScanItems - 1) / kScanItems);
    k_wscan_count<<<nwg, kScanTPB, 0, c.stream>>>(c.cnt, cap, c.scan_part);
    k_scan_part<<<1, 256, 0, c.stream>>>(c.scan_part, nwg, 1, c.ctr);
    k_wscan_apply<<<nwg, kScanTPB, 0, c.stream>>>(c.cnt, cap, c.scan_part, c.off);
    k_out_total<<<1, 64, 0, c.stream>>>(c.cnt, c.off, cap, c.ctr);
}

}  // namespace amr
