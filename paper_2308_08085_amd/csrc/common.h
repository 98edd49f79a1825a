// common.h -- device-side definitions shared by the HIP kernels of the AMR-LBM
// library: lattices, storage formats, the device view of the forest and the
// kernel parameter blocks.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/amr_lbm.h"

namespace amr {

constexpr int kNone = -1;
constexpr int kNSkip = -2;
constexpr int kSolid = -9;
constexpr int kMaxLevels = 8;

enum : int8_t {
    ST_UNREF = 0, ST_REF = 1, ST_REF_CHILD = 2, ST_REF_PERM = 3, ST_NEW = 6, ST_REMOVE = 7, ST_INACTIVE = 8
};
__host__ __device__ inline bool is_refined(int s) { return s == ST_REF || s == ST_REF_CHILD || s == ST_REF_PERM; }

// per-block flags kept by the connectivity rebuild
enum : uint8_t { BF_NSKIP = 1, BF_BOUNDARY = 2, BF_PARENT_MASK = 4, BF_SOLID = 8 };

// ---------------------------------------------------------------------------
// Velocity sets, numbered as in the paper's velocity-set figure.  3-D uses one
// 27-entry table (D3Q19 = its first 19 entries); 2-D its own 9-entry table.
// Weights are the standard quadrature weights.
// direction vectors, (x, y, z) per direction
constexpr int8_t kVec2[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
constexpr int8_t kVec3[27][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},    {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, 0, 1},   {-1, 0, -1},  {0, 1, 1},   {0, -1, -1}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, -1},  {-1, 0, 1},  {0, 1, -1},   {0, -1, 1},  {1, 1, 1},  {-1, -1, -1},
    {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1},  {-1, 1, 1},  {1, -1, -1}};

struct D2 {
    static constexpr int D = 2, NB = 9, MB = 16, NC = 4;
    __host__ __device__ static constexpr int cx(int p) { return kVec2[p][0]; }
    __host__ __device__ static constexpr int cy(int p) { return kVec2[p][1]; }
    __host__ __device__ static constexpr int cz(int) { return 0; }
};
struct D3 {
    static constexpr int D = 3, NB = 27, MB = 64, NC = 8;
    __host__ __device__ static constexpr int cx(int p) { return kVec3[p][0]; }
    __host__ __device__ static constexpr int cy(int p) { return kVec3[p][1]; }
    __host__ __device__ static constexpr int cz(int p) { return kVec3[p][2]; }
};

template <int Q> struct Lat;
template <> struct Lat<9> : D2 {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr double w(int p) { return p == 0 ? 4.0 / 9.0 : (p < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
    __host__ __device__ static constexpr int opp(int p) { return p == 0 ? 0 : (p < 5 ? 1 + ((p + 1) & 3) : 5 + ((p - 3) & 3)); }
};
template <> struct Lat<19> : D3 {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr double w(int p) { return p == 0 ? 1.0 / 3.0 : (p < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
    __host__ __device__ static constexpr int opp(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }
};
template <> struct Lat<27> : D3 {
    static constexpr int Q = 27;
    __host__ __device__ static constexpr double w(int p) {
        return p == 0 ? 8.0 / 27.0 : (p < 7 ? 2.0 / 27.0 : (p < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
    __host__ __device__ static constexpr int opp(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }
};

// index of the neighbour region with per-axis offsets r in {-1,0,1}, as a
// position 0..26 in (x fastest) offset order; LDS link tables are kept in this
// order so kernels can look links up arithmetically
__host__ __device__ constexpr int offset_slot(int rx, int ry, int rz) { return (rx + 1) + 3 * (ry + 1) + 9 * (rz + 1); }

// region slot (in the lattice's own link-table numbering: 0..8 in 2-D,
// 0..26 in 3-D) of a cell position given in local block coordinates that may
// lie one cell outside the block
template <typename Dd>
__host__ __device__ inline int region_of(int x, int y, int z) {
    const int rx = x < 0 ? -1 : (x > 3 ? 1 : 0);
    const int ry = y < 0 ? -1 : (y > 3 ? 1 : 0);
    const int rz = z < 0 ? -1 : (z > 3 ? 1 : 0);
    return offset_slot(rx, ry, rz) - (Dd::D == 2 ? 9 : 0);
}
template <typename Dd> constexpr int kCenterSlot = Dd::D == 2 ? 4 : 13;

// ---------------------------------------------------------------------------
// Storage formats.  Shifted forms keep g = f - w; arithmetic in R.  stnt is a
// non-temporal store: a collide-stream sweep's
// output is read only by the next sweep, after the whole level has streamed
// through the caches, so keeping it out of L2 leaves room there for the
// neighbour rows that the gather reads twice.
template <int S> struct Store;
template <> struct Store<AMR_F64> {
    using T = double; using R = double; static constexpr bool shift = false;
    __device__ static R ld(const T *p) { return *p; }
    __device__ static void st(T *p, R v) { *p = v; }
    __device__ static void stnt(T *p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<AMR_F32> {
    using T = float; using R = float; static constexpr bool shift = false;
    __device__ static R ld(const T *p) { return *p; }
    __device__ static void st(T *p, R v) { *p = v; }
    __device__ static void stnt(T *p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<AMR_F32S> {
    using T = float; using R = float; static constexpr bool shift = true;
    __device__ static R ld(const T *p) { return *p; }
    __device__ static void st(T *p, R v) { *p = v; }
    __device__ static void stnt(T *p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<AMR_F16S> {
    using T = __half; using R = float; static constexpr bool shift = true;
    __device__ static R ld(const T *p) { return __half2float(*p); }
    __device__ static void st(T *p, R v) { *p = __float2half_rn(v); }
    __device__ static void stnt(T *p, R v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, __float2half_rn(v)), reinterpret_cast<uint16_t *>(p));
    }
};
template <> struct Store<AMR_BF16S> {
    using T = __hip_bfloat16; using R = float; static constexpr bool shift = true;
    __device__ static R ld(const T *p) { return __bfloat162float(*p); }
    __device__ static void st(T *p, R v) { *p = __float2bfloat16(v); }
    __device__ static void stnt(T *p, R v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, __float2bfloat16(v)), reinterpret_cast<uint16_t *>(p));
    }
};

inline size_t storage_bytes(int s) { return s == AMR_F64 ? 8 : (s == AMR_F16S || s == AMR_BF16S ? 2 : 4); }

// ---------------------------------------------------------------------------
// Source-indexed storage.  Population p of cell x is kept where the cell it
// streams from wrote it: slot (block of x - c_p, p, cell of x - c_p) of the
// block-major rows [block][p][cell].  A collide-stream sweep therefore reads
// its cells' populations from its own and its neighbours' rows and writes
// only its own rows, whole rows per wave.  Two kinds of population have no
// upstream same-level cell:
//   - the source lies outside the fluid (domain face or solid block): the
//     population is the bounce-back of the cell's own outgoing population in
//     the opposite direction, and is kept in that otherwise unused slot
//     (x, opposite(p));
//   - the source lies in a region covered only by a coarser block (N_SKIP):
//     it is kept in the block's halo record, one per block with an N_SKIP
//     link, at entry halo_index(p, cell).
// The values are exactly those of a two-buffer push scheme; only where they
// live differs.
template <typename Lt>
struct HaloIndex {
    int16_t idx[Lt::Q][Lt::MB];
    int n;
    constexpr HaloIndex() : idx(), n(0) {
        for (int p = 0; p < Lt::Q; p++)
            for (int l = 0; l < Lt::MB; l++) {
                const int sx = (l & 3) - Lt::cx(p), sy = ((l >> 2) & 3) - Lt::cy(p), sz = (l >> 4) - Lt::cz(p);
                const bool inside = sx >= 0 && sx < 4 && sy >= 0 && sy < 4 && sz >= 0 && sz < 4;
                idx[p][l] = inside ? int16_t(-1) : int16_t(n++);
            }
    }
};
template <typename Lt> constexpr HaloIndex<Lt> kHalo{};
inline int halo_entries(int q) {
    return q == 9 ? kHalo<Lat<9>>.n : (q == 19 ? kHalo<Lat<19>>.n : kHalo<Lat<27>>.n);
}

// ---------------------------------------------------------------------------
// Device view of the forest.  Block metadata is structure-of-arrays: entry p
// of block B lives at [p * cap + B] (the paper's kappa + p N_blocks layout);
// distribution rows are block-major, [B][q][l], followed by the halo records.
struct DevMesh {
    int32_t cap;
    int64_t capc;
    int32_t lmax;
    int64_t halo_base;  // first halo slot in a distribution buffer (= cap * Q * Mb)
    int32_t nh;         // slots per halo record
    int32_t interp;     // AMR_INTERP_LINEAR / AMR_INTERP_CUBIC
    double *force;      // [cap][3] momentum exchange with solid blocks since the last reset
    int32_t *hid;       // halo record of each block, -1 if it has no N_SKIP link
    int32_t *parent;    // parent block, -1 on the root level
    int8_t *fresh;      // 1 for blocks created by the adaptation in progress
    int32_t *nbr, *nbrc, *X;
    int8_t *level, *status, *tag, *ldes, *viol;
    uint8_t *bflag;
    uint64_t *gmask, *imask;  // ghost / interface cell bitmasks (bit l)
};

struct BCParams {
    int32_t kind[6];
    double u[6][3];
};

struct LevelParams {
    int32_t par[kMaxLevels];     // buffer holding each level's current data
    double omega[kMaxLevels];
    double r_cf[kMaxLevels];     // coarse->fine rescaling of level L -> L+1
    double r_fc[kMaxLevels];     // fine->coarse rescaling of level L+1 -> L
};

// One simulation of a batch, as the fused solver kernels see it: its mesh
// views, both distribution buffers, relaxation and rescaling parameters,
// boundary conditions, and its launch-order / interface lists with their
// on-device counts.
struct SimDesc {
    DevMesh m;
    void *f[2];
    LevelParams lp;
    BCParams bc;
    const int32_t *order;   // [lmax][cap]
    const int32_t *iface;   // [lmax][cap]
    const int32_t *solid;   // [lmax][cap] leaf blocks next to a solid block
    const int32_t *nids;    // [kMaxLevels] on the device
    const int32_t *niface;  // [kMaxLevels] on the device
    const int32_t *nsolid;  // [kMaxLevels] on the device
    int32_t force_on;       // accumulate the momentum exchange (else no solid items)
};

// batch work item: simulation index in the top 8 bits, block ID below
constexpr int kItemSimShift = 24;
constexpr uint32_t kItemBlockMask = (1u << kItemSimShift) - 1u;
constexpr int kMaxBatchSims = 255;

// XCD-aware workgroup order: dispatch places workgroup w on XCD (w mod 8);
// give each XCD a contiguous range of work so neighbouring blocks share an L2.
__device__ inline int xcd_remap(int wg, int nwg) {
    int per = nwg >> 3;
    int full = per << 3;
    if (wg >= full) return wg;
    return (wg & 7) * per + (wg >> 3);
}

}  // namespace amr
