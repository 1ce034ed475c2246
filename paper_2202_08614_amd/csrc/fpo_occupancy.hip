// Occupancy at one time (gfx950): which parts of the union octree hold a leaf
// whose density is positive at time t.  The union octree of Sec. 4.2 keeps
// every cell that is occupied in some frame; at a given time many of its
// leaves have sigma(t) <= 0 (Eq. 7 through the ReLU), contribute nothing to
// the image, and need not be walked.  Both passes read sigma(t) from a
// snapshot (the decode pass's fpo_bake_times output), or from the density
// plane the same call writes beside it, so they agree with the snapshot
// render that consumes them.
//
//   fpo_prune_at: a copy of the child table per time in which every child
//   slot whose subtree holds no leaf with sigma_eff(t) > 0 is empty.  Rows are
//   resolved bottom up: a first pass clears transparent leaves, then each of
//   max_depth - 1 passes clears internal children whose (already cleared) row
//   is empty; after pass p the rows p levels above the deepest are exact.  A
//   pass may read a row another thread of the same pass is clearing; entries
//   only ever go from kept to empty, and a row is written whole only where an
//   entry changed, so a read sees each entry either kept or cleared: a stale
//   read keeps an entry one pass longer and the last pass is exact.
//
//   fpo_coarse_occupancy_at: the 64^3 occupancy bits of fpo_coarse_occupancy
//   restricted to leaves with sigma_eff(t) > 0 (set bits of the cells each
//   such leaf overlaps, then dilate by one cell in one block through LDS).
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"

namespace fpo {
namespace dev {

// Source of sigma(t) besides F32 and BF16 snapshot records: a density plane
// of one FP32 per leaf (fpo_bake_times sigma_out).
constexpr int kSigmaPlane = 100;

// sigma(t) of one leaf from a snapshot record (value 0), as the render reads
// it, or from a density plane.
template <int SDT>
__device__ inline float snapshot_sigma(const void* snap, int64_t leaf)
{
    if constexpr (SDT == kSigmaPlane) {
        return static_cast<const float*>(snap)[leaf];
    } else if constexpr (SDT == FPO_F32) {
        return static_cast<const float*>(snap)[leaf * 32];
    } else {
        const uint16_t b = static_cast<const uint16_t*>(snap)[leaf * 32];
        return __uint_as_float((uint32_t)b << 16);
    }
}

struct PruneLaunch {
    const int32_t* children;   // [n_nodes][8]
    int32_t* out;              // [n_t][n_nodes][8]
    const void* snap;          // [n_t] snapshots, snap_stride leaf records apart
    int64_t snap_stride;
    int64_t n_nodes;
    int32_t n_t;
    int32_t n_leaves;
    float sigma_scale;
    int64_t lo, cnt;           // node passes: rows lo .. lo + cnt - 1 of each time
};

// First pass: one thread per (time, node) row; leaves are kept iff opaque at t,
// internal children copied, empty slots stay empty.
template <int SDT>
__global__ __launch_bounds__(kBlock) void prune_leaves_kernel(PruneLaunch a)
{
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= a.n_nodes * a.n_t) return;
    const int t = (int)(id / a.n_nodes);
    const int64_t node = id - (int64_t)t * a.n_nodes;
    const size_t rec = SDT == kSigmaPlane ? 4 : SDT == FPO_F32 ? 128 : 64;
    const void* snap = static_cast<const char*>(a.snap) + (size_t)t * (size_t)a.snap_stride * rec;
    const int4* row = reinterpret_cast<const int4*>(a.children + node * 8);
    int e[8];
    const int4 r0 = row[0], r1 = row[1];
    e[0] = r0.x; e[1] = r0.y; e[2] = r0.z; e[3] = r0.w;
    e[4] = r1.x; e[5] = r1.y; e[6] = r1.z; e[7] = r1.w;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (e[c] < 0) {
            const int leaf = -e[c] - 1;
            const bool opaque = leaf < a.n_leaves && a.sigma_scale * fmaxf(snapshot_sigma<SDT>(snap, leaf), 0.0f) > 0.0f;
            e[c] = opaque ? e[c] : 0;
        } else if (e[c] >= a.n_nodes) {
            e[c] = 0;   // malformed entry: the walk treats it as empty too
        }
    }
    int4* o = reinterpret_cast<int4*>(a.out + ((int64_t)t * a.n_nodes + node) * 8);
    o[0] = make_int4(e[0], e[1], e[2], e[3]);
    o[1] = make_int4(e[4], e[5], e[6], e[7]);
}

// Later passes: clear internal children whose row at this time is empty,
// for rows a.lo .. a.lo + a.cnt - 1 (every row, or one level of the tree).
// Rows are read and written as two 16-byte words (a row another thread clears
// in the same pass may be read old or new; either is safe, see above).
__global__ __launch_bounds__(kBlock) void prune_nodes_kernel(PruneLaunch a)
{
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= a.cnt * a.n_t) return;
    const int t = (int)(id / a.cnt);
    const int64_t node = a.lo + (id - (int64_t)t * a.cnt);
    int4* base = reinterpret_cast<int4*>(a.out + (int64_t)t * a.n_nodes * 8);
    const int4 r0 = base[2 * node], r1 = base[2 * node + 1];
    int e[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
    bool changed = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (e[c] <= 0) continue;
        const int4 c0 = base[2 * (int64_t)e[c]], c1 = base[2 * (int64_t)e[c] + 1];
        const bool any = (c0.x | c0.y | c0.z | c0.w | c1.x | c1.y | c1.z | c1.w) != 0;
        if (!any) {
            e[c] = 0;
            changed = true;
        }
    }
    if (changed) {
        base[2 * node] = make_int4(e[0], e[1], e[2], e[3]);
        base[2 * node + 1] = make_int4(e[4], e[5], e[6], e[7]);
    }
}

// Two-level tables: one thread per (time, node, child octant a) writes the
// 8 entries (c, g_b), b < 8, of its 64-byte run: c = children[x][a] and g_b
// the entries of c's row when c is an internal node (else 0).
__global__ __launch_bounds__(kBlock) void grandchild_kernel(const int32_t* children, int64_t n_nodes, int32_t n_t,
                                                            int64_t n_rows, int2* out)
{
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= n_rows * 8 * n_t) return;
    const int64_t per_t = n_rows * 8;
    const int t = (int)(id / per_t);
    const int64_t xa = id - (int64_t)t * per_t;             // x * 8 + a
    const int32_t* tab = children + (int64_t)t * n_nodes * 8;
    const int c = tab[xa];
    int g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (c > 0 && c < n_nodes) {
        const int4* row = reinterpret_cast<const int4*>(tab + (int64_t)c * 8);
        const int4 r0 = row[0], r1 = row[1];
        g[0] = r0.x; g[1] = r0.y; g[2] = r0.z; g[3] = r0.w;
        g[4] = r1.x; g[5] = r1.y; g[6] = r1.z; g[7] = r1.w;
    }
    int4* o = reinterpret_cast<int4*>(out + ((int64_t)t * n_rows * 64 + xa * 8));
#pragma unroll
    for (int b = 0; b < 4; ++b) o[b] = make_int4(c, g[2 * b], c, g[2 * b + 1]);
}

struct OccLaunch {
    const int4* cells;         // [n_leaves] (depth, i, j, k), slot order
    const void* snap;
    uint32_t* bits;            // [FPO_COARSE_WORDS]
    int32_t n_leaves;
    int32_t max_depth;
    float sigma_scale;
};

__global__ __launch_bounds__(kBlock) void zero_words_kernel(uint32_t* w, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) w[i] = 0u;
}

// Mark the coarse cells each opaque leaf overlaps (undilated).
template <int SDT>
__global__ __launch_bounds__(kBlock) void occupancy_mark_kernel(OccLaunch a)
{
    const int leaf = blockIdx.x * kBlock + threadIdx.x;
    if (leaf >= a.n_leaves) return;
    if (!(a.sigma_scale * fmaxf(snapshot_sigma<SDT>(a.snap, leaf), 0.0f) > 0.0f)) return;
    const int4 c = a.cells[leaf];
    const int d = c.x;
    if (d < 1 || d > a.max_depth) return;
    constexpr int kLog = 6;   // 64 coarse cells per axis
    int lo[3], hi[3];
    const int v[3] = {c.y, c.z, c.w};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (d >= kLog) {
            lo[ax] = hi[ax] = v[ax] >> (d - kLog);
        } else {
            lo[ax] = v[ax] << (kLog - d);
            hi[ax] = lo[ax] + (1 << (kLog - d)) - 1;
        }
        lo[ax] = min(max(lo[ax], 0), FPO_COARSE_RES - 1);
        hi[ax] = min(max(hi[ax], 0), FPO_COARSE_RES - 1);
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                const int bit = (z * FPO_COARSE_RES + y) * FPO_COARSE_RES + x;
                const uint32_t m = 1u << (bit & 31);
                if (!(a.bits[bit >> 5] & m)) atomicOr(a.bits + (bit >> 5), m);
            }
}

// Dilate by one cell in x, y and z, in one block: the 32 KB grid is staged
// in LDS, each thread ORs the 27 neighbours of its words.
__global__ __launch_bounds__(1024) void occupancy_dilate_kernel(uint32_t* bits)
{
    constexpr int N = FPO_COARSE_RES;
    constexpr int kWords = FPO_COARSE_WORDS;
    __shared__ uint32_t s[kWords];
    for (int i = threadIdx.x; i < kWords; i += 1024) s[i] = bits[i];
    __syncthreads();
    // row (z, y) holds two words: x 0..31 and x 32..63
    for (int w = threadIdx.x; w < kWords; w += 1024) {
        const int row = w >> 1;
        const int half = w & 1;
        const int z = row / N, y = row % N;
        uint32_t acc = 0;
        for (int dz = -1; dz <= 1; ++dz) {
            const int zz = z + dz;
            if (zz < 0 || zz >= N) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= N) continue;
                const int r = zz * N + yy;
                const uint32_t lo = s[2 * r], hi = s[2 * r + 1];
                // the 64-bit row shifted by -1, 0, +1 in x, this word's 32 bits
                const uint64_t full = ((uint64_t)hi << 32) | lo;
                const uint64_t sp = full | (full << 1) | (full >> 1);
                acc |= half ? (uint32_t)(sp >> 32) : (uint32_t)sp;
            }
        }
        bits[w] = acc;
    }
}

}  // namespace dev
}  // namespace fpo

using namespace fpo;

namespace {

// Shared body of fpo_prune_at and fpo_prune_at_sigma: src holds n_t sources of
// sigma(t) (records of `kind` or a density plane), `stride` leaves apart.
fpo_status prune_impl(const fpo_tree_view* tree, const void* src, int kind, int64_t stride, int32_t n_t,
                      int32_t* children_out, void* stream, const char* name)
{
    fpo_status st = check_tree(tree, false, true);
    if (st != FPO_OK) return st;
    if (!src || !children_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (n_t > 1 && stride < tree->n_leaves) return fail(FPO_E_INVALID, "stride between times < n_leaves");
    if ((((uintptr_t)tree->children) | ((uintptr_t)children_out)) & 15)
        return fail(FPO_E_INVALID, "children and children_out must be 16-byte aligned");
    const int64_t rows = tree->n_nodes * (int64_t)n_t;
    if (rows > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rows");
    dev::PruneLaunch a;
    a.children = tree->children;
    a.out = children_out;
    a.snap = src;
    a.snap_stride = stride;
    a.n_nodes = tree->n_nodes;
    a.n_t = n_t;
    a.n_leaves = (int32_t)tree->n_leaves;
    a.sigma_scale = tree->layout.sigma_scale;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned grid = (unsigned)((rows + dev::kBlock - 1) / dev::kBlock);
    if (kind == FPO_F32)
        hipLaunchKernelGGL(dev::prune_leaves_kernel<FPO_F32>, dim3(grid), dim3(dev::kBlock), 0, s, a);
    else if (kind == FPO_BF16)
        hipLaunchKernelGGL(dev::prune_leaves_kernel<FPO_BF16>, dim3(grid), dim3(dev::kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(dev::prune_leaves_kernel<dev::kSigmaPlane>, dim3(grid), dim3(dev::kBlock), 0, s, a);
    if ((st = launch_status(name)) != FPO_OK) return st;
    if (tree->level_offsets) {
        // one pass per level, bottom up: the nodes of depth L clear their children
        // (depth L + 1), whose rows the pass before has settled; the deepest
        // nodes have leaf children only
        for (int L = tree->max_depth - 2; L >= 0; --L) {
            a.lo = tree->level_offsets[L];
            a.cnt = tree->level_offsets[L + 1] - a.lo;
            if (a.cnt == 0) continue;
            const unsigned g = (unsigned)((a.cnt * n_t + dev::kBlock - 1) / dev::kBlock);
            hipLaunchKernelGGL(dev::prune_nodes_kernel, dim3(g), dim3(dev::kBlock), 0, s, a);
            if ((st = launch_status(name)) != FPO_OK) return st;
        }
        return FPO_OK;
    }
    a.lo = 0;
    a.cnt = tree->n_nodes;
    for (int pass = 1; pass < tree->max_depth; ++pass) {
        hipLaunchKernelGGL(dev::prune_nodes_kernel, dim3(grid), dim3(dev::kBlock), 0, s, a);
        if ((st = launch_status(name)) != FPO_OK) return st;
    }
    return FPO_OK;
}

}  // namespace

extern "C" fpo_status fpo_prune_at(const fpo_tree_view* tree, const void* snapshots, fpo_dtype snapshot_dtype,
                                   int64_t snapshot_stride, int32_t n_t, int32_t* children_out, void* stream)
{
    ApiRange api_range_("fpo_prune_at");
    if (snapshot_dtype != FPO_F32 && snapshot_dtype != FPO_BF16)
        return fail(FPO_E_INVALID, "snapshot_dtype must be F32 or BF16");
    return prune_impl(tree, snapshots, snapshot_dtype, snapshot_stride, n_t, children_out, stream, "fpo_prune_at");
}

extern "C" fpo_status fpo_prune_at_sigma(const fpo_tree_view* tree, const float* sigma, int64_t sigma_stride,
                                         int32_t n_t, int32_t* children_out, void* stream)
{
    ApiRange api_range_("fpo_prune_at_sigma");
    return prune_impl(tree, sigma, dev::kSigmaPlane, sigma_stride, n_t, children_out, stream, "fpo_prune_at_sigma");
}

extern "C" fpo_status fpo_coarse_occupancy_at(const int32_t* leaf_cells, int64_t n_leaves, int32_t max_depth,
                                              const void* snapshot, fpo_dtype snapshot_dtype, float sigma_scale,
                                              uint32_t* bits_out, void* stream)
{
    ApiRange api_range_("fpo_coarse_occupancy_at");
    if (!leaf_cells || !snapshot || !bits_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_leaves < 1 || n_leaves > INT32_MAX - 1) return fail(FPO_E_INVALID, "n_leaves out of range");
    if (max_depth < 1 || max_depth > FPO_MAX_DEPTH) return fail(FPO_E_INVALID, "max_depth must be in 1..10");
    if (snapshot_dtype != FPO_F32 && snapshot_dtype != FPO_BF16)
        return fail(FPO_E_INVALID, "snapshot_dtype must be F32 or BF16");
    if (!(sigma_scale >= 0.0f)) return fail(FPO_E_INVALID, "sigma_scale must be >= 0");
    if (((uintptr_t)leaf_cells) & 15) return fail(FPO_E_INVALID, "leaf_cells must be 16-byte aligned");
    dev::OccLaunch a;
    a.cells = reinterpret_cast<const int4*>(leaf_cells);
    a.snap = snapshot;
    a.bits = bits_out;
    a.n_leaves = (int32_t)n_leaves;
    a.max_depth = max_depth;
    a.sigma_scale = sigma_scale;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(dev::zero_words_kernel, dim3((FPO_COARSE_WORDS + dev::kBlock - 1) / dev::kBlock),
                       dim3(dev::kBlock), 0, s, bits_out, FPO_COARSE_WORDS);
    const unsigned grid = (unsigned)((n_leaves + dev::kBlock - 1) / dev::kBlock);
    if (snapshot_dtype == FPO_F32)
        hipLaunchKernelGGL(dev::occupancy_mark_kernel<FPO_F32>, dim3(grid), dim3(dev::kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(dev::occupancy_mark_kernel<FPO_BF16>, dim3(grid), dim3(dev::kBlock), 0, s, a);
    hipLaunchKernelGGL(dev::occupancy_dilate_kernel, dim3(1), dim3(1024), 0, s, bits_out);
    return launch_status("fpo_coarse_occupancy_at");
}

extern "C" fpo_status fpo_grandchild_tables(const int32_t* children, int64_t n_nodes, int32_t n_t, int64_t n_rows,
                                            int32_t* out, void* stream)
{
    ApiRange api_range_("fpo_grandchild_tables");
    if (!children || !out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_nodes < 1 || n_nodes > INT32_MAX / 32) return fail(FPO_E_INVALID, "n_nodes out of range");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (n_rows < 1 || n_rows > n_nodes || n_rows > INT32_MAX / 512) return fail(FPO_E_INVALID, "n_rows out of range");
    if (((uintptr_t)children & 15) || ((uintptr_t)out & 15))
        return fail(FPO_E_INVALID, "children and out must be 16-byte aligned");
    const int64_t threads = n_rows * 8 * (int64_t)n_t;
    if (threads > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rows");
    hipLaunchKernelGGL(dev::grandchild_kernel, dim3((unsigned)((threads + dev::kBlock - 1) / dev::kBlock)),
                       dim3(dev::kBlock), 0, static_cast<hipStream_t>(stream), children, n_nodes, n_t, n_rows,
                       reinterpret_cast<int2*>(out));
    return launch_status("fpo_grandchild_tables");
}
