// Host side of libfpo: error reporting, octree construction, the FP64 time
// basis and camera packing.  No device work happens here.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "fpo.h"
#include "fpo_internal.h"

namespace fpo {

static thread_local std::string g_last_error;

fpo_status fail(fpo_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

fpo_status ok() { return FPO_OK; }

ApiRange::ApiRange(const char* name) { roctxRangePushA(name); }
ApiRange::~ApiRange() { roctxRangePop(); }

void fault_point_alloc()
{
    const char* f = std::getenv("FPO_FAULT");
    if (f && std::strcmp(f, "alloc") == 0) throw std::bad_alloc();
}

bool force_fallback()
{
    const char* f = std::getenv("FPO_FORCE_FALLBACK");
    return f && f[0] == '1' && f[1] == '\0';
}

fpo_status launch_status(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FPO_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return FPO_OK;
}

fpo_status check_tree(const fpo_tree_view* tree, bool need_coeffs, bool allow_layouts)
{
    if (!tree) return fail(FPO_E_INVALID, "tree is NULL");
    if (!tree->children) return fail(FPO_E_INVALID, "tree->children is NULL");
    // byte offsets into the child table are 32-bit: at most 2^26 - 1 nodes
    if (tree->n_nodes < 1 || tree->n_nodes > INT32_MAX / 32)
        return fail(FPO_E_INVALID, "tree->n_nodes out of range");
    if (tree->max_depth < 1 || tree->max_depth > FPO_MAX_DEPTH)
        return fail(FPO_E_INVALID, "tree->max_depth must be in 1..10");
    if (tree->n_leaves < 1 || tree->n_leaves > INT32_MAX - 1)
        return fail(FPO_E_INVALID, "tree->n_leaves out of range");
    if (tree->leaf_stride < tree->n_leaves) return fail(FPO_E_INVALID, "leaf_stride < n_leaves");
    const fpo_layout& L = tree->layout;
    if (L.sh_degree != FPO_SH_DEGREE) return fail(FPO_E_UNSUPPORTED, "only l_max = 2 is compiled");
    if (!default_layout(L) && !(allow_layouts && layout_supported(L.n_sigma, L.n_sh_fourier)))
        return fail(FPO_E_UNSUPPORTED, allow_layouts ? "layout (n1, n2) not compiled"
                                                     : "this call is compiled for the (n1=31, n2=5) layout only");
    if (!(L.period > 0.0f) || !std::isfinite(L.period)) return fail(FPO_E_INVALID, "layout.period must be > 0");
    if (!(L.sigma_scale >= 0.0f) || !std::isfinite(L.sigma_scale))
        return fail(FPO_E_INVALID, "layout.sigma_scale must be finite and >= 0");
    if (tree->grandchildren) {
        // 32-bit byte offsets into the two-level table: 512 bytes per row
        if (tree->n_grandchild_rows < 1 || tree->n_grandchild_rows > tree->n_nodes ||
            tree->n_grandchild_rows > INT32_MAX / 512)
            return fail(FPO_E_INVALID, "tree->n_grandchild_rows out of range");
        if (reinterpret_cast<uintptr_t>(tree->grandchildren) & 7)
            return fail(FPO_E_INVALID, "tree->grandchildren must be 8-byte aligned");
    }
    if (tree->level_offsets) {
        const int64_t* lo = tree->level_offsets;
        if (lo[0] != 0 || lo[tree->max_depth] != tree->n_nodes)
            return fail(FPO_E_INVALID, "tree->level_offsets must start at 0 and end at n_nodes");
        for (int L = 0; L < tree->max_depth; ++L)
            if (lo[L + 1] < lo[L]) return fail(FPO_E_INVALID, "tree->level_offsets must not decrease");
    }
    if (tree->bounds) {
        const int32_t G = int32_t(1) << tree->max_depth;
        for (int a = 0; a < 3; ++a)
            if (tree->bounds[a] < 0 || tree->bounds[a] >= tree->bounds[3 + a] || tree->bounds[3 + a] > G)
                return fail(FPO_E_INVALID, "tree->bounds must hold 0 <= lo < hi <= 2^max_depth on every axis");
    }
    if (need_coeffs) {
        if (!tree->coeffs) return fail(FPO_E_INVALID, "tree->coeffs is NULL");
        if (tree->dtype != FPO_F32 && tree->dtype != FPO_BF16 && tree->dtype != FPO_FP8_E4M3)
            return fail(FPO_E_INVALID, "unknown coefficient dtype");
        if (tree->dtype != FPO_F32 && !tree->leaf_scale)
            return fail(FPO_E_INVALID, "quantised coefficients need leaf_scale");
    }
    return FPO_OK;
}

fpo_status check_opts(const fpo_render_opts* opts, const fpo_tree_view* tree, bool allow_skip, bool allow_record,
                      bool skip_workspace)
{
    if (!opts) return fail(FPO_E_INVALID, "opts is NULL");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(opts->bg[c])) return fail(FPO_E_INVALID, "opts->bg must be finite");
    if (!(opts->stop_T >= 0.0f && opts->stop_T < 1.0f)) return fail(FPO_E_INVALID, "opts->stop_T must be in [0, 1)");
    if (opts->flags == FPO_RAYS_RECORD) {
        if (!allow_record) return fail(FPO_E_INVALID, "FPO_RAYS_RECORD is for fpo_render_rays and fpo_render_backward");
        if (opts->snapshot) return fail(FPO_E_UNSUPPORTED, "FPO_RAYS_RECORD runs in Fourier mode only");
    } else if (opts->flags != 0) {
        if (!allow_skip) return fail(FPO_E_INVALID, "opts->flags must be 0 for this call");
        if (opts->flags != FPO_RENDER_SKIP_COARSE && opts->flags != FPO_RENDER_SKIP_PROPOSAL)
            return fail(FPO_E_INVALID, "opts->flags must be 0, FPO_RENDER_SKIP_COARSE or FPO_RENDER_SKIP_PROPOSAL");
        if (!opts->coarse_bits) return fail(FPO_E_INVALID, "skip modes need opts->coarse_bits");
        if (opts->flags == FPO_RENDER_SKIP_PROPOSAL && !opts->proposal)
            return fail(FPO_E_INVALID, "FPO_RENDER_SKIP_PROPOSAL needs opts->proposal");
        if (skip_workspace && (!opts->workspace || (reinterpret_cast<uintptr_t>(opts->workspace) & 7) != 0))
            return fail(FPO_E_INVALID, "skip modes need an 8-byte aligned opts->workspace");
        if ((reinterpret_cast<uintptr_t>(opts->proposal) & 15) != 0)
            return fail(FPO_E_INVALID, "opts->proposal must be 16-byte aligned");
    }
    if (opts->snapshot) {
        if (opts->snapshot_dtype != FPO_F32 && opts->snapshot_dtype != FPO_BF16)
            return fail(FPO_E_INVALID, "snapshot_dtype must be F32 or BF16");
        if (opts->snapshot_cam_stride < 0) return fail(FPO_E_INVALID, "snapshot_cam_stride < 0");
    }
    (void)tree;
    return FPO_OK;
}

fpo_status record_layout(const fpo_render_opts* opts, int64_t n_rays, RecordLayout& out)
{
    if (!opts->workspace || (reinterpret_cast<uintptr_t>(opts->workspace) & 15) != 0)
        return fail(FPO_E_INVALID, "FPO_RAYS_RECORD needs a 16-byte aligned opts->workspace");
    const int64_t head = (4 * n_rays + 255) / 256 * 256;
    const int64_t per_ray = (opts->workspace_bytes - head) / FPO_RECORD_BYTES / std::max<int64_t>(n_rays, 1);
    if (opts->workspace_bytes < head || per_ray < 1)
        return fail(FPO_E_INVALID, "opts->workspace_bytes below the counts and one record per ray");
    out.count = static_cast<int32_t*>(opts->workspace);
    out.records = static_cast<char*>(opts->workspace) + head;
    out.cap = (int32_t)std::min<int64_t>(per_ray, 1 << 20);
    return FPO_OK;
}

static void normalize3(double v[3])
{
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

fpo_status camera_frame(const fpo_camera& cam, float out[12])
{
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(cam.eye[a]) || !std::isfinite(cam.fwd[a]) || !std::isfinite(cam.up[a]))
            return fail(FPO_E_INVALID, "camera vectors must be finite");
    if (cam.width < 1 || cam.height < 1) return fail(FPO_E_INVALID, "camera size must be positive");
    if (!(cam.fov_y_deg > 0.0f && cam.fov_y_deg < 180.0f))
        return fail(FPO_E_INVALID, "camera fov_y_deg must be in (0, 180)");
    if (!std::isfinite(cam.time)) return fail(FPO_E_INVALID, "camera time must be finite");
    double f[3] = {cam.fwd[0], cam.fwd[1], cam.fwd[2]};
    const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fn > 0.0)) return fail(FPO_E_INVALID, "camera fwd is zero");
    normalize3(f);
    double r[3] = {f[1] * cam.up[2] - f[2] * cam.up[1], f[2] * cam.up[0] - f[0] * cam.up[2],
                   f[0] * cam.up[1] - f[1] * cam.up[0]};
    const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rn > 1e-12)) return fail(FPO_E_INVALID, "camera up is parallel to fwd");
    normalize3(r);
    const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    const double tan_h = std::tan(0.5 * (double)cam.fov_y_deg * M_PI / 180.0);
    const double tan_x = tan_h * (double)cam.width / (double)cam.height;
    for (int a = 0; a < 3; ++a) {
        out[a] = cam.eye[a];
        out[3 + a] = (float)f[a];
        out[6 + a] = (float)(r[a] * tan_x);
        out[9 + a] = (float)(u[a] * tan_h);
    }
    return FPO_OK;
}

void basis_row(double t, double period, int n, float* out)
{
    for (int i = 0; i < FPO_BASIS_STRIDE; ++i) {
        double v = 0.0;
        if (i < n) {
            // Eq. 8: cos(i pi t / T) for even i, sin((i + 1) pi t / T) for odd i.
            v = (i % 2 == 0) ? std::cos((double)i * M_PI * t / period)
                             : std::sin((double)(i + 1) * M_PI * t / period);
        }
        out[i] = (float)v;
    }
}

// Spread the low 10 bits of v so that bit b lands at bit 3b.
static uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

}  // namespace fpo

using namespace fpo;

extern "C" const char* fpo_last_error(void) { return g_last_error.c_str(); }

extern "C" fpo_status fpo_leaf_bounds(const int32_t* leaf_dijk, int64_t n_leaves, int32_t max_depth,
                                      int32_t* bounds_out)
{
    ApiRange api_range_("fpo_leaf_bounds");
    if (!leaf_dijk || !bounds_out) return fail(FPO_E_INVALID, "leaf_dijk and bounds_out must not be NULL");
    if (n_leaves < 1) return fail(FPO_E_INVALID, "n_leaves out of range");
    if (max_depth < 1 || max_depth > FPO_MAX_DEPTH) return fail(FPO_E_INVALID, "max_depth must be in 1..10");
    const int32_t G = int32_t(1) << max_depth;
    int32_t lo[3] = {G, G, G}, hi[3] = {0, 0, 0};
    for (int64_t l = 0; l < n_leaves; ++l) {
        const int32_t* c = leaf_dijk + 4 * l;
        if (c[0] < 1 || c[0] > max_depth) return fail(FPO_E_INVALID, "leaf " + std::to_string(l) + ": depth out of range");
        const int32_t sh = max_depth - c[0], g = int32_t(1) << c[0];
        for (int a = 0; a < 3; ++a) {
            if (c[1 + a] < 0 || c[1 + a] >= g)
                return fail(FPO_E_INVALID, "leaf " + std::to_string(l) + ": coordinate out of range");
            lo[a] = std::min(lo[a], c[1 + a] << sh);
            hi[a] = std::max(hi[a], (c[1 + a] + 1) << sh);
        }
    }
    for (int a = 0; a < 3; ++a) {
        bounds_out[a] = lo[a];
        bounds_out[3 + a] = hi[a];
    }
    return FPO_OK;
}

extern "C" fpo_status fpo_build_tree(const int32_t* leaf_dijk, int64_t n_leaves, int32_t max_depth,
                                     int32_t* children_out, int64_t cap_nodes, int64_t* n_nodes_out,
                                     int64_t* perm_out)
{
    ApiRange api_range_("fpo_build_tree");
    try {
        if (!leaf_dijk) return fail(FPO_E_INVALID, "leaf_dijk is NULL");
        if (!n_nodes_out) return fail(FPO_E_INVALID, "n_nodes_out is NULL");
        if (n_leaves < 1 || n_leaves > INT32_MAX - 1) return fail(FPO_E_INVALID, "n_leaves out of range");
        if (max_depth < 1 || max_depth > FPO_MAX_DEPTH) return fail(FPO_E_INVALID, "max_depth must be in 1..10");
        const int D = max_depth;
        fault_point_alloc();
        std::vector<uint64_t> code(n_leaves);   // Morton code of the leaf's min corner on the finest lattice
        for (int64_t l = 0; l < n_leaves; ++l) {
            const int32_t d = leaf_dijk[4 * l], i = leaf_dijk[4 * l + 1], j = leaf_dijk[4 * l + 2],
                          k = leaf_dijk[4 * l + 3];
            if (d < 1 || d > D) return fail(FPO_E_INVALID, "leaf " + std::to_string(l) + ": depth out of range");
            const int64_t g = int64_t(1) << d;
            if (i < 0 || j < 0 || k < 0 || i >= g || j >= g || k >= g)
                return fail(FPO_E_INVALID, "leaf " + std::to_string(l) + ": coordinate out of range");
            const int sh = D - d;
            code[l] = spread3((uint64_t)i << sh) | (spread3((uint64_t)j << sh) << 1) | (spread3((uint64_t)k << sh) << 2);
        }
        std::vector<int64_t> order(n_leaves);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
            return code[a] < code[b] || (code[a] == code[b] && a < b);
        });
        // Octree cells are contiguous Morton ranges: leaves are disjoint iff the
        // sorted ranges do not overlap.
        for (int64_t s = 1; s < n_leaves; ++s) {
            const int64_t a = order[s - 1], b = order[s];
            const int da = leaf_dijk[4 * a];
            const uint64_t end_a = code[a] + (uint64_t(1) << (3 * (D - da)));
            if (code[b] < end_a) {
                const bool dup = code[a] == code[b] && leaf_dijk[4 * a] == leaf_dijk[4 * b];
                return fail(FPO_E_INVALID, std::string(dup ? "duplicate leaves " : "overlapping leaves ") +
                                               std::to_string(a) + " and " + std::to_string(b));
            }
        }
        // Internal nodes per level: distinct level-L prefixes of leaves deeper than L,
        // numbered breadth first in Morton order.
        std::vector<std::vector<uint64_t>> prefixes(D);
        std::vector<int64_t> base(D + 1, 0);
        for (int L = 0; L < D; ++L) {
            auto& P = prefixes[L];
            for (int64_t s = 0; s < n_leaves; ++s) {
                const int64_t l = order[s];
                if (leaf_dijk[4 * l] <= L) continue;
                const uint64_t p = code[l] >> (3 * (D - L));
                if (P.empty() || P.back() != p) P.push_back(p);
            }
            base[L + 1] = base[L] + (int64_t)P.size();
        }
        const int64_t n_nodes = base[D];
        *n_nodes_out = n_nodes;
        if (n_nodes > INT32_MAX) return fail(FPO_E_INVALID, "too many nodes");
        if (!children_out) return FPO_OK;
        if (cap_nodes < n_nodes) return fail(FPO_E_CAPACITY, "children_out holds fewer than n_nodes rows");
        auto node_id = [&](int L, uint64_t p) -> int64_t {
            const auto& P = prefixes[L];
            auto it = std::lower_bound(P.begin(), P.end(), p);
            return base[L] + (it - P.begin());
        };
        std::memset(children_out, 0, sizeof(int32_t) * 8 * (size_t)n_nodes);
        for (int L = 1; L < D; ++L)
            for (size_t n = 0; n < prefixes[L].size(); ++n) {
                const uint64_t p = prefixes[L][n];
                const int64_t parent = node_id(L - 1, p >> 3);
                children_out[parent * 8 + (p & 7)] = (int32_t)(base[L] + (int64_t)n);
            }
        for (int64_t s = 0; s < n_leaves; ++s) {
            const int64_t l = order[s];
            const int d = leaf_dijk[4 * l];
            const uint64_t p = code[l] >> (3 * (D - d));
            const int64_t parent = node_id(d - 1, p >> 3);
            children_out[parent * 8 + (p & 7)] = -(int32_t)(s + 1);
            if (perm_out) perm_out[s] = l;
        }
        return FPO_OK;
    } catch (const std::bad_alloc&) {
        return fail(FPO_E_NOMEM, "out of host memory");
    }
}

// Union leaves over Morton-sorted cells: a cell with no cell strictly inside
// it is a union leaf if some cell covers it (itself or an ancestor); else it
// splits into its eight children.
namespace {
struct Cell {
    uint64_t code;   // Morton code of the min corner on the finest lattice
    int32_t depth;
};

void union_rec(const std::vector<Cell>& cs, size_t a, size_t b, int d, uint64_t code, int D, bool covered,
               std::vector<Cell>& out)
{
    // cs[a, b): cells with code in [code, code + 8^(D-d)) and depth >= d
    while (a < b && cs[a].depth == d && cs[a].code == code) {
        covered = true;
        ++a;
    }
    if (a == b) {
        if (covered && d > 0) out.push_back({code, d});
        return;
    }
    const uint64_t child = uint64_t(1) << (3 * (D - d - 1));
    size_t lo = a;
    for (int o = 0; o < 8; ++o) {
        const uint64_t end = code + (uint64_t)(o + 1) * child;
        size_t hi = lo;
        while (hi < b && cs[hi].code < end) ++hi;
        union_rec(cs, lo, hi, d + 1, code + (uint64_t)o * child, D, covered, out);
        lo = hi;
    }
}

uint64_t compact3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> (3 * b)) & 1ull) << b;
    return r;
}
}  // namespace

extern "C" fpo_status fpo_union_leaves(const int32_t* leaf_dijk, int64_t n_cells, int32_t max_depth,
                                       int32_t* union_out, int64_t cap, int64_t* n_union_out)
{
    ApiRange api_range_("fpo_union_leaves");
    try {
        if (!leaf_dijk || !n_union_out) return fail(FPO_E_INVALID, "NULL argument");
        if (n_cells < 1) return fail(FPO_E_INVALID, "n_cells must be >= 1");
        if (max_depth < 1 || max_depth > FPO_MAX_DEPTH) return fail(FPO_E_INVALID, "max_depth must be in 1..10");
        const int D = max_depth;
        fault_point_alloc();
        std::vector<Cell> cs((size_t)n_cells);
        for (int64_t l = 0; l < n_cells; ++l) {
            const int32_t d = leaf_dijk[4 * l], i = leaf_dijk[4 * l + 1], j = leaf_dijk[4 * l + 2],
                          k = leaf_dijk[4 * l + 3];
            if (d < 1 || d > D) return fail(FPO_E_INVALID, "cell " + std::to_string(l) + ": depth out of range");
            const int64_t g = int64_t(1) << d;
            if (i < 0 || j < 0 || k < 0 || i >= g || j >= g || k >= g)
                return fail(FPO_E_INVALID, "cell " + std::to_string(l) + ": coordinate out of range");
            const int sh = D - d;
            cs[(size_t)l] = {spread3((uint64_t)i << sh) | (spread3((uint64_t)j << sh) << 1) | (spread3((uint64_t)k << sh) << 2), d};
        }
        std::sort(cs.begin(), cs.end(), [](const Cell& x, const Cell& y) {
            return x.code < y.code || (x.code == y.code && x.depth < y.depth);
        });
        std::vector<Cell> out;
        union_rec(cs, 0, cs.size(), 0, 0, D, false, out);
        *n_union_out = (int64_t)out.size();
        if (!union_out) return FPO_OK;
        if (cap < (int64_t)out.size()) return fail(FPO_E_CAPACITY, "union_out holds fewer than n_union rows");
        for (size_t u = 0; u < out.size(); ++u) {
            const int sh = D - out[u].depth;
            union_out[4 * u] = out[u].depth;
            union_out[4 * u + 1] = (int32_t)(compact3(out[u].code) >> sh);
            union_out[4 * u + 2] = (int32_t)(compact3(out[u].code >> 1) >> sh);
            union_out[4 * u + 3] = (int32_t)(compact3(out[u].code >> 2) >> sh);
        }
        return FPO_OK;
    } catch (const std::bad_alloc&) {
        return fail(FPO_E_NOMEM, "out of host memory");
    }
}

extern "C" fpo_status fpo_prune_leaves(const float* sigma_max, int64_t n_leaves, float threshold, int64_t* keep_out,
                                       int64_t* n_keep_out)
{
    ApiRange api_range_("fpo_prune_leaves");
    if (!sigma_max || !keep_out || !n_keep_out) return fail(FPO_E_INVALID, "NULL argument");
    if (n_leaves < 0) return fail(FPO_E_INVALID, "n_leaves < 0");
    if (!std::isfinite(threshold)) return fail(FPO_E_INVALID, "threshold must be finite");
    int64_t n = 0;
    for (int64_t l = 0; l < n_leaves; ++l)
        if (sigma_max[l] >= threshold) keep_out[n++] = l;
    *n_keep_out = n;
    return FPO_OK;
}

extern "C" fpo_status fpo_coarse_occupancy(const int32_t* leaf_dijk, int64_t n_leaves, int32_t max_depth,
                                           uint32_t* bits_out)
{
    ApiRange api_range_("fpo_coarse_occupancy");
    if (!leaf_dijk || !bits_out) return fail(FPO_E_INVALID, "NULL argument");
    if (n_leaves < 1) return fail(FPO_E_INVALID, "n_leaves must be >= 1");
    if (max_depth < 1 || max_depth > FPO_MAX_DEPTH) return fail(FPO_E_INVALID, "max_depth must be in 1..10");
    constexpr int N = FPO_COARSE_RES;   // 2^6 cells per axis
    constexpr int kLog = 6;
    for (int64_t l = 0; l < n_leaves; ++l) {
        const int32_t d = leaf_dijk[4 * l];
        if (d < 1 || d > max_depth) return fail(FPO_E_INVALID, "leaf " + std::to_string(l) + ": depth out of range");
        const int64_t g = int64_t(1) << d;
        for (int a = 1; a <= 3; ++a)
            if (leaf_dijk[4 * l + a] < 0 || leaf_dijk[4 * l + a] >= g)
                return fail(FPO_E_INVALID, "leaf " + std::to_string(l) + ": coordinate out of range");
    }
    std::vector<uint8_t> occ;
    try {
        fault_point_alloc();
        occ.assign((size_t)N * N * N, 0);
    } catch (const std::bad_alloc&) {
        return fail(FPO_E_NOMEM, "out of host memory");
    }
    for (int64_t l = 0; l < n_leaves; ++l) {
        const int d = leaf_dijk[4 * l];
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            const int64_t v = leaf_dijk[4 * l + 1 + a];
            if (d >= kLog) {
                lo[a] = hi[a] = (int)(v >> (d - kLog));
            } else {
                lo[a] = (int)(v << (kLog - d));
                hi[a] = lo[a] + (1 << (kLog - d)) - 1;
            }
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) occ[((size_t)z * N + y) * N + x] = 1;
    }
    std::memset(bits_out, 0, sizeof(uint32_t) * FPO_COARSE_WORDS);
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                bool any = false;
                for (int dz = -1; dz <= 1 && !any; ++dz)
                    for (int dy = -1; dy <= 1 && !any; ++dy)
                        for (int dx = -1; dx <= 1 && !any; ++dx) {
                            const int X = x + dx, Y = y + dy, Z = z + dz;
                            if (X < 0 || Y < 0 || Z < 0 || X >= N || Y >= N || Z >= N) continue;
                            any = occ[((size_t)Z * N + Y) * N + X] != 0;
                        }
                if (any) {
                    const int idx = (z * N + y) * N + x;
                    bits_out[idx >> 5] |= 1u << (idx & 31);
                }
            }
    return FPO_OK;
}

extern "C" fpo_status fpo_time_basis(const double* times, int32_t n_t, const fpo_layout* layout, float* basis_out)
{
    ApiRange api_range_("fpo_time_basis");
    if (!times || !layout || !basis_out) return fail(FPO_E_INVALID, "NULL argument");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (layout->n_sigma < 1 || layout->n_sigma > FPO_BASIS_STRIDE || layout->n_sh_fourier > layout->n_sigma)
        return fail(FPO_E_INVALID, "layout sizes out of range");
    if (!(layout->period > 0.0f)) return fail(FPO_E_INVALID, "layout.period must be > 0");
    for (int32_t r = 0; r < n_t; ++r)
        if (!std::isfinite(times[r])) return fail(FPO_E_INVALID, "times must be finite");
    for (int32_t r = 0; r < n_t; ++r)
        basis_row(times[r], (double)layout->period, layout->n_sigma, basis_out + (int64_t)r * FPO_BASIS_STRIDE);
    return FPO_OK;
}

extern "C" fpo_status fpo_camera_pack(const fpo_camera* cams, int32_t n_cams, float* table_out)
{
    ApiRange api_range_("fpo_camera_pack");
    if (!cams || !table_out) return fail(FPO_E_INVALID, "NULL argument");
    if (n_cams < 1) return fail(FPO_E_INVALID, "n_cams must be >= 1");
    for (int32_t c = 0; c < n_cams; ++c) {
        float fr[12];
        fpo_status st = camera_frame(cams[c], fr);
        if (st != FPO_OK) return st;
        float* row = table_out + (int64_t)c * FPO_CAMERA_FLOATS;
        for (int q = 0; q < 12; ++q) row[q] = fr[q];
        row[12] = (float)cams[c].width;
        row[13] = (float)cams[c].height;
        row[14] = 0.0f;
        row[15] = 0.0f;
    }
    return FPO_OK;
}
