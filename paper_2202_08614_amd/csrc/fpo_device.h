// Device-side building blocks of libfpo (gfx950): ray set-up, the sparse
// octree walk, leaf-record coefficient gathers, the per-leaf inverse real
// Fourier transform (Eq. 7, 9), the SH colour (Eq. 1) and front-to-back
// compositing.  Shared by the render, trace and backward kernels so that all
// three walk exactly the same segments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpo.h"

namespace fpo {
namespace dev {

constexpr int kBlock = 256;          // threads per block: 4 wave64
constexpr int kWave = 64;
constexpr int kStackLevels = FPO_MAX_DEPTH;

// Plain-old-data view of a tree, passed by value to kernels.
struct TreeDev {
    const int32_t* children;
    const uint4* recs;      // leaf records: R 16-byte words per leaf slot
    const float* scale;     // per-leaf scale for quantised stores
    int64_t stride;         // leaf slots (leaf_stride)
    int32_t n_nodes;
    int32_t n_leaves;
    int32_t max_depth;
    float sigma_scale;
    const int2* gc;         // two-level table [n_gc][64] (children, grandchild), or null
    int32_t n_gc;           // rows of gc (0 without one)
    float box_lo[3], box_hi[3];   // the leaves' bounds in cube units (default: the unit cube)
};

// Host helper: the kernel-side view of a validated fpo_tree_view.
inline TreeDev tree_dev(const fpo_tree_view* t)
{
    TreeDev d;
    d.children = t->children;
    d.gc = reinterpret_cast<const int2*>(t->grandchildren);
    d.n_gc = t->grandchildren ? (int32_t)t->n_grandchild_rows : 0;
    d.recs = static_cast<const uint4*>(t->coeffs);
    d.scale = t->leaf_scale;
    d.stride = t->leaf_stride;
    d.n_nodes = (int32_t)t->n_nodes;
    d.n_leaves = (int32_t)t->n_leaves;
    d.max_depth = t->max_depth;
    d.sigma_scale = t->layout.sigma_scale;
    // lattice bounds / 2^max_depth: exact in FP32
    const float cell = 1.0f / (float)(1 << t->max_depth);
    for (int a = 0; a < 3; ++a) {
        d.box_lo[a] = t->bounds ? (float)t->bounds[a] * cell : 0.0f;
        d.box_hi[a] = t->bounds ? (float)t->bounds[3 + a] * cell : 1.0f;
    }
    return d;
}

// --------------------------------------------------------------------------
// Coefficient words.  W coefficients per 16-byte word; R words per leaf
// record (a multiple of 128 bytes, so that a record starts a cache line and
// the words holding the 31 density coefficients share one line).
// --------------------------------------------------------------------------
template <int DT> struct Pack;

template <> struct Pack<FPO_F32> {
    static constexpr int W = 4;
    static constexpr int R = 48;
    __device__ static inline void unpack(const uint4& w, float* o)
    {
        o[0] = __uint_as_float(w.x); o[1] = __uint_as_float(w.y);
        o[2] = __uint_as_float(w.z); o[3] = __uint_as_float(w.w);
    }
};

template <> struct Pack<FPO_BF16> {
    static constexpr int W = 8;
    static constexpr int R = 24;
    __device__ static inline void unpack(const uint4& w, float* o)
    {
        const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(v[i] << 16);
            o[2 * i + 1] = __uint_as_float(v[i] & 0xFFFF0000u);
        }
    }
};

// OCP E4M3FN byte -> FP32.  Placing the 7 magnitude bits at bit 20 gives an
// FP32 whose value is 2^(e-127) (1 + m/8) for e >= 1 and the FP32 subnormal
// 2^-126 (m/8) for e = 0; scaling by 2^120 maps both onto 2^(e-7)(1 + m/8)
// and 2^-6 (m/8), the E4M3 normal and subnormal values.
__device__ inline float e4m3_to_f32(uint32_t byte)
{
    const uint32_t bits = ((byte & 0x7Fu) << 20) | ((byte & 0x80u) << 24);
    return __uint_as_float(bits) * 0x1p120f;
}

template <> struct Pack<FPO_FP8_E4M3> {
    static constexpr int W = 16;
    static constexpr int R = 16;
    __device__ static inline void unpack(const uint4& w, float* o)
    {
        const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int b = 0; b < 4; ++b) o[4 * i + b] = e4m3_to_f32((v[i] >> (8 * b)) & 0xFFu);
    }
};

// --------------------------------------------------------------------------
// Real spherical harmonics of degree <= 2 (Eq. 1): orthonormal, Condon-Shortley
// phase, index j = l^2 + l + m.  Constants: Y00 = 1/(2 sqrt(pi)),
// Y1m = sqrt(3/(4 pi)), Y2{-2,-1,1} = sqrt(15/pi)/2, Y20 = sqrt(5/pi)/4,
// Y22 = sqrt(15/pi)/4.
// --------------------------------------------------------------------------
__device__ inline void sh9(float x, float y, float z, float* Y)
{
    const float c0 = 0.28209479177387814f;
    const float c1 = 0.48860251190291992f;
    const float c2 = 1.09254843059207907f;
    const float c20 = 0.31539156525252005f;
    const float c22 = 0.54627421529603953f;
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2 * x * y;
    Y[5] = -c2 * y * z;
    Y[6] = c20 * (3.0f * z * z - 1.0f);
    Y[7] = -c2 * x * z;
    Y[8] = c22 * (x * x - y * y);
}

// --------------------------------------------------------------------------
// Ray set-up: normalise d, clip against the unit cube, re-base the origin at
// the entry point so that distances along the ray stay small.
// --------------------------------------------------------------------------
struct Ray {
    float o[3];     // entry point (origin + t_in d)
    float d[3];     // unit direction
    float inv[3];   // 1 / d (unused where d == 0)
    float t_in;     // distance from the caller's origin to the entry point
    float t_len;    // length inside the cube
};

// Clip the ray to the box [lo, hi] (cube units) instead of the unit cube:
// the entry point is then on the box's face and t_len the chord inside it.
__host__ __device__ inline bool setup_ray_in(const float* lo_b, const float* hi_b, float ox, float oy, float oz,
                                             float dx, float dy, float dz, Ray& r)
{
    const float n2 = dx * dx + dy * dy + dz * dz;
    if (!(n2 > 0.0f)) return false;
    const float inv_n = 1.0f / sqrtf(n2);
    const float o[3] = {ox, oy, oz};
    const float d[3] = {dx * inv_n, dy * inv_n, dz * inv_n};
    float lo = 0.0f, hi = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.d[a] = d[a];
        if (d[a] == 0.0f) {
            r.inv[a] = 0.0f;
            if (o[a] < lo_b[a] || o[a] > hi_b[a]) return false;
            continue;
        }
        const float inv = 1.0f / d[a];
        r.inv[a] = inv;
        float t1 = (lo_b[a] - o[a]) * inv;
        float t2 = (hi_b[a] - o[a]) * inv;
        if (t1 > t2) { const float s = t1; t1 = t2; t2 = s; }
        lo = fmaxf(lo, t1);
        hi = fminf(hi, t2);
    }
    if (!(lo < hi)) return false;
    r.t_in = lo;
    r.t_len = hi - lo;
#pragma unroll
    for (int a = 0; a < 3; ++a) r.o[a] = fmaf(lo, d[a], o[a]);
    return true;
}

__host__ __device__ inline bool setup_ray(float ox, float oy, float oz, float dx, float dy, float dz, Ray& r)
{
    const float lo_b[3] = {0.0f, 0.0f, 0.0f}, hi_b[3] = {1.0f, 1.0f, 1.0f};
    return setup_ray_in(lo_b, hi_b, ox, oy, oz, dx, dy, dz, r);
}

// --------------------------------------------------------------------------
// Sparse octree walk.
//
// Every axis the ray runs down is mirrored (lattice coordinate x -> G - x,
// octant bit flipped), so that in the walk's frame all direction components
// are >= 0 and a cell is always left through its upper faces.  The walk keeps
// the chain of internal nodes above the current cell, each with the octant of
// its child the ray is in (a per-lane stack in LDS), and the cell's corner on
// the finest lattice (G = 2^D cells per axis), held as exact small integers in
// FP32 so that a plane's crossing time (p - x) k needs no conversion.
// One iteration:
//   - descend while the current slot holds an internal node: the ray's cell
//     on the finest lattice at t_cur (x + t_cur / k per axis, clamped into
//     the slot) is found once, and each level's octant is one bit of it per
//     axis; from a node the two-level table covers, one read gives both the
//     child's and the grandchild's entries;
//   - report a leaf segment [t_cur, t_exit), t_exit the first upper face the
//     ray reaches (ties x < y < z);
//   - step to the neighbouring slot of the same size across that face (the
//     other coordinates are unchanged): a sibling in the same node flips one
//     octant bit; otherwise pop to the deepest node that still contains it,
//     found from the highest bit the step changed, whose stacked octant flips
//     the same bit.
// The step and the load of the next slot's child-table entry come before the
// current leaf is shaded (they do not depend on it), so that load and the
// leaf's own loads are in flight together.
// Each step moves the exit axis forward by a whole slot and never moves any
// axis back, so the walk ends within 3G steps.  Rays parallel to an axis use a
// tiny direction instead of zero: their crossing times on that axis exceed
// any chord.
//
// Visitor: bool segment(int leaf, float t0, float t1) returns true to stop.
// Distances are measured from the entry point r.o.  With a stop distance
// t_end the walk consults stop.more() once a step ends at or past t_end.
// --------------------------------------------------------------------------
// Visitors that load a leaf's data may start the loads as soon as the walk
// knows the leaf, before it works out the step to the next slot.
template <class Visitor>
__device__ inline void prefetch_leaf(Visitor&, int) {}

struct NoStop {
    __device__ inline bool more(float, float&) { return false; }
};

// TWO: descend through the two-level table where the tree has one (the
// snapshot camera renders; elsewhere the extra registers cost occupancy).
template <bool TWO = false, int STRIDE = kBlock, class Visitor, class Stop>
__device__ inline void walk(const TreeDev& T, const Ray& r, int* stk, Visitor& vis, float t_end, Stop& stop)
{
    // The child table is read through a buffer resource: 32-bit byte offsets
    // (no 64-bit address arithmetic per step), and a read past the table
    // returns 0 (an empty slot).
    const __amdgpu_buffer_rsrc_t ct =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(T.children), (short)0, T.n_nodes * 32, 0x00020000);
    // the two-level table, 512 bytes per row (absent: no rows, never read)
    const __amdgpu_buffer_rsrc_t gt =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<int2*>(T.gc), (short)0, T.n_gc * 512, 0x00020000);
    const int D = T.max_depth;
    const int G = 1 << D;
    const float fG = (float)G;
    int mirror = 0;
    float xf[3], k[3];   // entry point in (mirrored) lattice units; time per lattice unit
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool neg = r.d[a] < 0.0f;
        mirror |= (neg ? 1 : 0) << a;
        const float da = fmaxf(fabsf(r.d[a]), 1e-20f);
        k[a] = 1.0f / (da * fG);
        const float p = r.o[a] * fG;
        xf[a] = neg ? fG - p : p;
    }
    // current slot: table entry `no` = (node << 3) | octant of the child table,
    // corner pos (mirrored lattice, exact in FP32), edge 2^csh; each stacked
    // entry is kept under the edge exponent of its child slot
    int csh = D - 1;
    float t_cur = 0.0f;
    float pos[3];
    int no = 0;
    {
        const float half = (float)(G >> 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool up = (half - xf[a]) * k[a] <= t_cur;
            pos[a] = up ? half : 0.0f;
            no |= (up ? 1 : 0) << a;
        }
    }
    no ^= mirror;
    int ch_next = __builtin_amdgcn_raw_buffer_load_b32(ct, no * 4, 0, 0);
    const int max_steps = 3 * G + 4;
    for (int it = 0; it < max_steps; ++it) {
        int ch = ch_next;
        if (ch > 0 && ch < T.n_nodes && csh > 0) {
            // The finest-lattice cell q the ray is in at t_cur (mirrored
            // frame), clamped into the current slot: every level below takes
            // its octant from one bit of q per axis.  A point that rounds
            // across an inner plane only moves the walk by a zero-length
            // segment or a sliver of one.
            int q[3];
            {
                const float top = __builtin_ldexpf(1.0f, csh) - 1.0f;
                const float tg = t_cur * fG;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    q[a] = (int)__builtin_amdgcn_fmed3f(fmaf(tg, fabsf(r.d[a]), xf[a]), pos[a], pos[a] + top);
            }
            do {
                stk[csh * STRIDE] = no;    // the node and the child the ray is in
                csh -= 1;
                const int bits = (__builtin_amdgcn_ubfe(q[0], csh, 1) | (__builtin_amdgcn_ubfe(q[1], csh, 1) << 1) |
                                  (__builtin_amdgcn_ubfe(q[2], csh, 1) << 2)) ^ mirror;
                if (TWO && ch < T.n_gc && csh > 0) {
                    // two levels in one read: (child entry, grandchild entry)
                    const int b2 = (__builtin_amdgcn_ubfe(q[0], csh - 1, 1) |
                                    (__builtin_amdgcn_ubfe(q[1], csh - 1, 1) << 1) |
                                    (__builtin_amdgcn_ubfe(q[2], csh - 1, 1) << 2)) ^ mirror;
                    const auto e = __builtin_amdgcn_raw_buffer_load_b64(gt, (ch * 64 + bits * 8 + b2) * 8, 0, 0);
                    no = (ch << 3) | bits;
                    ch = e[0];
                    if (ch > 0 && ch < T.n_nodes) {
                        stk[csh * STRIDE] = no;
                        csh -= 1;
                        no = (ch << 3) | b2;
                        ch = e[1];
                    }
                } else {
                    no = (ch << 3) | bits;
                    ch = __builtin_amdgcn_raw_buffer_load_b32(ct, no * 4, 0, 0);
                }
            } while (ch > 0 && ch < T.n_nodes && csh > 0);
            const int m = -1 << csh;
#pragma unroll
            for (int a = 0; a < 3; ++a) pos[a] = (float)(q[a] & m);
        }
        if (ch > 0) ch = 0;   // malformed table or past the deepest level: treat as empty
        const float sz = __builtin_ldexpf(1.0f, csh);
        float te[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) te[a] = (pos[a] + sz - xf[a]) * k[a];
        int ax = 0;
        float t_exit = te[0];
        if (te[1] < t_exit) { t_exit = te[1]; ax = 1; }
        if (te[2] < t_exit) { t_exit = te[2]; ax = 2; }
        t_exit = fmaxf(t_exit, t_cur);
        if (ch < 0 && -ch - 1 < T.n_leaves) prefetch_leaf(vis, -ch - 1);
        // step to the next slot and request its entry before shading this one
        const float old = ax == 0 ? pos[0] : ax == 1 ? pos[1] : pos[2];
        const float nwf = old + sz;
        const bool more = nwf < fG;
        if (more) {
            pos[0] = ax == 0 ? nwf : pos[0];
            pos[1] = ax == 1 ? nwf : pos[1];
            pos[2] = ax == 2 ? nwf : pos[2];
            // highest bit the step changes: csh plus the run of ones above it in the old corner
            const int h = csh + __builtin_ctz(~((int)old >> csh));
            if (h > csh) {
                // pop to the deepest node that contains the new slot (stacked under the slot size h)
                csh = h;
                no = stk[h * STRIDE] ^ (1 << ax);
#pragma unroll
                for (int a = 0; a < 3; ++a) pos[a] = __builtin_ldexpf(floorf(__builtin_ldexpf(pos[a], -h)), h);
            } else {
                no ^= 1 << ax;
            }
            ch_next = __builtin_amdgcn_raw_buffer_load_b32(ct, no * 4, 0, 0);
        }
        if (ch < 0) {
            const int leaf = -ch - 1;
            if (leaf < T.n_leaves && vis.segment(leaf, t_cur, t_exit)) return;
        }
        if (t_exit >= t_end && !stop.more(t_exit, t_end)) return;
        if (!more) return;
        t_cur = t_exit;
    }
}

template <bool TWO = false, int STRIDE = kBlock, class Visitor>
__device__ inline void walk(const TreeDev& T, const Ray& r, int* stk, Visitor& vis)
{
    NoStop ns;
    walk<TWO, STRIDE>(T, r, stk, vis, __builtin_inff(), ns);
}

// Record geometry of a coefficient layout (n1 density terms, n2 terms per SH
// coefficient): words per record rounded up to whole 128-byte lines.  The
// default layout (31, 5) gives Pack<DT>::R.
template <int DT, int N1, int N2>
struct Rec {
    static constexpr int W = Pack<DT>::W;
    static constexpr int kCoeff = N1 + 3 * FPO_N_SH * N2;
    static constexpr int R = ((kCoeff + W - 1) / W + 7) / 8 * 8;
};
static_assert(Rec<FPO_F32, FPO_N_SIGMA, FPO_N_SH_FOURIER>::R == Pack<FPO_F32>::R, "F32 record");
static_assert(Rec<FPO_BF16, FPO_N_SIGMA, FPO_N_SH_FOURIER>::R == Pack<FPO_BF16>::R, "BF16 record");
static_assert(Rec<FPO_FP8_E4M3, FPO_N_SIGMA, FPO_N_SH_FOURIER>::R == Pack<FPO_FP8_E4M3>::R, "FP8 record");

// --------------------------------------------------------------------------
// Leaf evaluation at time t (Eq. 7 and Eq. 9): sigma_raw = sum_{i<n1} k^sigma_i
// b_i and h_c = sum_j z_{c,j} Y_j with z_{c,j} = sum_{i<n2} k^z_{c,j,i} b_i.
// ----------------------------------------------------------------------------
template <int DT, int N1 = FPO_N_SIGMA, int N2 = FPO_N_SH_FOURIER>
struct LeafEval {
    static constexpr int W = Pack<DT>::W;
    static constexpr int R = Rec<DT, N1, N2>::R;
    static constexpr int kSigmaWords = (N1 + 1 + W - 1) / W;   // words holding q <= n1
    static constexpr int kWords = (Rec<DT, N1, N2>::kCoeff + W - 1) / W;

    // Loads the words holding q <= n1 and returns sigma_raw (scaled for
    // quantised stores).  `k` keeps the unpacked values for colour().
    __device__ static inline float sigma(const TreeDev& T, int leaf, const float* b, float* k, float& scale)
    {
        const uint4* P = T.recs + (int64_t)leaf * R;
#pragma unroll
        for (int g = 0; g < kSigmaWords; ++g) {
            const uint4 w = P[g];
            Pack<DT>::unpack(w, k + g * W);
        }
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < N1; ++q) s = fmaf(k[q], b[q], s);
        scale = (DT == FPO_F32) ? 1.0f : T.scale[leaf];
        return s * scale;
    }

    // Colour pre-activations h[3]; k holds the first kSigmaWords words.
    __device__ static inline void colour(const TreeDev& T, int leaf, const float* b, const float* Y,
                                         const float* k, float scale, float* h)
    {
        const uint4* P = T.recs + (int64_t)leaf * R;
        float kz[(kWords - kSigmaWords + 1) * W];
        // coefficient q >= n1 lives at kz[q - n1 + off]
        constexpr int off = N1 - (kSigmaWords - 1) * W;   // index of q = n1 inside the last sigma word
#pragma unroll
        for (int e = 0; e < W; ++e) kz[e] = k[(kSigmaWords - 1) * W + e];
#pragma unroll
        for (int g = kSigmaWords; g < kWords; ++g) {
            const uint4 w = P[g];
            Pack<DT>::unpack(w, kz + (g - kSigmaWords + 1) * W);
        }
        h[0] = h[1] = h[2] = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < FPO_N_SH; ++j) {
                const int base = off + (c * FPO_N_SH + j) * N2;
                float z = 0.0f;
#pragma unroll
                for (int i = 0; i < N2; ++i) z = fmaf(kz[base + i], b[i], z);
                h[c] = fmaf(z, Y[j], h[c]);
            }
        h[0] *= scale; h[1] *= scale; h[2] *= scale;
    }
};

__device__ inline float sigmoidf_(float h) { return __builtin_amdgcn_rcpf(1.0f + __expf(-h)); }

// Snapshot records: 32 values per leaf slot (row 0 = sigma(t) before
// activation, rows 1 + c*9 + j = z_{c,j}(t), rows 28..31 zero), F32 (8 words,
// 128 bytes) or BF16 (4 words, 64 bytes).
template <int SDT>
struct SnapEval {
    static constexpr int W = Pack<SDT>::W;      // values per word: 4 or 8
    static constexpr int R = 32 / W;            // words per record: 8 or 4
    __device__ static inline float sigma(const void* S, int leaf, float* v)
    {
        const uint4 w = static_cast<const uint4*>(S)[(int64_t)leaf * R];
        Pack<SDT>::unpack(w, v);
        return v[0];
    }
    __device__ static inline void colour(const void* S, int leaf, const float* Y, float* v, float* h)
    {
        const uint4* P = static_cast<const uint4*>(S) + (int64_t)leaf * R;
#pragma unroll
        for (int g = 1; g < R; ++g) Pack<SDT>::unpack(P[g], v + g * W);
        dot(v, Y, h);
    }
    // The same reads through a buffer resource over the snapshot (records
    // within 4 GiB): one 32-bit offset per lane instead of a 64-bit address,
    // which keeps the camera render within 64 VGPRs (8 waves per SIMD).
    __device__ static inline uint4 word(__amdgpu_buffer_rsrc_t rs, int leaf, int g)
    {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, (uint32_t)leaf * (R * 16) + g * 16, 0, 0);
        return make_uint4(x[0], x[1], x[2], x[3]);
    }
    __device__ static inline float sigma(__amdgpu_buffer_rsrc_t rs, int leaf, float* v)
    {
        Pack<SDT>::unpack(word(rs, leaf, 0), v);
        return v[0];
    }
    __device__ static inline void colour(__amdgpu_buffer_rsrc_t rs, int leaf, const float* Y, float* v, float* h)
    {
#pragma unroll
        for (int g = 1; g < R; ++g) Pack<SDT>::unpack(word(rs, leaf, g), v + g * W);
        dot(v, Y, h);
    }
    __device__ static inline void dot(const float* v, const float* Y, float* h)
    {
        h[0] = h[1] = h[2] = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < FPO_N_SH; ++j) h[c] = fmaf(v[1 + c * FPO_N_SH + j], Y[j], h[c]);
    }
};

// --------------------------------------------------------------------------
// Front-to-back compositing visitor.  MODE: a coefficient dtype (Fourier
// mode) or 16 + snapshot dtype (snapshot mode).
// --------------------------------------------------------------------------
constexpr int kSnapF32 = 16 + FPO_F32;
constexpr int kSnapBF16 = 16 + FPO_BF16;

template <int MODE, int N1 = FPO_N_SIGMA, int N2 = FPO_N_SH_FOURIER, bool BUF = false>
struct Shade {
    const TreeDev& T;
    const float* b;       // basis row (Fourier mode)
    const void* snap;     // snapshot records (snapshot mode)
    __amdgpu_buffer_rsrc_t srs;   // BUF: the same records through a buffer resource
    float Y[9];
    float Tr;             // transmittance
    float C[3];
    float stop_T;

    __device__ inline bool segment(int leaf, float t0, float t1)
    {
        const float delta = t1 - t0;
        float h[3];
        if constexpr (MODE >= 16) {
            // only the optical depth sigma_eff * delta stays live through the
            // colour reads (the 64-VGPR budget of the snapshot render)
            constexpr int SDT = MODE - 16;
            float v[32];
            float sraw;
            if constexpr (BUF) sraw = SnapEval<SDT>::sigma(srs, leaf, v);
            else sraw = SnapEval<SDT>::sigma(snap, leaf, v);
            const float od = T.sigma_scale * fmaxf(sraw, 0.0f) * delta;
            if (!(od > 0.0f)) return false;
            if constexpr (BUF) SnapEval<SDT>::colour(srs, leaf, Y, v, h);
            else SnapEval<SDT>::colour(snap, leaf, Y, v, h);
            return composite(__expf(-od), h);
        } else {
            using E = LeafEval<MODE, N1, N2>;
            float k[E::kSigmaWords * E::W];
            float scale;
            const float sraw = E::sigma(T, leaf, b, k, scale);
            const float sig = T.sigma_scale * fmaxf(sraw, 0.0f);
            if (!(sig * delta > 0.0f)) return false;   // transparent: contributes nothing
            E::colour(T, leaf, b, Y, k, scale, h);
            return composite(__expf(-sig * delta), h);
        }
    }

    // Front-to-back compositing of a segment of transmittance e and SH sums h;
    // true once the ray's transmittance is below stop_T.
    __device__ inline bool composite(float e, const float* h)
    {
        const float w = Tr * (1.0f - e);
#pragma unroll
        for (int c = 0; c < 3; ++c) C[c] = fmaf(w, sigmoidf_(h[c]), C[c]);
        Tr *= e;
        return Tr < stop_T;
    }
};

// --------------------------------------------------------------------------
// One ray per wave, for small ray batches and the backward: a fine-tuning
// batch of a few thousand rays fills only a few dozen wave slots at one ray
// per lane, and one lane scattering 166 gradients per sample is bound by the
// number of lines its atomics touch.  All
// 64 lanes walk the same ray (uniform branches, broadcast child loads).  The
// 166 F32 coefficients of a leaf are spread over the lanes, lane l holding
// q = l, l + 64, l + 128, so a record is read (and a gradient record
// written) with three coalesced accesses, and the dot products of Eq. 7 and
// Eq. 9 with the SH sums of Eq. 1 become wave sums.
// --------------------------------------------------------------------------

// fpo_render_rays runs batches of at most this many rays one ray per wave (F32
// Fourier mode); above it one ray per lane fills the machine and is faster.
// The backward always runs one ray per wave: its coalesced gradient writes
// beat one ray per lane at every batch size.
constexpr int64_t kWaveRayBatch = 32768;

// Sum over the wave.  Within each row of 16 lanes, four DPP steps add lane
// pairs, quads, half rows and rows (every lane adds the same two partial sums,
// a + b and b + a being equal in IEEE arithmetic, so the row's lanes agree);
// the four row sums are then read into scalar registers and added in one
// fixed order.  All lanes hold the same bits, branches on the result stay
// uniform, and no step goes through LDS.
template <int CTRL>
__device__ inline float dpp_add(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ inline float wave_sum(float v)
{
    v = dpp_add<0xb1>(v);     // quad_perm [1, 0, 3, 2]: pairs
    v = dpp_add<0x4e>(v);     // quad_perm [2, 3, 0, 1]: quads
    v = dpp_add<0x141>(v);    // row_half_mirror: half rows
    v = dpp_add<0x140>(v);    // row_mirror: rows
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return (r0 + r1) + (r2 + r3);
}

// This lane's coefficient slots for one ray: q = lane + 64 s, s < 3.  A
// density slot (q < 31) weighs b_q; an SH slot q = 31 + (9 c + j) 5 + i
// weighs Y_j b_i and feeds channel c.
struct WaveSlots {
    float w[3];
    int c[3];        // channel of an SH slot, -1 density, -2 past the 166 coefficients
    __device__ inline void init(int lane, const float* brow, const float* Y)
    {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int q = lane + kWave * s;
            if (q >= FPO_N_COEFF) {
                w[s] = 0.0f;
                c[s] = -2;
            } else if (q < FPO_N_SIGMA) {
                w[s] = brow[q];
                c[s] = -1;
            } else {
                const int u = q - FPO_N_SIGMA;
                const int ch = u / (FPO_N_SH * FPO_N_SH_FOURIER);
                const int rem = u - ch * (FPO_N_SH * FPO_N_SH_FOURIER);
                const int j = rem / FPO_N_SH_FOURIER;
                const int i = rem - j * FPO_N_SH_FOURIER;
                float yj = Y[0];
#pragma unroll
                for (int jj = 1; jj < FPO_N_SH; ++jj) yj = j == jj ? Y[jj] : yj;
                w[s] = yj * brow[i];
                c[s] = ch;
            }
        }
    }
};

// Fourier-mode F32 shading of one ray by a whole wave.  GRAD = false
// composites front to back (C, Tr).  GRAD = true recomputes the same walk and
// scatters dL/dk: with C the colour accumulated so far, Cf the forward
// pass's final colour and g = dL/dCf,
//     dL/dsigma_i = delta_i s sum_c g_c (T_{i+1} col_c - (Cf_c - C_c)),
//     dL/dh_c     = g_c T_i alpha_i col_c (1 - col_c),
// then dL/dk = dL/dsigma b_q (density) or dL/dh_c Y_j b_i (SH).
//
// Segment records (REC, forward only): every segment with positive optical
// depth is written as {leaf, delta, T_i, C_i[3]} (C_i the colour accumulated
// before it), 32 bytes, so that the backward can treat the ray's segments
// independently of each other.
template <bool GRAD, bool REC = false>
struct WaveShade {
    static_assert(!(GRAD && REC), "segment records are written by the forward");
    const TreeDev& T;
    WaveSlots sl;
    int lane;
    float Tr;
    float C[3];
    float stop_T;
    float Cf[3];          // GRAD only
    float g[3];           // GRAD only
    float* grad;          // GRAD only: F32 leaf records, 192 floats per slot
    float4* rec;          // REC: this ray's segment records
    int rec_cap;
    int rec_n;
    float pk[3];          // this lane's coefficients of the leaf being shaded

    // Load this lane's three coefficients of a leaf (all three before the
    // density sum decides whether the colour is needed: one memory round trip
    // per segment instead of two).
    __device__ inline void prefetch(int leaf)
    {
        constexpr int kRecFloats = 4 * Pack<FPO_F32>::R;
        const float* rc = reinterpret_cast<const float*>(T.recs) + (int64_t)leaf * kRecFloats + lane;
        pk[0] = rc[0];
        pk[1] = rc[kWave];
        pk[2] = sl.c[2] >= 0 ? rc[2 * kWave] : 0.0f;
    }

    // One segment entered with transmittance Tr_in after colour A (updated in
    // place), its coefficients loaded by prefetch(leaf).  Returns false for a
    // transparent segment (nothing to do); otherwise e = exp(-sigma delta).
    __device__ inline bool shade(int leaf, float delta, float Tr_in, float* A, float& e)
    {
        constexpr int kRecFloats = 4 * Pack<FPO_F32>::R;
        const float k[3] = {pk[0], pk[1], pk[2]};
        const float sraw = wave_sum(sl.c[0] == -1 ? sl.w[0] * k[0] : 0.0f);
        const float sig = T.sigma_scale * fmaxf(sraw, 0.0f);
        if (!(sig * delta > 0.0f)) return false;   // transparent: contributes nothing
        float h[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) h[ch] = fmaf(sl.c[s] == ch ? sl.w[s] : 0.0f, k[s], h[ch]);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) h[ch] = wave_sum(h[ch]);
        e = __expf(-sig * delta);
        const float w = Tr_in * (1.0f - e);
        if constexpr (!GRAD) {
            if constexpr (REC) {
                if (lane == 0 && rec_n < rec_cap) {
                    rec[2 * rec_n] = make_float4(__int_as_float(leaf), delta, Tr_in, A[0]);
                    rec[2 * rec_n + 1] = make_float4(A[1], A[2], 0.0f, 0.0f);
                }
                ++rec_n;
            }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) A[ch] = fmaf(w, sigmoidf_(h[ch]), A[ch]);
        } else {
            const float T_next = Tr_in * e;
            float dsig = 0.0f, dh[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float col = sigmoidf_(h[ch]);
                A[ch] = fmaf(w, col, A[ch]);
                dsig = fmaf(g[ch], T_next * col - (Cf[ch] - A[ch]), dsig);
                dh[ch] = g[ch] * w * col * (1.0f - col);
            }
            dsig *= delta * T.sigma_scale;    // sigma_raw > 0 here
            float* gr = grad + (int64_t)leaf * kRecFloats + lane;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int ch = sl.c[s];
                if (ch == -2) continue;
                const float dv = ch == -1 ? dsig : ch == 0 ? dh[0] : ch == 1 ? dh[1] : dh[2];
                unsafeAtomicAdd(gr + kWave * s, dv * sl.w[s]);
            }
        }
        return true;
    }

    __device__ inline bool segment(int leaf, float t0, float t1)
    {
        float e;
        if (!shade(leaf, t1 - t0, Tr, C, e)) return false;
        Tr *= e;
        return Tr < stop_T;
    }
};

template <bool GRAD, bool REC>
__device__ inline void prefetch_leaf(WaveShade<GRAD, REC>& v, int leaf)
{
    v.prefetch(leaf);
}

}  // namespace dev
}  // namespace fpo
