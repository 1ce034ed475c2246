// libfpo render entry points: camera renders, ray renders, traces, camera
// ray generation and coefficient packing (gfx950).
//
// Work mapping for camera renders: one wave64 renders an 8x8 pixel tile, a
// 256-thread block a 16x16 tile.  Blocks are dispatched round-robin over the
// 8 XCDs of the MI355X (each with its own L2); the block-to-tile map hands
// each XCD a contiguous band of tiles so that neighbouring rays, which cross
// the same leaves, share one L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"
#include "fpo_proposal.h"

namespace fpo {
namespace dev {

constexpr int kCamsPerLaunch = 16;
// Camera kernel blocks: cam_waves(mode) waves of 8x8 pixels, over a 16x16
// tile (4 waves, snapshot modes) or one 8x8 tile (1 wave, Fourier modes).
// The Fourier kernels hold 94 or more VGPRs (at most 5 waves per SIMD), and
// one-wave blocks let a finished wave's slot take the next block at once:
// 2.4% (1.9% with two launches in flight) per launch; the snapshot kernel
// (64 VGPRs) was 1.9% slower so.
constexpr int cam_waves(int mode) { return mode >= 16 ? 4 : 1; }
constexpr int cam_tile_w(int waves) { return waves >= 2 ? 16 : 8; }
constexpr int cam_tile_h(int waves) { return waves >= 4 ? 16 : 8; }

struct CamDev {
    float frame[12];                 // eye, forward, right * tan_x, up * tan_y
    float basis[FPO_BASIS_STRIDE];   // Eq. 8 at the camera's time
    const void* snap;                // snapshot planes for this camera (snapshot mode)
};

struct CamLaunch {
    TreeDev tree;
    CamDev cam[kCamsPerLaunch];
    float* rgb;                      // [n_cams][H][W][3] of this launch
    float* Tout;                     // [n_cams][H][W] or null
    const float2* skip;              // skip modes: [n_cams][H][W] (t_start, t_end) from the cube entry
    const uint32_t* bits;            // coarse occupancy (suffix checks)
    int32_t W, H, bx_per_cam, blocks_per_cam, n_cams;
    int32_t cbx_per_cam, cblocks_per_cam;   // camera kernel tiles (cam_tile_w x cam_tile_h of the mode)
    uint32_t snap_bytes;             // BUF kernels: bytes of one camera's snapshot records
    float bg[3];
    float stop_T;
};
static_assert(sizeof(CamLaunch) <= 4096, "kernel argument block too large");

// Skip pre-pass: per pixel, the part of the chord the render has to walk.
struct SkipLaunch {
    float frame[kCamsPerLaunch][12];
    float tau[kCamsPerLaunch];       // t / T mod 1 of each camera
    const uint32_t* bits;
    const unsigned char* packed;     // proposal weights (MLP variant)
    float2* skip;                    // [n_cams][H][W]
    int32_t W, H, bx_per_cam, blocks_per_cam, n_cams;
};

// Block index -> logical tile, giving XCD x (blocks x, x+8, ...) the
// contiguous range [x * per, (x + 1) * per).  gridDim.x is a multiple of 8.
__device__ inline int xcd_band(int bid, int nblocks)
{
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Skip pre-pass: per pixel, a part of the chord [t_start, t_end] outside
// which the ray provably meets no leaf.  Coarse variant: the first and last
// set coarse cells on the chord (a forward and a backward scan).  Proposal
// variant: the network's entry guess is accepted if the scan up to it is
// clear, else the walk starts at the first set cell that scan met; its exit
// guess is accepted if the backward scan from the cube exit down to it is
// clear, else the walk ends at the exit of the last set cell; a predicted
// miss is checked like the coarse variant (forward scan only).  (inf, inf)
// marks a ray with nothing to walk.
//
// The proposal variant runs in two kernels: proposal_infer_kernel evaluates
// the network (FP16 matrix cores, its fragments in LDS, grid-stride over
// tiles so each block reads the weights once) and leaves each pixel's
// prediction (s_in, s_out as fractions of the chord, s_in < 0 for a predicted
// miss) in the skip buffer; skip_scan_kernel<true> then turns it into the
// proven interval.  The scans are latency-bound and run at the occupancy of a
// small kernel instead of the network's.
struct PixelRay {
    int ci, px, py;
    bool inside;
};

__device__ inline PixelRay pixel_of(const SkipLaunch& a, int lin)
{
    PixelRay p;
    p.ci = lin / a.blocks_per_cam;
    const int tb = lin - p.ci * a.blocks_per_cam;
    const int bx = tb % a.bx_per_cam;
    const int by = tb / a.bx_per_cam;
    const int wv = threadIdx.x >> 6;
    const int ln = threadIdx.x & 63;
    p.px = bx * 16 + (wv & 1) * 8 + (ln & 7);
    p.py = by * 16 + (wv >> 1) * 8 + (ln >> 3);
    p.inside = p.px < a.W && p.py < a.H;
    return p;
}

__device__ inline bool pixel_ray(const SkipLaunch& a, const PixelRay& p, Ray& r)
{
    const float* fr = a.frame[p.ci];
    const float sx = (float)(2 * p.px + 1 - a.W) / (float)a.W;
    const float sy = (float)(a.H - 2 * p.py - 1) / (float)a.H;
    const float dx = fr[3] + sx * fr[6] + sy * fr[9];
    const float dy = fr[4] + sx * fr[7] + sy * fr[10];
    const float dz = fr[5] + sx * fr[8] + sy * fr[11];
    return setup_ray(fr[0], fr[1], fr[2], dx, dy, dz, r) && p.inside;
}

__global__ __launch_bounds__(kBlock) void proposal_infer_kernel(SkipLaunch a)
{
    __shared__ uint2 s_frag[kFrags * 64];
    __shared__ float s_bias[132];
    const uint2* F = reinterpret_cast<const uint2*>(a.packed);
    for (int i = threadIdx.x; i < kFrags * 64; i += kBlock) s_frag[i] = F[i];
    if (threadIdx.x < 132) s_bias[threadIdx.x] = reinterpret_cast<const float*>(a.packed + kPackedBias)[threadIdx.x];
    __syncthreads();
    const int total = a.n_cams * a.blocks_per_cam;
    const int padded = (total + 7) / 8 * 8;
    for (int it = blockIdx.x; it < padded; it += gridDim.x) {
        const int lin = xcd_band(it, padded);
        if (lin >= total) continue;                     // whole blocks: every wave stays complete
        const PixelRay p = pixel_of(a, lin);
        Ray r;
        const bool ok = pixel_ray(a, p, r);
        float x[kMlpIn];
        proposal_inputs(r, a.tau[p.ci], x);
        if (!ok)
            for (int c = 0; c < kMlpIn; ++c) x[c] = 0.0f;
        float o3[3] = {0.0f, 0.0f, 0.0f};
        mlp_infer_wave(s_frag, s_bias, x, o3);          // wave-wide: every lane is active here
        if (p.inside)
            a.skip[((int64_t)p.ci * a.H + p.py) * a.W + p.px] =
                o3[0] > 0.0f ? make_float2(sigmoidf_(o3[1]), sigmoidf_(o3[2])) : make_float2(-1.0f, 0.0f);
    }
}

template <bool PROP>
__global__ __launch_bounds__(kBlock) void skip_scan_kernel(SkipLaunch a)
{
    const int total = a.n_cams * a.blocks_per_cam;
    const int lin = xcd_band(blockIdx.x, gridDim.x);
    if (lin >= total) return;
    const PixelRay p = pixel_of(a, lin);
    if (!p.inside) return;
    Ray r;
    const bool ok = pixel_ray(a, p, r);
    const int64_t pix = ((int64_t)p.ci * a.H + p.py) * a.W + p.px;
    float ts = __builtin_inff(), te = __builtin_inff();
    if (ok) {
        const float len = r.t_len;
        const float2 pred = PROP ? a.skip[pix] : make_float2(-1.0f, 0.0f);
        float pe[3], nd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pe[c] = fmaf(len, r.d[c], r.o[c]);
            nd[c] = -r.d[c];
        }
        if (!PROP || pred.x < 0.0f) {
            const float f = coarse_scan(a.bits, r.o, r.d, len);
            if (f < len) {
                ts = f;
                te = PROP ? len : len - coarse_scan(a.bits, pe, nd, len - f);
            }
        } else {
            // entry: accept the guess if the chord up to it is clear; exit:
            // accept the guess if the chord after it is clear, else take the
            // exit of the last set cell
            ts = coarse_scan(a.bits, r.o, r.d, pred.x * len);
            const float span = len - fmaxf(pred.y * len, ts);
            te = span > 0.0f ? len - coarse_scan(a.bits, pe, nd, span) : len;
        }
    }
    a.skip[pix] = make_float2(ts, te);
}

// SKIP: walk only the proven part [t_start, t_end] of each chord that the
// skip pre-pass left in a.skip.  BUF (snapshot modes, records within 4 GiB):
// snapshot reads through a buffer resource, and at most 64 VGPRs.
template <int MODE, bool SKIP, int N1 = FPO_N_SIGMA, int N2 = FPO_N_SH_FOURIER, bool BUF = false,
          int WAVES = cam_waves(MODE)>
__global__ __launch_bounds__(64 * WAVES, BUF ? 32 / WAVES : 1) void render_cam_kernel(CamLaunch a)
{
    static_assert(!BUF || MODE >= 16, "buffer reads serve snapshot records only");
    constexpr int kThreads = 64 * WAVES;
    constexpr int kTileW = cam_tile_w(WAVES);
    constexpr int kTileH = cam_tile_h(WAVES);
    __shared__ int s_stack[kStackLevels * kThreads];
    const int lin = xcd_band(blockIdx.x, gridDim.x);
    if (lin >= a.n_cams * a.cblocks_per_cam) return;
    const int ci = lin / a.cblocks_per_cam;
    const int tb = lin - ci * a.cblocks_per_cam;
    const int bx = tb % a.cbx_per_cam;
    const int by = tb / a.cbx_per_cam;
    const int wv = threadIdx.x >> 6;
    const int ln = threadIdx.x & 63;
    const int px = bx * kTileW + (wv & 1) * 8 + (ln & 7);
    const int py = by * kTileH + (wv >> 1) * 8 + (ln >> 3);
    if (px >= a.W || py >= a.H) return;

    const CamDev& cam = a.cam[ci];
    float b[FPO_BASIS_STRIDE];
#pragma unroll
    for (int i = 0; i < FPO_BASIS_STRIDE; ++i) b[i] = cam.basis[i];
    // exact integer numerators: no cancellation near the image centre
    const float sx = (float)(2 * px + 1 - a.W) / (float)a.W;
    const float sy = (float)(a.H - 2 * py - 1) / (float)a.H;
    const float dx = cam.frame[3] + sx * cam.frame[6] + sy * cam.frame[9];
    const float dy = cam.frame[4] + sx * cam.frame[7] + sy * cam.frame[10];
    const float dz = cam.frame[5] + sx * cam.frame[8] + sy * cam.frame[11];

    Shade<MODE, N1, N2, BUF> sh{a.tree, b, cam.snap};
    if constexpr (BUF)
        sh.srs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(cam.snap), (short)0, (int)a.snap_bytes, 0x00020000);
    sh.Tr = 1.0f;
    sh.C[0] = sh.C[1] = sh.C[2] = 0.0f;
    sh.stop_T = a.stop_T;
    Ray r;
    const int64_t pix = ((int64_t)ci * a.H + py) * a.W + px;
    // the plain walk starts on the face of the leaves' bounds (rays that miss
    // them end here); the skip pre-pass measures along the cube's chord
    bool hit;
    if constexpr (SKIP) hit = setup_ray(cam.frame[0], cam.frame[1], cam.frame[2], dx, dy, dz, r);
    else hit = setup_ray_in(a.tree.box_lo, a.tree.box_hi, cam.frame[0], cam.frame[1], cam.frame[2], dx, dy, dz, r);
    if (hit) {
        sh9(r.d[0], r.d[1], r.d[2], sh.Y);
        if constexpr (!SKIP) {
            walk<(MODE >= 16), kThreads>(a.tree, r, s_stack + threadIdx.x, sh);
        } else {
            const float2 se = a.skip[pix];
            if (se.x < r.t_len) {
#pragma unroll
                for (int c = 0; c < 3; ++c) r.o[c] = fmaf(se.x, r.d[c], r.o[c]);
                r.t_len -= se.x;
                NoStop ns;
                walk<(MODE >= 16), kThreads>(a.tree, r, s_stack + threadIdx.x, sh, se.y - se.x, ns);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) a.rgb[pix * 3 + c] = fmaf(sh.Tr, a.bg[c], sh.C[c]);
    if (a.Tout) a.Tout[pix] = sh.Tr;
}

struct RaysLaunch {
    TreeDev tree;
    const float* o;
    const float* d;
    const int32_t* t_idx;
    const float* basis;     // [n_t][32]
    const void* snap;
    int64_t snap_stride;    // leaf records between consecutive time indices' snapshots
    int64_t n;
    int32_t n_t;
    float* rgb;
    float* Tout;
    float bg[3];
    float stop_T;
    int32_t* rec_count;     // segment records (one ray per wave only): per-ray count, -1 on overflow
    float4* rec;            // [n][rec_cap] records of 32 bytes
    int32_t rec_cap;
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void render_rays_kernel(RaysLaunch a)
{
    __shared__ int s_stack[kStackLevels * kBlock];
    const int64_t r_id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r_id >= a.n) return;
    int ti = a.t_idx[r_id];
    ti = min(max(ti, 0), a.n_t - 1);
    float b[FPO_BASIS_STRIDE];
    const float4* brow = reinterpret_cast<const float4*>(a.basis + (int64_t)ti * FPO_BASIS_STRIDE);
#pragma unroll
    for (int i = 0; i < FPO_BASIS_STRIDE / 4; ++i) {
        const float4 v = brow[i];
        b[4 * i] = v.x; b[4 * i + 1] = v.y; b[4 * i + 2] = v.z; b[4 * i + 3] = v.w;
    }
    const void* snap = a.snap;
    if constexpr (MODE >= 16) {
        const size_t rec = (MODE - 16) == FPO_F32 ? 128 : 64;
        snap = static_cast<const char*>(a.snap) + (size_t)ti * (size_t)a.snap_stride * rec;
    }
    Shade<MODE> sh{a.tree, b, snap};
    sh.Tr = 1.0f;
    sh.C[0] = sh.C[1] = sh.C[2] = 0.0f;
    sh.stop_T = a.stop_T;
    Ray r;
    if (setup_ray_in(a.tree.box_lo, a.tree.box_hi, a.o[3 * r_id], a.o[3 * r_id + 1], a.o[3 * r_id + 2],
                  a.d[3 * r_id], a.d[3 * r_id + 1], a.d[3 * r_id + 2], r)) {
        sh9(r.d[0], r.d[1], r.d[2], sh.Y);
        walk(a.tree, r, s_stack + threadIdx.x, sh);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) a.rgb[r_id * 3 + c] = fmaf(sh.Tr, a.bg[c], sh.C[c]);
    if (a.Tout) a.Tout[r_id] = sh.Tr;
}

// F32 Fourier-mode render of a small ray batch, one ray per wave.  REC: also
// write each ray's segment records (FPO_RAYS_RECORD).
template <bool REC>
__global__ __launch_bounds__(kBlock, REC ? 8 : 1) void render_rays_wave_kernel(RaysLaunch a)
{
    __shared__ int s_stack[kStackLevels * kBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t r_id = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (r_id >= a.n) return;
    const int ti = min(max(a.t_idx[r_id], 0), a.n_t - 1);
    WaveShade<false, REC> sh{a.tree};
    sh.lane = lane;
    sh.Tr = 1.0f;
    sh.C[0] = sh.C[1] = sh.C[2] = 0.0f;
    sh.stop_T = a.stop_T;
    if constexpr (REC) {
        sh.rec = a.rec + r_id * a.rec_cap * 2;
        sh.rec_cap = a.rec_cap;
    }
    Ray r;
    if (setup_ray_in(a.tree.box_lo, a.tree.box_hi, a.o[3 * r_id], a.o[3 * r_id + 1], a.o[3 * r_id + 2],
                  a.d[3 * r_id], a.d[3 * r_id + 1], a.d[3 * r_id + 2], r)) {
        float Y[FPO_N_SH];
        sh9(r.d[0], r.d[1], r.d[2], Y);
        sh.sl.init(lane, a.basis + (int64_t)ti * FPO_BASIS_STRIDE, Y);
        walk<true>(a.tree, r, s_stack + threadIdx.x, sh);
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.rgb[r_id * 3 + c] = fmaf(sh.Tr, a.bg[c], sh.C[c]);
        if (a.Tout) a.Tout[r_id] = sh.Tr;
        if constexpr (REC) a.rec_count[r_id] = sh.rec_n <= a.rec_cap ? sh.rec_n : -1;
    }
}

// Records the walk's segments, with distances from the caller's origin.
struct TraceVisitor {
    int32_t* ids;
    float* t01;
    int32_t cap;
    int32_t n;
    float t_in;
    __device__ inline bool segment(int leaf, float t0, float t1)
    {
        if (n < cap) {
            ids[n] = leaf;
            t01[2 * n] = t_in + t0;
            t01[2 * n + 1] = t_in + t1;
        }
        ++n;
        return false;
    }
};

struct TraceLaunch {
    TreeDev tree;
    const float* o;
    const float* d;
    int64_t n;
    int32_t cap;
    int32_t* ids;
    float* t01;
    int32_t* n_visits;
};

__global__ __launch_bounds__(kBlock) void trace_rays_kernel(TraceLaunch a)
{
    __shared__ int s_stack[kStackLevels * kBlock];
    const int64_t r_id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r_id >= a.n) return;
    TraceVisitor v{a.ids + r_id * a.cap, a.t01 + r_id * a.cap * 2, a.cap, 0, 0.0f};
    Ray r;
    if (setup_ray_in(a.tree.box_lo, a.tree.box_hi, a.o[3 * r_id], a.o[3 * r_id + 1], a.o[3 * r_id + 2],
                  a.d[3 * r_id], a.d[3 * r_id + 1], a.d[3 * r_id + 2], r)) {
        v.t_in = r.t_in;
        walk(a.tree, r, s_stack + threadIdx.x, v);
    }
    a.n_visits[r_id] = v.n;
}

__global__ __launch_bounds__(kBlock) void camera_rays_kernel(const float* table, int32_t n_cams,
                                                             const int32_t* cam, const int32_t* py,
                                                             const int32_t* px, int64_t n, float* o, float* d)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    const int ci = min(max(cam[r], 0), n_cams - 1);
    const float* f = table + (int64_t)ci * FPO_CAMERA_FLOATS;
    const int W = (int)f[12], H = (int)f[13];
    const float sx = (float)(2 * px[r] + 1 - W) / (float)W;
    const float sy = (float)(H - 2 * py[r] - 1) / (float)H;
    float v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = f[3 + a] + sx * f[6 + a] + sy * f[9 + a];
    const float inv = 1.0f / sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[3 * r + a] = f[a];
        d[3 * r + a] = v[a] * inv;
    }
}

// dst word (slot, g) = coefficients 4g .. 4g+3 of leaf perm[slot] (F32
// records of 48 words; padding words and slots >= n_leaves are zero).
__global__ __launch_bounds__(kBlock) void pack_coeffs_kernel(const float* src, const int64_t* perm,
                                                             int64_t n_leaves, int64_t stride, float4* dst,
                                                             int R, int n_coeff)
{
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= R * stride) return;
    const int64_t slot = id / R;
    const int g = (int)(id - slot * R);
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (slot < n_leaves) {
        const int64_t p = perm[slot];
        if (p >= 0 && p < n_leaves) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = 4 * g + e;
                if (q < n_coeff) v[e] = src[p * n_coeff + q];
            }
        }
    }
    dst[id] = make_float4(v[0], v[1], v[2], v[3]);
}

}  // namespace dev

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
using dev::tree_dev;

static int mode_of(const fpo_tree_view* t, const fpo_render_opts* o)
{
    if (o->snapshot) return 16 + (int)o->snapshot_dtype;
    return (int)t->dtype;
}

}  // namespace fpo

using namespace fpo;

template <int MODE, bool BUF = false>
static void launch_cam(const dev::CamLaunch& a, int grid, int skip, hipStream_t s)
{
    if (skip != 0)
        hipLaunchKernelGGL((dev::render_cam_kernel<MODE, true, FPO_N_SIGMA, FPO_N_SH_FOURIER, BUF>), dim3(grid),
                           dim3(64 * dev::cam_waves(MODE)), 0, s, a);
    else
        hipLaunchKernelGGL((dev::render_cam_kernel<MODE, false, FPO_N_SIGMA, FPO_N_SH_FOURIER, BUF>), dim3(grid),
                           dim3(64 * dev::cam_waves(MODE)), 0, s, a);
}

// Fourier-mode render of another coefficient layout (n1, n2) = key / 100,
// key % 100 from a store of DT; false if the layout is not compiled.
template <int DT>
static bool launch_layout(const dev::CamLaunch& a, int key, int grid, hipStream_t s)
{
    switch (key) {
#define FPO_LAY(A, B) case A * 100 + B: \
        hipLaunchKernelGGL((dev::render_cam_kernel<DT, false, A, B>), dim3(grid), dim3(64 * dev::cam_waves(DT)), 0, s, a); return true
        FPO_LAY(11, 5); FPO_LAY(21, 5); FPO_LAY(11, 11); FPO_LAY(21, 11); FPO_LAY(31, 11);
#undef FPO_LAY
        default: return false;
    }
}

// The body of fpo_render: cameras go out in launches of at most
// cams_per_launch (<= 16); the skip modes' scratch (opts->workspace) holds
// one launch's pixels and is reused by every launch of the call.
static fpo_status render_impl(const fpo_tree_view* tree, const fpo_camera* cams, int32_t n_cams,
                              const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream,
                              int cams_per_launch)
{
    fpo_status st = check_tree(tree, opts == nullptr || opts->snapshot == nullptr, true);
    if (st != FPO_OK) return st;
    if ((st = check_opts(opts, tree, true)) != FPO_OK) return st;
    // the snapshot render does not read coefficients, so any compiled layout goes
    const bool variant = !default_layout(tree->layout) && !opts->snapshot;
    if (variant && opts->flags != 0)
        return fail(FPO_E_UNSUPPORTED, "layouts other than (31, 5) render without skipping only");
    if (!cams || n_cams < 1) return fail(FPO_E_INVALID, "cams is NULL or n_cams < 1");
    if (!rgb_out) return fail(FPO_E_INVALID, "rgb_out is NULL");
    const int W = cams[0].width, H = cams[0].height;
    for (int i = 0; i < n_cams; ++i)
        if (cams[i].width != W || cams[i].height != H)
            return fail(FPO_E_INVALID, "all cameras of one call must share width and height");
    if ((int64_t)W * H > (1ll << 30)) return fail(FPO_E_INVALID, "image too large");
    const int skip = force_fallback() ? 0 : opts->flags;     // FPO_FORCE_FALLBACK=1: plain traversal
    const int per_launch = std::max(1, std::min(cams_per_launch, dev::kCamsPerLaunch));
    if (skip != 0) {
        const int64_t need = (int64_t)std::min(n_cams, per_launch) * W * H * 8;
        if (opts->workspace_bytes < need)
            return fail(FPO_E_INVALID, "opts->workspace_bytes < min(n_cams, 16) * W * H * 8");
    }
    // Validate every camera before launching anything.
    static thread_local dev::CamLaunch a;
    static thread_local dev::SkipLaunch sk;
    std::memset(&a, 0, sizeof(a));
    for (int i = 0; i < n_cams; ++i) {
        float fr[12];
        if ((st = camera_frame(cams[i], fr)) != FPO_OK) return st;
    }
    a.tree = tree_dev(tree);
    a.W = W;
    a.H = H;
    a.bx_per_cam = (W + 15) / 16;
    a.blocks_per_cam = a.bx_per_cam * ((H + 15) / 16);
    for (int c = 0; c < 3; ++c) a.bg[c] = opts->bg[c];
    a.stop_T = opts->stop_T;
    const int mode = mode_of(tree, opts);
    {
        const int waves = variant ? dev::cam_waves(tree->dtype) : dev::cam_waves(mode);
        const int tw = dev::cam_tile_w(waves), th = dev::cam_tile_h(waves);
        a.cbx_per_cam = (W + tw - 1) / tw;
        a.cblocks_per_cam = a.cbx_per_cam * ((H + th - 1) / th);
    }
    const size_t snap_rec = opts->snapshot_dtype == FPO_F32 ? 128 : 64;   // bytes per leaf record
    // snapshot records within 4 GiB per camera are read with 32-bit offsets
    const bool snap_buf = opts->snapshot && (uint64_t)tree->n_leaves * snap_rec <= 0xFFFFFFFFull;
    a.snap_bytes = snap_buf ? (uint32_t)((uint64_t)tree->n_leaves * snap_rec) : 0u;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int c0 = 0; c0 < n_cams; c0 += per_launch) {
        const int nc = std::min(per_launch, n_cams - c0);
        a.n_cams = nc;
        for (int i = 0; i < nc; ++i) {
            const fpo_camera& cam = cams[c0 + i];
            camera_frame(cam, a.cam[i].frame);
            basis_row(cam.time, (double)tree->layout.period, tree->layout.n_sigma, a.cam[i].basis);
            a.cam[i].snap = opts->snapshot
                ? static_cast<const char*>(opts->snapshot) + (size_t)(c0 + i) * (size_t)opts->snapshot_cam_stride * snap_rec
                : nullptr;
        }
        a.rgb = rgb_out + (int64_t)c0 * W * H * 3;
        a.Tout = T_out ? T_out + (int64_t)c0 * W * H : nullptr;
        const int64_t total = (int64_t)nc * a.blocks_per_cam;
        const int64_t ctotal = (int64_t)nc * a.cblocks_per_cam;
        if (ctotal > INT32_MAX - 8) return fail(FPO_E_INVALID, "launch too large");
        const int grid = (int)((total + 7) / 8 * 8);           // skip pre-pass: 16x16 tiles
        const int cam_grid = (int)((ctotal + 7) / 8 * 8);       // camera kernel tiles
        if (skip != 0) {
            sk.n_cams = nc;
            sk.W = W;
            sk.H = H;
            sk.bx_per_cam = a.bx_per_cam;
            sk.blocks_per_cam = a.blocks_per_cam;
            for (int i = 0; i < nc; ++i) {
                for (int q = 0; q < 12; ++q) sk.frame[i][q] = a.cam[i].frame[q];
                const double per = (double)tree->layout.period;
                double tau = std::fmod(cams[c0 + i].time / per, 1.0);
                if (tau < 0.0) tau += 1.0;
                sk.tau[i] = (float)tau;
            }
            sk.bits = opts->coarse_bits;
            sk.packed = static_cast<const unsigned char*>(opts->proposal);
            sk.skip = static_cast<float2*>(opts->workspace);
            a.skip = sk.skip;
            a.bits = opts->coarse_bits;
            if (skip == FPO_RENDER_SKIP_PROPOSAL) {
                hipLaunchKernelGGL(dev::proposal_infer_kernel, dim3(std::min(grid, 1024)), dim3(dev::kBlock), 0, s, sk);
                hipLaunchKernelGGL(dev::skip_scan_kernel<true>, dim3(grid), dim3(dev::kBlock), 0, s, sk);
            } else {
                hipLaunchKernelGGL(dev::skip_scan_kernel<false>, dim3(grid), dim3(dev::kBlock), 0, s, sk);
            }
            if ((st = launch_status("fpo_render (skip pre-pass)")) != FPO_OK) return st;
        }
        if (variant) {
            const int key = tree->layout.n_sigma * 100 + tree->layout.n_sh_fourier;
            bool ok = false;
            switch (tree->dtype) {
                case FPO_F32: ok = launch_layout<FPO_F32>(a, key, cam_grid, s); break;
                case FPO_BF16: ok = launch_layout<FPO_BF16>(a, key, cam_grid, s); break;
                default: ok = launch_layout<FPO_FP8_E4M3>(a, key, cam_grid, s); break;
            }
            if (!ok) return fail(FPO_E_UNSUPPORTED, "layout (n1, n2) not compiled");
            if ((st = launch_status("fpo_render")) != FPO_OK) return st;
            continue;
        }
        switch (mode) {
            case FPO_F32: launch_cam<FPO_F32>(a, cam_grid, skip, s); break;
            case FPO_BF16: launch_cam<FPO_BF16>(a, cam_grid, skip, s); break;
            case FPO_FP8_E4M3: launch_cam<FPO_FP8_E4M3>(a, cam_grid, skip, s); break;
            case dev::kSnapF32:
                if (snap_buf) launch_cam<dev::kSnapF32, true>(a, cam_grid, skip, s);
                else launch_cam<dev::kSnapF32>(a, cam_grid, skip, s);
                break;
            case dev::kSnapBF16:
                if (snap_buf) launch_cam<dev::kSnapBF16, true>(a, cam_grid, skip, s);
                else launch_cam<dev::kSnapBF16>(a, cam_grid, skip, s);
                break;
            default: return fail(FPO_E_INVALID, "unknown render mode");
        }
        if ((st = launch_status("fpo_render")) != FPO_OK) return st;
    }
    return FPO_OK;
}

extern "C" fpo_status fpo_render(const fpo_tree_view* tree, const fpo_camera* cams, int32_t n_cams,
                                 const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream)
{
    ApiRange api_range_("fpo_render");
    return render_impl(tree, cams, n_cams, opts, rgb_out, T_out, stream, dev::kCamsPerLaunch);
}

// ---------------------------------------------------------------------------
// fpo_render_noalloc: fpo_render whose skip-mode scratch is a file-scope
// device array instead of a caller workspace.  Each device that loads the
// library holds its own copy (kNoallocScratchBytes) until the process ends.
// Host code never passes the array's name to a kernel: its device address
// comes from hipGetSymbolAddress, once per device, with that device current.
// ---------------------------------------------------------------------------
namespace fpo {
namespace dev {
constexpr int64_t kNoallocScratchBytes = FPO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
}  // namespace dev

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first
// call from that device).
static fpo_status scratch_address(void** out)
{
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices)
        return fail(FPO_E_DEVICE, "fpo_render_noalloc: no current HIP device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[d]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(dev::scratch));
        if (e != hipSuccess || !p)
            return fail(FPO_E_DEVICE, std::string("fpo_render_noalloc: hipGetSymbolAddress failed: ") +
                                          hipGetErrorString(e));
        g_scratch_ptr[d] = p;
    }
    *out = g_scratch_ptr[d];
    return FPO_OK;
}
}  // namespace fpo

extern "C" fpo_status fpo_render_noalloc(const fpo_tree_view* tree, const fpo_camera* cams, int32_t n_cams,
                                         const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream)
{
    ApiRange api_range_("fpo_render_noalloc");
    // every host-side check before the device is touched
    fpo_status st = check_tree(tree, opts == nullptr || opts->snapshot == nullptr, true);
    if (st != FPO_OK) return st;
    if ((st = check_opts(opts, tree, true, false, false)) != FPO_OK) return st;
    if (opts->flags == 0) return render_impl(tree, cams, n_cams, opts, rgb_out, T_out, stream, dev::kCamsPerLaunch);
    if (!cams || n_cams < 1) return fail(FPO_E_INVALID, "cams is NULL or n_cams < 1");
    const int64_t per_cam = (int64_t)cams[0].width * cams[0].height * 8;
    if (cams[0].width < 1 || cams[0].height < 1) return fail(FPO_E_INVALID, "bad image size");
    if (per_cam > FPO_NOALLOC_SCRATCH_BYTES)
        return fail(FPO_E_CAPACITY, "fpo_render_noalloc: one camera's skip scratch (8 W H bytes) exceeds "
                                    "FPO_NOALLOC_SCRATCH_BYTES; use fpo_render with a workspace");
    void* ptr = nullptr;
    if ((st = scratch_address(&ptr)) != FPO_OK) return st;
    fpo_render_opts o = *opts;
    o.workspace = ptr;
    o.workspace_bytes = FPO_NOALLOC_SCRATCH_BYTES;
    const int per_launch = (int)std::min<int64_t>(dev::kCamsPerLaunch, FPO_NOALLOC_SCRATCH_BYTES / per_cam);
    return render_impl(tree, cams, n_cams, &o, rgb_out, T_out, stream, per_launch);
}

template <int MODE>
static void launch_rays(const dev::RaysLaunch& a, int64_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(dev::render_rays_kernel<MODE>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s, a);
}

extern "C" fpo_status fpo_render_rays(const fpo_tree_view* tree, const float* o, const float* d,
                                      const int32_t* t_idx, const float* basis, int32_t n_t, int64_t n_rays,
                                      const fpo_render_opts* opts, float* rgb_out, float* T_out, void* stream)
{
    ApiRange api_range_("fpo_render_rays");
    fpo_status st = check_tree(tree, opts == nullptr || opts->snapshot == nullptr);
    if (st != FPO_OK) return st;
    const bool record = opts && opts->flags == FPO_RAYS_RECORD;
    if ((st = check_opts(opts, tree, false, true)) != FPO_OK) return st;
    if (n_rays < 0) return fail(FPO_E_INVALID, "n_rays < 0");
    if (n_rays == 0) return FPO_OK;
    RecordLayout rl;
    if (record) {
        if (mode_of(tree, opts) != FPO_F32 || n_rays > dev::kWaveRayBatch)
            return fail(FPO_E_UNSUPPORTED, "FPO_RAYS_RECORD needs F32 Fourier mode and at most 32768 rays");
        if ((st = record_layout(opts, n_rays, rl)) != FPO_OK) return st;
    }
    if (!o || !d || !t_idx || !basis || !rgb_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (n_rays > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rays");
    dev::RaysLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.tree = tree_dev(tree);
    a.o = o; a.d = d; a.t_idx = t_idx; a.basis = basis; a.n_t = n_t; a.n = n_rays;
    a.snap = opts->snapshot;
    a.snap_stride = opts->snapshot_cam_stride;
    a.rgb = rgb_out; a.Tout = T_out;
    for (int c = 0; c < 3; ++c) a.bg[c] = opts->bg[c];
    a.stop_T = opts->stop_T;
    if (record) {
        a.rec_count = rl.count;
        a.rec = reinterpret_cast<float4*>(rl.records);
        a.rec_cap = rl.cap;
    }
    const int64_t grid = (n_rays + dev::kBlock - 1) / dev::kBlock;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int mode = mode_of(tree, opts);
    if (mode == FPO_F32 && n_rays <= dev::kWaveRayBatch) {
        const int64_t wgrid = (n_rays + dev::kBlock / dev::kWave - 1) / (dev::kBlock / dev::kWave);
        if (record)
            hipLaunchKernelGGL(dev::render_rays_wave_kernel<true>, dim3((unsigned)wgrid), dim3(dev::kBlock), 0, s, a);
        else
            hipLaunchKernelGGL(dev::render_rays_wave_kernel<false>, dim3((unsigned)wgrid), dim3(dev::kBlock), 0, s, a);
        return launch_status("fpo_render_rays");
    }
    switch (mode) {
        case FPO_F32: launch_rays<FPO_F32>(a, grid, s); break;
        case FPO_BF16: launch_rays<FPO_BF16>(a, grid, s); break;
        case FPO_FP8_E4M3: launch_rays<FPO_FP8_E4M3>(a, grid, s); break;
        case dev::kSnapF32: launch_rays<dev::kSnapF32>(a, grid, s); break;
        case dev::kSnapBF16: launch_rays<dev::kSnapBF16>(a, grid, s); break;
        default: return fail(FPO_E_INVALID, "unknown render mode");
    }
    return launch_status("fpo_render_rays");
}

extern "C" fpo_status fpo_trace_rays(const fpo_tree_view* tree, const float* o, const float* d, int64_t n_rays,
                                     int32_t max_visits, int32_t* leaf_ids, float* t01, int32_t* n_visits,
                                     void* stream)
{
    ApiRange api_range_("fpo_trace_rays");
    fpo_status st = check_tree(tree, false);
    if (st != FPO_OK) return st;
    if (n_rays < 0 || max_visits < 0) return fail(FPO_E_INVALID, "negative size");
    if (n_rays == 0) return FPO_OK;
    if (!o || !d || !n_visits || (max_visits > 0 && (!leaf_ids || !t01)))
        return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_rays > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rays");
    dev::TraceLaunch a;
    a.tree = tree_dev(tree);
    a.o = o; a.d = d; a.n = n_rays; a.cap = max_visits; a.ids = leaf_ids; a.t01 = t01; a.n_visits = n_visits;
    const int64_t grid = (n_rays + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::trace_rays_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return launch_status("fpo_trace_rays");
}

extern "C" fpo_status fpo_camera_rays(const float* cam_table, int32_t n_cams, const int32_t* cam,
                                      const int32_t* py, const int32_t* px, int64_t n,
                                      float* o_out, float* d_out, void* stream)
{
    ApiRange api_range_("fpo_camera_rays");
    if (n < 0) return fail(FPO_E_INVALID, "n < 0");
    if (n == 0) return FPO_OK;
    if (!cam_table || !cam || !py || !px || !o_out || !d_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_cams < 1) return fail(FPO_E_INVALID, "n_cams must be >= 1");
    if (n > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rays");
    const int64_t grid = (n + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::camera_rays_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), cam_table, n_cams, cam, py, px, n, o_out, d_out);
    return launch_status("fpo_camera_rays");
}

extern "C" fpo_status fpo_pack_coeffs(const float* src, const int64_t* perm, int64_t n_leaves,
                                      int64_t leaf_stride, const fpo_layout* layout, float* dst, void* stream)
{
    ApiRange api_range_("fpo_pack_coeffs");
    if (!src || !perm || !dst) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_leaves < 1 || leaf_stride < n_leaves) return fail(FPO_E_INVALID, "bad n_leaves / leaf_stride");
    const int n1 = layout ? layout->n_sigma : FPO_N_SIGMA;
    const int n2 = layout ? layout->n_sh_fourier : FPO_N_SH_FOURIER;
    if (!layout_supported(n1, n2)) return fail(FPO_E_UNSUPPORTED, "layout (n1, n2) not compiled");
    const int n_coeff = n1 + 3 * FPO_N_SH * n2;
    const int R = record_words(FPO_F32, n1, n2);
    const int64_t total = (int64_t)R * leaf_stride;
    if (total > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many leaves");
    const int64_t grid = (total + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::pack_coeffs_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), src, perm, n_leaves, leaf_stride,
                       reinterpret_cast<float4*>(dst), R, n_coeff);
    return launch_status("fpo_pack_coeffs");
}
