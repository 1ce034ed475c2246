// libfpo construction entry points (Sec. 4.2): per-frame values on the
// union leaves, and the per-leaf DFT of Eq. 10-12 that turns them into
// Fourier coefficients.
//
// Values of one frame and one leaf travel as snapshot records (32 F32 values:
// 0 = sigma, 1 + c*9 + j = z_{c,j}, 28..31 zero), the same records a time bake
// produces, so that the DFT of T records sampled at t = 0 .. T-1 is the exact
// inverse of fpo_bake_times for band-limited leaves.
//
// DFT kernel.  A 256-thread block takes 64 leaves; its wave g covers one
// quarter of each leaf's outputs (g = 0: the 31 density coefficients; g = 1..3:
// nine SH coefficients x 5 Fourier terms), so every wave runs one uniform code
// path.  The weighted basis c_i IDFT_i(t) of all frames sits in LDS (c_0 = 1/T,
// c_i = 2/T, or 1/T for every i with the printed weights), computed from exact
// integer phases (i t mod 2T) with sinpi / cospi.  The 64 records of a tile are
// contiguous in every frame: the block stages 4 frames of them at a time into
// LDS with whole-line loads, then each wave reads its values from there; the
// next 4 frames' loads are in flight in registers meanwhile.  The kernel
// streams T records per leaf and is bound by HBM reads.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"

namespace fpo {
namespace dev {

// Union leaf `slot` (cell d, i, j, k) in the frame's octree: the frame leaf that
// is the cell or contains it, else empty.  A frame node that is still internal
// at the cell's depth means the cell list does not refine the frame.
__global__ __launch_bounds__(kBlock) void frame_values_kernel(TreeDev ft, const int64_t* __restrict__ perm,
                                                              const float4* __restrict__ vals,
                                                              const int4* __restrict__ cells, int64_t n,
                                                              float4* __restrict__ out, int* __restrict__ n_bad)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int4 c = cells[s];
    const int D = ft.max_depth;
    int leaf = -1;
    bool bad = c.x < 1 || c.x > D;
    if (!bad) {
        const int sh = D - c.x;
        const int x = c.y << sh, y = c.z << sh, z = c.w << sh;
        int node = 0;
        for (int lvl = 0; lvl < c.x; ++lvl) {
            const int b = D - 1 - lvl;
            const int oct = ((x >> b) & 1) | (((y >> b) & 1) << 1) | (((z >> b) & 1) << 2);
            const int ch = ft.children[node * 8 + oct];
            if (ch < 0) {
                leaf = -ch - 1;
                break;
            }
            if (ch == 0) break;
            if (ch >= ft.n_nodes || lvl + 1 >= c.x) {
                bad = true;
                break;
            }
            node = ch;
        }
    }
    if (bad) atomicAdd(n_bad, 1);
    float4* o = out + s * 8;
    if (leaf >= 0 && leaf < ft.n_leaves && !bad) {
        const float4* v = vals + perm[leaf] * 8;
#pragma unroll
        for (int w = 0; w < 7; ++w) o[w] = v[w];
        o[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else {
#pragma unroll
        for (int w = 0; w < 8; ++w) o[w] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}


struct DftLaunch {
    const float* frames;     // [T][stride][32]
    float* coeffs;           // [stride][192]
    float* sigma_max;        // [stride] or null
    int64_t n_leaves, stride;
    int32_t T;
    int32_t literal;
};

constexpr int kDftFrames = 4;     // frames staged per LDS pass
constexpr int kRecPad = 33;       // LDS floats per staged record (32 + 1 against bank conflicts)

__global__ __launch_bounds__(256) void dft_kernel(DftLaunch a)
{
    // dynamic LDS: basis [T][32] then the staged records [kDftFrames][64 * kRecPad]
    extern __shared__ float lds[];
    const int T = a.T;
    float (*B)[FPO_N_SIGMA + 1] = reinterpret_cast<float (*)[FPO_N_SIGMA + 1]>(lds);
    float (*X)[64 * kRecPad] = reinterpret_cast<float (*)[64 * kRecPad]>(lds + T * (FPO_N_SIGMA + 1));
    for (int e = threadIdx.x; e < T * FPO_N_SIGMA; e += 256) {
        const int t = e / FPO_N_SIGMA, i = e % FPO_N_SIGMA;
        // Eq. 8 at t: cos(i pi t / T) (even i), sin((i + 1) pi t / T) (odd i), exact phase
        const int m = (i & 1) ? i + 1 : i;
        const int ph = (int)(((int64_t)m * t) % (2 * T));
        const float x = (float)ph / (float)T;
        const float v = (i & 1) ? sinpif(x) : cospif(x);
        const float c = (i == 0 || a.literal) ? 1.0f / (float)T : 2.0f / (float)T;
        B[t][i] = c * v;
    }
    __syncthreads();
    const int g = threadIdx.x >> 6;          // wave: output group
    const int ll = threadIdx.x & 63;         // leaf within the tile
    const int q0 = 9 * (g - 1);              // SH coefficients q0 .. q0 + 8 (g >= 1), record values 1 + q
    const int64_t n_tiles = (a.n_leaves + 63) / 64;
    const int steps_per_tile = (T + kDftFrames - 1) / kDftFrames;
    // The block's work is a flat sequence of (tile, frame group) steps.  The
    // record words of step k + 1 are loaded into registers while step k is
    // computed, so the loads overlap the arithmetic.
    int64_t tile = blockIdx.x;
    int step = 0;
    float4 pf[kDftFrames * 2];
    auto fetch = [&](int64_t tl, int st) {
        const int64_t l0 = tl * 64;
        const int nl = (int)min<int64_t>(64, a.n_leaves - l0);
        const int f0 = st * kDftFrames;
#pragma unroll
        for (int u = 0; u < kDftFrames * 2; ++u) {
            const int e = u * 256 + threadIdx.x;      // [frame][record][word]: 512 float4 per frame
            const int f = e >> 9, w = e & 511;
            const int rl = w >> 3;
            pf[u] = (f0 + f < T && rl < nl)
                        ? reinterpret_cast<const float4*>(a.frames + ((int64_t)(f0 + f) * a.stride + l0) * 32)[w]
                        : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    };
    if (tile < n_tiles) fetch(tile, 0);
    float acc[45];
    float smax = -__builtin_inff();
#pragma unroll
    for (int e = 0; e < 45; ++e) acc[e] = 0.0f;
    while (tile < n_tiles) {
        const int64_t l0 = tile * 64;
        const int nl = (int)min<int64_t>(64, a.n_leaves - l0);
        const int t0 = step * kDftFrames;
        const int nf = min(kDftFrames, T - t0);
        // park this step's words in LDS (the previous step's reads are done)
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kDftFrames * 2; ++u) {
            const int e = u * 256 + threadIdx.x;
            const int f = e >> 9, w = e & 511;
            const int rl = w >> 3, rw = w & 7;
            float* d = &X[f][rl * kRecPad + rw * 4];
            d[0] = pf[u].x; d[1] = pf[u].y; d[2] = pf[u].z; d[3] = pf[u].w;
        }
        __syncthreads();
        // next step's loads, in flight during this step's arithmetic
        int64_t n_tile = tile;
        int n_step = step + 1;
        if (n_step == steps_per_tile) {
            n_step = 0;
            n_tile += gridDim.x;
        }
        if (n_tile < n_tiles) fetch(n_tile, n_step);
        for (int f = 0; f < nf; ++f) {
            const float* r = &X[f][ll * kRecPad];
            const float* bt = B[t0 + f];
            if (g == 0) {
                const float sv = r[0];
                smax = fmaxf(smax, sv);
#pragma unroll
                for (int i = 0; i < FPO_N_SIGMA; ++i) acc[i] = fmaf(sv, bt[i], acc[i]);
            } else {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const float z = r[1 + q0 + q];
#pragma unroll
                    for (int i = 0; i < FPO_N_SH_FOURIER; ++i) acc[q * 5 + i] = fmaf(z, bt[i], acc[q * 5 + i]);
                }
            }
        }
        if (step + 1 == steps_per_tile) {
            const int64_t l = l0 + ll;
            if (ll < nl) {
                float* out = a.coeffs + l * 192;
                if (g == 0) {
#pragma unroll
                    for (int i = 0; i < FPO_N_SIGMA; ++i) out[i] = acc[i];
                    if (a.sigma_max) a.sigma_max[l] = smax;
                } else {
                    float* o = out + FPO_N_SIGMA + q0 * FPO_N_SH_FOURIER;
#pragma unroll
                    for (int e = 0; e < 45; ++e) o[e] = acc[e];
                    if (g == 3)
                        for (int e = FPO_N_COEFF; e < 192; ++e) out[e] = 0.0f;
                }
            }
#pragma unroll
            for (int e = 0; e < 45; ++e) acc[e] = 0.0f;
            smax = -__builtin_inff();
        }
        tile = n_tile;
        step = n_step;
    }
}

}  // namespace dev
}  // namespace fpo

using namespace fpo;

extern "C" fpo_status fpo_frame_values(const fpo_tree_view* frame_tree, const int64_t* frame_perm,
                                       const float* frame_values, const int32_t* union_cells, int64_t n_union,
                                       float* out, int32_t* n_bad, void* stream)
{
    ApiRange api_range_("fpo_frame_values");
    fpo_status st = check_tree(frame_tree, false);
    if (st != FPO_OK) return st;
    if (n_union < 0) return fail(FPO_E_INVALID, "n_union < 0");
    if (n_union == 0) return FPO_OK;
    if (!frame_perm || !frame_values || !union_cells || !out || !n_bad) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_union > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many union leaves");
    const int64_t grid = (n_union + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::frame_values_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), dev::tree_dev(frame_tree), frame_perm,
                       reinterpret_cast<const float4*>(frame_values), reinterpret_cast<const int4*>(union_cells),
                       n_union, reinterpret_cast<float4*>(out), n_bad);
    return launch_status("fpo_frame_values");
}

extern "C" fpo_status fpo_dft_frames(const float* frames, int32_t n_frames, int64_t n_leaves, int64_t leaf_stride,
                                     int32_t literal, float* coeffs_out, float* sigma_max_out, void* stream)
{
    ApiRange api_range_("fpo_dft_frames");
    if (!frames || !coeffs_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_frames < 1 || n_frames > FPO_MAX_FRAMES) return fail(FPO_E_INVALID, "n_frames must be in 1..FPO_MAX_FRAMES");
    if (n_leaves < 0 || leaf_stride < n_leaves) return fail(FPO_E_INVALID, "need 0 <= n_leaves <= leaf_stride");
    if ((reinterpret_cast<uintptr_t>(frames) & 15) != 0 || (reinterpret_cast<uintptr_t>(coeffs_out) & 15) != 0)
        return fail(FPO_E_INVALID, "frames and coeffs_out must be 16-byte aligned");
    if (n_leaves == 0) return FPO_OK;
    dev::DftLaunch a;
    a.frames = frames;
    a.coeffs = coeffs_out;
    a.sigma_max = sigma_max_out;
    a.n_leaves = n_leaves;
    a.stride = leaf_stride;
    a.T = n_frames;
    a.literal = literal ? 1 : 0;
    const int64_t tiles = (n_leaves + 63) / 64;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles, 4096);
    const size_t lds = sizeof(float) * ((size_t)n_frames * (FPO_N_SIGMA + 1) + (size_t)dev::kDftFrames * 64 * dev::kRecPad);
    hipLaunchKernelGGL(dev::dft_kernel, dim3(grid), dim3(256), lds, static_cast<hipStream_t>(stream), a);
    return launch_status("fpo_dft_frames");
}
