// libfpo PlenOctree fusion (Sec. 3, fine stage; Eq. 3-5).
//
// Observe pass, per view: every pixel ray walks the static PlenOctree front
// to back with the transmittance of the current leaf values; each leaf
// segment entered with T > tau is an observation of the radiance field at its
// midpoint, weighted by T times its length, accumulated per leaf with FP32
// atomics.  Apply pass: one update of Eq. 3-5 for every leaf observed in the
// view, with the view's length-weighted mean transmittance as T_i.
//
// Readings of the paper: its query points are the leaf segments (a sampler
// stepping along the ray puts a number of points proportional to the chord
// into a leaf); all observations of one leaf in one view make one update;
// z_{c,j} is updated with Y_j(d) c_c(x, d), the colour projected on the SH
// basis of the view direction.  The radiance field is an analytic stand-in
// for the generalizable network (Gaussian mixture density, logistic
// view-dependent colour).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"

namespace fpo {
namespace dev {

struct FieldDev {
    float mu[FPO_FIELD_MAX_GAUSS][3];
    float inv2w2[FPO_FIELD_MAX_GAUSS];    // 1 / (2 w_g^2)
    float a[FPO_FIELD_MAX_GAUSS];
    int32_t n;
    float u[3][3];
    float v[3][3];
    float b[3];
};

struct FusionLaunch {
    TreeDev tree;
    const float* values;    // [stride][32] leaf records: sigma, z_{c,j} at 1 + 9c + j
    float* acc;             // [stride][FPO_FUSION_ACC]
    float frame[12];        // eye, forward, right * tan_x, up * tan_y
    int32_t W, H, bx;       // image size, 16 x 16 tiles per row
    float tau;
    FieldDev f;
};

__device__ inline float field_sigma(const FieldDev& f, const float x[3])
{
    float s = 0.0f;
#pragma unroll
    for (int g = 0; g < FPO_FIELD_MAX_GAUSS; ++g) {
        if (g >= f.n) break;
        const float dx = x[0] - f.mu[g][0], dy = x[1] - f.mu[g][1], dz = x[2] - f.mu[g][2];
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        s = fmaf(f.a[g], __expf(-r2 * f.inv2w2[g]), s);
    }
    return s;
}

constexpr int kObs = 30;            // accumulator values per observation
constexpr int kObsStride = 36;      // LDS floats per staged observation (9 x 16 bytes: spreads banks)

// The lanes that shade a segment in the same step stage their observations in
// the wave's LDS buffer and then add them to the accumulators together: the
// (observation, value) pairs are dealt out over those lanes, so one atomic
// instruction covers consecutive values of one or two leaf records instead of
// the same value of up to 64 different leaves.
struct FusionVisitor {
    const float* values;
    float* acc;
    const FieldDev& f;
    float* stage;           // this wave's [64][kObsStride] LDS buffer
    int lane;
    float o[3];             // entry point: walk distances are measured from it
    float d[3];             // unit direction
    float Y[FPO_N_SH];
    float T;
    float tau;
    float sigma_scale;

    __device__ inline bool segment(int leaf, float t0, float t1)
    {
        if (!(T > tau)) return true;
        const float delta = t1 - t0;
        const bool obs = delta > 0.0f;
        const uint64_t act = __ballot(obs);
        if (obs) {
            const int k = __popcll(act);
            const int rank = __popcll(act & ((1ull << lane) - 1ull));
            const float tm = 0.5f * (t0 + t1);
            const float x[3] = {fmaf(tm, d[0], o[0]), fmaf(tm, d[1], o[1]), fmaf(tm, d[2], o[2])};
            const float sig = field_sigma(f, x);
            float col[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float h = f.b[c];
#pragma unroll
                for (int a = 0; a < 3; ++a) h = fmaf(f.u[c][a], x[a], fmaf(f.v[c][a], d[a], h));
                col[c] = sigmoidf_(h);
            }
            const float w = T * delta;
            float v[kObsStride];
            v[0] = w;
            v[1] = w * sig;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < FPO_N_SH; ++j) v[2 + c * FPO_N_SH + j] = w * col[c] * Y[j];
            v[29] = delta;
            v[30] = 0.0f;
            v[31] = __int_as_float(leaf);
#pragma unroll
            for (int e = 32; e < kObsStride; ++e) v[e] = 0.0f;
            float4* st = reinterpret_cast<float4*>(stage + rank * kObsStride);
#pragma unroll
            for (int q = 0; q < kObsStride / 4; ++q) st[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int p = rank; p < k * kObs; p += k) {
                const int s = p / kObs;
                const int e = p - s * kObs;
                const float* src = stage + s * kObsStride;
                const int l = __float_as_int(src[31]);
                unsafeAtomicAdd(acc + (int64_t)l * FPO_FUSION_ACC + e, src[e]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            T *= __expf(-sigma_scale * fmaxf(values[(int64_t)leaf * 32], 0.0f) * delta);
        }
        return !(T > tau);
    }
};

// One camera; 16 x 16 pixel tiles per block, 8 x 8 per wave (as the render).
__global__ __launch_bounds__(kBlock) void fusion_observe_kernel(FusionLaunch a)
{
    __shared__ int s_stack[kStackLevels * kBlock];
    __shared__ __align__(16) float s_obs[kBlock / kWave][kWave * kObsStride];
    const int wv = threadIdx.x >> 6;
    const int ln = threadIdx.x & 63;
    const int bxi = blockIdx.x % a.bx;
    const int byi = blockIdx.x / a.bx;
    const int px = bxi * 16 + (wv & 1) * 8 + (ln & 7);
    const int py = byi * 16 + (wv >> 1) * 8 + (ln >> 3);
    if (px >= a.W || py >= a.H) return;
    const float sx = (float)(2 * px + 1 - a.W) / (float)a.W;
    const float sy = (float)(a.H - 2 * py - 1) / (float)a.H;
    const float dx = a.frame[3] + sx * a.frame[6] + sy * a.frame[9];
    const float dy = a.frame[4] + sx * a.frame[7] + sy * a.frame[10];
    const float dz = a.frame[5] + sx * a.frame[8] + sy * a.frame[11];
    Ray r;
    if (!setup_ray(a.frame[0], a.frame[1], a.frame[2], dx, dy, dz, r)) return;
    FusionVisitor vis{a.values, a.acc, a.f, s_obs[wv], ln};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vis.o[c] = r.o[c];
        vis.d[c] = r.d[c];
    }
    sh9(r.d[0], r.d[1], r.d[2], vis.Y);
    vis.T = 1.0f;
    vis.tau = a.tau;
    vis.sigma_scale = a.tree.sigma_scale;
    walk(a.tree, r, s_stack + threadIdx.x, vis);
}

// Eq. 3-5 for every observed leaf, then clear its accumulator.
__global__ __launch_bounds__(kBlock) void fusion_apply_kernel(float4* values, float* weight, int32_t* count,
                                                              float4* acc, int64_t n)
{
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n) return;
    float4* A4 = acc + l * (FPO_FUSION_ACC / 4);
    const float len = A4[7].y;                       // acc[29]
    if (!(len > 0.0f)) return;
    float A[FPO_FUSION_ACC];
    float V[32];
    float4* V4 = values + l * 8;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        const float4 x = A4[w];
        A[4 * w] = x.x; A[4 * w + 1] = x.y; A[4 * w + 2] = x.z; A[4 * w + 3] = x.w;
        const float4 y = V4[w];
        V[4 * w] = y.x; V[4 * w + 1] = y.y; V[4 * w + 2] = y.z; V[4 * w + 3] = y.w;
    }
    const float inv = 1.0f / len;
    const float Ti = A[0] * inv;                     // length-weighted mean transmittance
    const float Wp = weight[l];
    const float den = 1.0f / (Wp + Ti);
    V[0] = fmaf(Wp, V[0], A[1] * inv) * den;                                  // Eq. 3
#pragma unroll
    for (int q = 0; q < 27; ++q) V[1 + q] = fmaf(Wp, V[1 + q], A[2 + q] * inv) * den;   // Eq. 4
    const int32_t C = count[l] + 1;                                             // Eq. 5
    count[l] = C;
    weight[l] = (float)(C - 1) / (float)C * Wp + Ti / (float)C;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        V4[w] = make_float4(V[4 * w], V[4 * w + 1], V[4 * w + 2], V[4 * w + 3]);
        A4[w] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

}  // namespace dev
}  // namespace fpo

using namespace fpo;

extern "C" fpo_status fpo_fusion_observe(const fpo_tree_view* tree, const float* values, const fpo_camera* cam,
                                         const fpo_field* field, float tau, float* acc, void* stream)
{
    ApiRange api_range_("fpo_fusion_observe");
    fpo_status st = check_tree(tree, false, true);
    if (st != FPO_OK) return st;
    if (!values || !acc) return fail(FPO_E_INVALID, "NULL device pointer");
    if (!cam || !field) return fail(FPO_E_INVALID, "NULL camera or field");
    if (!(tau > 0.0f && tau < 1.0f)) return fail(FPO_E_INVALID, "tau must be in (0, 1)");
    if (field->n_gauss < 0 || field->n_gauss > FPO_FIELD_MAX_GAUSS)
        return fail(FPO_E_INVALID, "field n_gauss must be in 0..FPO_FIELD_MAX_GAUSS");
    dev::FusionLaunch a;
    std::memset(&a, 0, sizeof(a));
    if ((st = camera_frame(*cam, a.frame)) != FPO_OK) return st;
    if ((int64_t)cam->width * cam->height > (1ll << 30)) return fail(FPO_E_INVALID, "image too large");
    for (int g = 0; g < field->n_gauss; ++g) {
        const float w = field->w[g];
        if (!(w > 0.0f) || !std::isfinite(w)) return fail(FPO_E_INVALID, "field widths must be positive");
        for (int c = 0; c < 3; ++c) a.f.mu[g][c] = field->mu[g][c];
        a.f.inv2w2[g] = (float)(1.0 / (2.0 * (double)w * (double)w));
        a.f.a[g] = field->a[g];
    }
    a.f.n = field->n_gauss;
    std::memcpy(a.f.u, field->u, sizeof(a.f.u));
    std::memcpy(a.f.v, field->v, sizeof(a.f.v));
    std::memcpy(a.f.b, field->b, sizeof(a.f.b));
    a.tree = dev::tree_dev(tree);
    a.values = values;
    a.acc = acc;
    a.W = cam->width;
    a.H = cam->height;
    a.bx = (cam->width + 15) / 16;
    a.tau = tau;
    const int64_t grid = (int64_t)a.bx * ((cam->height + 15) / 16);
    hipLaunchKernelGGL(dev::fusion_observe_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return launch_status("fpo_fusion_observe");
}

extern "C" fpo_status fpo_fusion_apply(float* values, float* weight, int32_t* count, float* acc, int64_t n_leaves,
                                       void* stream)
{
    ApiRange api_range_("fpo_fusion_apply");
    if (n_leaves < 0) return fail(FPO_E_INVALID, "n_leaves < 0");
    if (n_leaves == 0) return FPO_OK;
    if (!values || !weight || !count || !acc) return fail(FPO_E_INVALID, "NULL device pointer");
    if (((reinterpret_cast<uintptr_t>(values)) | (reinterpret_cast<uintptr_t>(acc))) & 15)
        return fail(FPO_E_INVALID, "values and acc must be 16-byte aligned");
    if (n_leaves > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many leaves");
    const int64_t grid = (n_leaves + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::fusion_apply_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<float4*>(values), weight, count,
                       reinterpret_cast<float4*>(acc), n_leaves);
    return launch_status("fpo_fusion_apply");
}
