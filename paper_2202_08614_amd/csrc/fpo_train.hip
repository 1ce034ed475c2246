// libfpo fine-tuning entry points (Sec. 4.3): the backward pass of the
// render into the leaf Fourier coefficients, the L2 photometric loss of
// Eq. 13 and a fused Adam update over the coefficient planes.
//
// Backward: per ray, the forward walk is recomputed, or, when the forward
// recorded its segments (FPO_RAYS_RECORD), each recorded segment is taken on
// its own; besides the records, the only forward state used is the ray's
// final colour.  Walking
// front to back with transmittance T_i and accumulated colour A_i, the
// suffix R_i = C - A_i gives
//     dL/dsigma_i = delta_i * sum_c g_c (T_{i+1} c_{i,c} - R_{i,c}),
//     dL/dh_{i,c} = g_c T_i alpha_i c_{i,c} (1 - c_{i,c}),
// and through Eq. 7 / Eq. 9 and the SH basis of Eq. 1
//     dL/dk^sigma_q     = s [sigma_raw > 0] dL/dsigma_i b_q,
//     dL/dk^z_{c,j,i}   = dL/dh_{i,c} Y_j b_i.
// One wave per ray (or, from records, per segment): each lane owns up to three
// of a leaf's 166 coefficients, so every sample's gradients go out as three
// coalesced FP32 atomic adds into records laid out like the F32 coefficient
// store.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"

namespace fpo {
namespace dev {

struct BackwardLaunch {
    TreeDev tree;
    const float* o;
    const float* d;
    const int32_t* t_idx;
    const float* basis;
    int64_t n;
    int32_t n_t;
    const float* rgb_fwd;
    const float* grad_rgb;
    float* grad;
    float stop_T;
    const int32_t* rec_count;   // segment records of the forward (FPO_RAYS_RECORD)
    const float4* rec;
    int32_t rec_cap;
};

// Waves per ray when the forward recorded its segments.
constexpr int kRecGroups = 8;

// The backward, one ray per wave.
__global__ __launch_bounds__(kBlock) void render_backward_wave_kernel(BackwardLaunch a)
{
    __shared__ int s_stack[kStackLevels * kBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t r_id = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (r_id >= a.n) return;
    const int ti = min(max(a.t_idx[r_id], 0), a.n_t - 1);
    WaveShade<true> sh{a.tree};
    sh.lane = lane;
    sh.Tr = 1.0f;
    sh.stop_T = a.stop_T;
    sh.grad = a.grad;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sh.C[c] = 0.0f;
        sh.Cf[c] = a.rgb_fwd[r_id * 3 + c];
        sh.g[c] = a.grad_rgb[r_id * 3 + c];
    }
    if (sh.g[0] == 0.0f && sh.g[1] == 0.0f && sh.g[2] == 0.0f) return;
    Ray r;
    if (setup_ray_in(a.tree.box_lo, a.tree.box_hi, a.o[3 * r_id], a.o[3 * r_id + 1], a.o[3 * r_id + 2],
                  a.d[3 * r_id], a.d[3 * r_id + 1], a.d[3 * r_id + 2], r)) {
        float Y[FPO_N_SH];
        sh9(r.d[0], r.d[1], r.d[2], Y);
        sh.sl.init(lane, a.basis + (int64_t)ti * FPO_BASIS_STRIDE, Y);
        walk<true>(a.tree, r, s_stack + threadIdx.x, sh);
    }
}

// The backward from segment records: wave (r, q) takes ray r's recorded
// segments q, q + 8, ...; each already carries the transmittance and the
// colour accumulated in front of it, so no walk is needed and the segments of
// one ray run side by side.  A ray whose records overflowed is walked again by
// its wave q = 0.
__global__ __launch_bounds__(kBlock) void render_backward_rec_kernel(BackwardLaunch a)
{
    __shared__ int s_stack[kStackLevels * kBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w_id = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t r_id = w_id / kRecGroups;
    const int q = (int)(w_id - r_id * kRecGroups);
    if (r_id >= a.n) return;
    int cnt = a.rec_count[r_id];
    if (cnt > a.rec_cap) cnt = -1;       // not a count the forward writes: walk the ray instead
    if (cnt < 0 ? q != 0 : q >= cnt) return;
    WaveShade<true> sh{a.tree};
    sh.lane = lane;
    sh.Tr = 1.0f;
    sh.stop_T = a.stop_T;
    sh.grad = a.grad;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sh.C[c] = 0.0f;
        sh.Cf[c] = a.rgb_fwd[r_id * 3 + c];
        sh.g[c] = a.grad_rgb[r_id * 3 + c];
    }
    if (sh.g[0] == 0.0f && sh.g[1] == 0.0f && sh.g[2] == 0.0f) return;
    Ray r;
    if (!setup_ray_in(a.tree.box_lo, a.tree.box_hi, a.o[3 * r_id], a.o[3 * r_id + 1], a.o[3 * r_id + 2],
                   a.d[3 * r_id], a.d[3 * r_id + 1], a.d[3 * r_id + 2], r))
        return;
    const int ti = min(max(a.t_idx[r_id], 0), a.n_t - 1);
    float Y[FPO_N_SH];
    sh9(r.d[0], r.d[1], r.d[2], Y);
    sh.sl.init(lane, a.basis + (int64_t)ti * FPO_BASIS_STRIDE, Y);
    if (cnt < 0) {
        walk<true>(a.tree, r, s_stack + threadIdx.x, sh);
        return;
    }
    const float4* rr = a.rec + r_id * a.rec_cap * 2;
    for (int i = q; i < cnt; i += kRecGroups) {
        const float4 x0 = rr[2 * i];
        const float4 x1 = rr[2 * i + 1];
        const int leaf = __float_as_int(x0.x);
        if (leaf < 0 || leaf >= a.tree.n_leaves) continue;   // only the forward's leaves are read
        float A[3] = {x0.w, x1.x, x1.y};
        float e;
        sh.prefetch(leaf);
        sh.shade(leaf, x0.y, x0.z, A, e);
    }
}

// Mean over rays of the squared RGB error against target pixels, and its
// gradient: loss += sum_c (rgb - target)^2 / n, grad = 2 (rgb - target) / n.
__global__ __launch_bounds__(kBlock) void l2_loss_kernel(const float* rgb, const float* images,
                                                         const int32_t* img, const int32_t* py,
                                                         const int32_t* px, int64_t n, int32_t n_img,
                                                         int32_t W, int32_t H, float* grad, float* loss)
{
    __shared__ float s_part[kBlock / kWave];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float part = 0.0f;
    if (r < n) {
        const int ii = min(max(img[r], 0), n_img - 1);
        const int yy = min(max(py[r], 0), H - 1);
        const int xx = min(max(px[r], 0), W - 1);
        const float* tgt = images + (((int64_t)ii * H + yy) * W + xx) * 3;
        const float inv_n = 1.0f / (float)n;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = rgb[r * 3 + c] - tgt[c];
            part = fmaf(e, e, part);
            grad[r * 3 + c] = 2.0f * e * inv_n;
        }
        part *= inv_n;
    }
    // wave reduction, then one atomic per block
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) s += s_part[w];
        unsafeAtomicAdd(loss, s);
    }
}

// Adam (Kingma and Ba 2015) over n floats; the gradient is cleared after use.
// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
// cs: null, or device {c1, c2} written by adam_count_kernel (then c1, c2 are unused).
__global__ __launch_bounds__(kBlock) void adam_kernel(float4* p, float4* g, float4* m, float4* v, int64_t n4,
                                                      float lr, float b1, float b2, float eps, float c1, float c2,
                                                      const float* cs)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n4) return;
    if (cs) {
        c1 = cs[0];
        c2 = cs[1];
    }
    float4 pp = p[i], gg = g[i], mm = m[i], vv = v[i];
    float* P = &pp.x;
    float* G = &gg.x;
    float* M = &mm.x;
    float* V = &vv.x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        M[e] = fmaf(b1, M[e], (1.0f - b1) * G[e]);
        V[e] = fmaf(b2, V[e], (1.0f - b2) * G[e] * G[e]);
        const float mh = M[e] * c1;
        const float vh = V[e] * c2;
        P[e] -= lr * mh / (sqrtf(vh) + eps);
    }
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
    g[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Adam on touched records only: one wave per record of rq float4 (rq <= 64).
// A record whose gradient is zero everywhere is skipped as a whole (its
// parameters and moments are left as they are, and its zero gradient needs no
// clearing); the others get the update of adam_kernel.  The wave reads the
// gradient once, and only touched records cost parameter and moment traffic.
__global__ __launch_bounds__(kBlock) void adam_touched_kernel(float4* p, float4* g, float4* m, float4* v,
                                                              int64_t n_rec, int rq, float lr, float b1, float b2,
                                                              float eps, float c1, float c2, const float* cs)
{
    const int64_t rec = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (rec >= n_rec) return;                       // uniform over the wave
    const int lane = threadIdx.x & (kWave - 1);
    const bool in = lane < rq;
    const int64_t i = rec * rq + lane;
    const float4 gg = in ? g[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const bool nz = gg.x != 0.0f || gg.y != 0.0f || gg.z != 0.0f || gg.w != 0.0f;
    if (!__any(nz) || !in) return;
    if (cs) {
        c1 = cs[0];
        c2 = cs[1];
    }
    float4 pp = p[i], mm = m[i], vv = v[i];
    float* P = &pp.x;
    const float* G = &gg.x;
    float* M = &mm.x;
    float* V = &vv.x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        M[e] = fmaf(b1, M[e], (1.0f - b1) * G[e]);
        V[e] = fmaf(b2, V[e], (1.0f - b2) * G[e] * G[e]);
        P[e] -= lr * (M[e] * c1) / (sqrtf(V[e] * c2) + eps);
    }
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
    g[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Step count kept on the device: state = {int32 step, float c1, float c2, 0}.
// One thread advances the step and writes the bias corrections for it, so a
// captured graph that replays this launch and adam_kernel advances by one
// step per replay.  Everything stays in FP32: b is an exact FP32 value, so
// log(b) is the log of the exact argument, and 1 - b^t = -expm1(t log b)
// avoids both the cancellation of forming b^t first and the t-fold rounding
// of a running product; c is within a few FP32 ulps of 1 / (1 - b^t) at every
// step.
__device__ inline float adam_bias_correction(float b, int32_t t)
{
    return 1.0f / -expm1f((float)t * logf(b));
}

__global__ void adam_count_kernel(int32_t* state, float b1, float b2)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int32_t t = state[0] + 1;
    state[0] = t;
    float* cs = reinterpret_cast<float*>(state + 1);
    cs[0] = b1 > 0.0f ? adam_bias_correction(b1, t) : 1.0f;
    cs[1] = b2 > 0.0f ? adam_bias_correction(b2, t) : 1.0f;
}

}  // namespace dev

}  // namespace fpo

using namespace fpo;

extern "C" fpo_status fpo_render_backward(const fpo_tree_view* tree, const float* o, const float* d,
                                          const int32_t* t_idx, const float* basis, int32_t n_t, int64_t n_rays,
                                          const fpo_render_opts* opts, const float* rgb_fwd,
                                          const float* grad_rgb, float* grad_coeffs, void* stream)
{
    ApiRange api_range_("fpo_render_backward");
    fpo_status st = check_tree(tree, true);
    if (st != FPO_OK) return st;
    if ((st = check_opts(opts, tree, false, true)) != FPO_OK) return st;
    if (opts->snapshot) return fail(FPO_E_UNSUPPORTED, "backward runs in Fourier mode only");
    if (tree->dtype != FPO_F32) return fail(FPO_E_UNSUPPORTED, "backward needs the F32 coefficient store");
    if (n_rays < 0) return fail(FPO_E_INVALID, "n_rays < 0");
    if (n_rays == 0) return FPO_OK;
    if (!o || !d || !t_idx || !basis || !rgb_fwd || !grad_rgb || !grad_coeffs)
        return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (n_rays > (int64_t)INT32_MAX * (dev::kBlock / dev::kWave)) return fail(FPO_E_INVALID, "too many rays");
    dev::BackwardLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.tree = dev::tree_dev(tree);
    a.o = o; a.d = d; a.t_idx = t_idx; a.basis = basis; a.n = n_rays; a.n_t = n_t;
    a.rgb_fwd = rgb_fwd; a.grad_rgb = grad_rgb; a.grad = grad_coeffs;
    a.stop_T = opts->stop_T;
    if (opts->flags == FPO_RAYS_RECORD) {
        if (n_rays > dev::kWaveRayBatch)
            return fail(FPO_E_UNSUPPORTED, "FPO_RAYS_RECORD needs at most 32768 rays");
        RecordLayout rl;
        if ((st = record_layout(opts, n_rays, rl)) != FPO_OK) return st;
        a.rec_count = rl.count;
        a.rec = static_cast<const float4*>(rl.records);
        a.rec_cap = rl.cap;
        const int64_t waves = n_rays * dev::kRecGroups;
        const int64_t rgrid = (waves + dev::kBlock / dev::kWave - 1) / (dev::kBlock / dev::kWave);
        hipLaunchKernelGGL(dev::render_backward_rec_kernel, dim3((unsigned)rgrid), dim3(dev::kBlock), 0,
                           static_cast<hipStream_t>(stream), a);
        return launch_status("fpo_render_backward");
    }
    const int64_t wgrid = (n_rays + dev::kBlock / dev::kWave - 1) / (dev::kBlock / dev::kWave);
    hipLaunchKernelGGL(dev::render_backward_wave_kernel, dim3((unsigned)wgrid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return launch_status("fpo_render_backward");
}

extern "C" fpo_status fpo_l2_loss(const float* rgb, const float* images, int32_t n_images, int32_t width,
                                  int32_t height, const int32_t* image_idx, const int32_t* py, const int32_t* px,
                                  int64_t n_rays, float* grad_rgb, float* loss, void* stream)
{
    ApiRange api_range_("fpo_l2_loss");
    if (n_rays < 0) return fail(FPO_E_INVALID, "n_rays < 0");
    if (n_rays == 0) return FPO_OK;
    if (!rgb || !images || !image_idx || !py || !px || !grad_rgb || !loss)
        return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_images < 1 || width < 1 || height < 1) return fail(FPO_E_INVALID, "bad image shape");
    if (n_rays > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rays");
    const int64_t grid = (n_rays + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::l2_loss_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), rgb, images, image_idx, py, px, n_rays, n_images, width,
                       height, grad_rgb, loss);
    return launch_status("fpo_l2_loss");
}

extern "C" fpo_status fpo_adam_step(float* params, float* grad, float* m, float* v, int64_t n, float lr,
                                    float beta1, float beta2, float eps, int32_t step, void* stream)
{
    ApiRange api_range_("fpo_adam_step");
    if (!params || !grad || !m || !v) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n < 0 || n % 4 != 0) return fail(FPO_E_INVALID, "n must be a non-negative multiple of 4");
    if (step < 1) return fail(FPO_E_INVALID, "step counts from 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
        return fail(FPO_E_INVALID, "betas must be in [0, 1)");
    if (!(lr >= 0.0f) || !(eps > 0.0f)) return fail(FPO_E_INVALID, "lr must be >= 0 and eps > 0");
    if ((((uintptr_t)params) | ((uintptr_t)grad) | ((uintptr_t)m) | ((uintptr_t)v)) & 15)
        return fail(FPO_E_INVALID, "buffers must be 16-byte aligned");
    if (n == 0) return FPO_OK;
    const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)step));
    const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)step));
    const int64_t n4 = n / 4;
    if (n4 > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many parameters");
    const int64_t grid = (n4 + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::adam_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<float4*>(params), reinterpret_cast<float4*>(grad), reinterpret_cast<float4*>(m),
                       reinterpret_cast<float4*>(v), n4, lr, beta1, beta2, eps, (float)c1, (float)c2,
                       static_cast<const float*>(nullptr));
    return launch_status("fpo_adam_step");
}

extern "C" fpo_status fpo_adam_step_dev(float* params, float* grad, float* m, float* v, int64_t n, float lr,
                                        float beta1, float beta2, float eps, int32_t* state, void* stream)
{
    ApiRange api_range_("fpo_adam_step_dev");
    if (!params || !grad || !m || !v || !state) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n < 0 || n % 4 != 0) return fail(FPO_E_INVALID, "n must be a non-negative multiple of 4");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
        return fail(FPO_E_INVALID, "betas must be in [0, 1)");
    if (!(lr >= 0.0f) || !(eps > 0.0f)) return fail(FPO_E_INVALID, "lr must be >= 0 and eps > 0");
    if ((((uintptr_t)params) | ((uintptr_t)grad) | ((uintptr_t)m) | ((uintptr_t)v) | ((uintptr_t)state)) & 15)
        return fail(FPO_E_INVALID, "buffers must be 16-byte aligned");
    const int64_t n4 = n / 4;
    if (n4 > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many parameters");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(dev::adam_count_kernel, dim3(1), dim3(dev::kWave), 0, s, state, beta1, beta2);
    if (n4 > 0) {
        const int64_t grid = (n4 + dev::kBlock - 1) / dev::kBlock;
        hipLaunchKernelGGL(dev::adam_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0, s,
                           reinterpret_cast<float4*>(params), reinterpret_cast<float4*>(grad),
                           reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n4, lr, beta1, beta2, eps,
                           0.0f, 0.0f, reinterpret_cast<const float*>(state + 1));
    }
    return launch_status("fpo_adam_step_dev");
}

extern "C" fpo_status fpo_adam_step_touched(float* params, float* grad, float* m, float* v, int64_t n_records,
                                           int32_t record_floats, float lr, float beta1, float beta2, float eps,
                                           int32_t step, int32_t* state, void* stream)
{
    ApiRange api_range_("fpo_adam_step_touched");
    if (!params || !grad || !m || !v) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_records < 0) return fail(FPO_E_INVALID, "n_records < 0");
    if (record_floats < 4 || record_floats % 4 != 0 || record_floats > 4 * dev::kWave)
        return fail(FPO_E_INVALID, "record_floats must be a multiple of 4 in [4, 256]");
    if (!state && step < 1) return fail(FPO_E_INVALID, "step counts from 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
        return fail(FPO_E_INVALID, "betas must be in [0, 1)");
    if (!(lr >= 0.0f) || !(eps > 0.0f)) return fail(FPO_E_INVALID, "lr must be >= 0 and eps > 0");
    if ((((uintptr_t)params) | ((uintptr_t)grad) | ((uintptr_t)m) | ((uintptr_t)v) | ((uintptr_t)state)) & 15)
        return fail(FPO_E_INVALID, "buffers must be 16-byte aligned");
    const int64_t grid = (n_records + dev::kBlock / dev::kWave - 1) / (dev::kBlock / dev::kWave);
    if (grid > (int64_t)INT32_MAX) return fail(FPO_E_INVALID, "too many records");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float c1 = 0.0f, c2 = 0.0f;
    if (state) {
        hipLaunchKernelGGL(dev::adam_count_kernel, dim3(1), dim3(dev::kWave), 0, s, state, beta1, beta2);
    } else {
        c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
        c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    }
    if (n_records == 0) return launch_status("fpo_adam_step_touched");
    hipLaunchKernelGGL(dev::adam_touched_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0, s,
                       reinterpret_cast<float4*>(params), reinterpret_cast<float4*>(grad),
                       reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n_records, record_floats / 4, lr,
                       beta1, beta2, eps, c1, c2, state ? reinterpret_cast<const float*>(state + 1) : nullptr);
    return launch_status("fpo_adam_step_touched");
}
