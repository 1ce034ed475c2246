// libfpo learned proposal (not part of the paper): training labels from the
// plain walk, the MLP's FP32 training kernels, FP16 fragment packing and the
// matrix-core inference the render's skip pre-pass uses.
//
// Training step for a batch of n rays (fpo_mlp_loss_grad):
//   1. mlp_grad_rays_kernel, one thread per ray: encoding, forward pass,
//      loss, dL/d(outputs) and the back-propagated hidden-layer deltas; the
//      per-ray vectors every weight gradient needs go to a feature-major
//      workspace (row f, column ray).
//   2. mlp_wgrad_kernel: dW = sum over rays of input (x) delta, one thread per
//      weight, tiles of 16 x 16 weights x 1024 rays staged through LDS; one
//      partial sum per ray split.
//   3. mlp_reduce_kernel: the splits summed in a fixed order (deterministic)
//      into the gradient, and the per-ray losses into the batch loss.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"
#include "fpo_proposal.h"

namespace fpo {
namespace dev {

// ---------------------------------------------------------------------------
// Labels
// ---------------------------------------------------------------------------
template <int MODE>
struct LabelVisitor {
    const TreeDev& T;
    const float* b;
    const void* snap;
    float Tr;
    float stop_T;
    float t_first, t_last;
    bool hit;

    __device__ inline bool segment(int leaf, float t0, float t1)
    {
        const float delta = t1 - t0;
        float sraw;
        if constexpr (MODE >= 16) {
            float v[32];
            sraw = SnapEval<MODE - 16>::sigma(snap, leaf, v);
        } else {
            float k[LeafEval<MODE>::kSigmaWords * LeafEval<MODE>::W];
            float scale;
            sraw = LeafEval<MODE>::sigma(T, leaf, b, k, scale);
        }
        const float sig = T.sigma_scale * fmaxf(sraw, 0.0f);
        if (!(sig * delta > 0.0f)) return false;
        if (!hit) t_first = t0;
        hit = true;
        t_last = t1;
        Tr *= __expf(-sig * delta);
        return Tr < stop_T;
    }
};

struct LabelLaunch {
    TreeDev tree;
    const float* o;
    const float* d;
    const int32_t* t_idx;
    const float* basis;
    const float* tau;
    const void* snap;
    int64_t snap_stride;
    int64_t n;
    int32_t n_t;
    float stop_T;
    float* labels;
    float* inputs;
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void labels_kernel(LabelLaunch a)
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
    LabelVisitor<MODE> lv{a.tree, b, snap, 1.0f, a.stop_T, 0.0f, 0.0f, false};
    const float ox = a.o[3 * r_id], oy = a.o[3 * r_id + 1], oz = a.o[3 * r_id + 2];
    Ray r;
    float x[kMlpIn];
    float len = 1.0f;
    if (setup_ray(ox, oy, oz, a.d[3 * r_id], a.d[3 * r_id + 1], a.d[3 * r_id + 2], r)) {
        len = r.t_len;
        walk(a.tree, r, s_stack + threadIdx.x, lv);
        proposal_inputs(r, a.tau[ti], x);
    } else {
        // no chord: origin and normalised direction
        const float dx = a.d[3 * r_id], dy = a.d[3 * r_id + 1], dz = a.d[3 * r_id + 2];
        const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
        x[0] = ox; x[1] = oy; x[2] = oz;
        x[3] = dx * inv; x[4] = dy * inv; x[5] = dz * inv;
        x[6] = a.tau[ti];
    }
    a.labels[3 * r_id] = lv.hit ? 1.0f : 0.0f;
    a.labels[3 * r_id + 1] = lv.hit ? lv.t_first / len : 0.0f;
    a.labels[3 * r_id + 2] = lv.hit ? lv.t_last / len : 0.0f;
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) a.inputs[kMlpIn * r_id + c] = x[c];
}

// ---------------------------------------------------------------------------
// FP32 training kernels
// ---------------------------------------------------------------------------
constexpr int kRowG = 0;                 // encoded inputs, 84 rows
constexpr int kRowA1 = kRowG + kMlpPE;   // hidden activations of layer 1
constexpr int kRowA2 = kRowA1 + kMlpH;   // of layer 2
constexpr int kRowD1 = kRowA2 + kMlpH;   // deltas of layer 1 pre-activations
constexpr int kRowD2 = kRowD1 + kMlpH;   // of layer 2
constexpr int kRowGO = kRowD2 + kMlpH;   // dL/d(outputs), 3 rows
constexpr int kRowLoss = kRowGO + 3;     // per-ray loss
constexpr int kRows = kRowLoss + 1;
constexpr int kChunk = 64;               // rays per LDS stage of the weight gradient
constexpr int kSplit = 1024;             // rays per partial sum
constexpr int kParamsPad = FPO_MLP_N_PARAMS_PADDED;
constexpr float kQIn = 0.1f;
constexpr float kQOut = 0.9f;

__device__ inline void encode_f32(const float* x, float* g)
{
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c)
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const float a = x[c] * (float)(1 << f);
            g[12 * c + 2 * f] = sinpif(a);
            g[12 * c + 2 * f + 1] = cospif(a);
        }
}

// Forward pass of one ray in FP32.  Keeps a1 (needed by layer 2) and the
// ReLU masks of both hidden layers.
struct Fwd {
    float a1[kMlpH];
    float a2[kMlpH];
    uint64_t m1, m2;
    float o[3];
};

__device__ inline void forward_f32(const float* __restrict__ P, const float* g, Fwd& F)
{
    float z[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) z[j] = P[kP1 + kMlpPE * kMlpH + j];
#pragma unroll
    for (int k = 0; k < kMlpPE; ++k) {
        const float gk = g[k];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) z[j] = fmaf(gk, P[kP1 + k * kMlpH + j], z[j]);
    }
    F.m1 = 0;
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        F.a1[j] = fmaxf(z[j], 0.0f);
        F.m1 |= (uint64_t)(z[j] > 0.0f) << j;
    }
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) z[j] = P[kP2 + kMlpH * kMlpH + j];
#pragma unroll
    for (int k = 0; k < kMlpH; ++k) {
        const float ak = F.a1[k];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) z[j] = fmaf(ak, P[kP2 + k * kMlpH + j], z[j]);
    }
    F.m2 = 0;
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        F.a2[j] = fmaxf(z[j], 0.0f);
        F.m2 |= (uint64_t)(z[j] > 0.0f) << j;
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) F.o[e] = P[kP3 + kMlpH * 3 + e];
#pragma unroll
    for (int k = 0; k < kMlpH; ++k)
#pragma unroll
        for (int e = 0; e < 3; ++e) F.o[e] = fmaf(F.a2[k], P[kP3 + k * 3 + e], F.o[e]);
}

__global__ __launch_bounds__(kBlock) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                             int64_t n, float* __restrict__ out)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    float x[kMlpIn], g[kMlpPE];
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) x[c] = X[r * kMlpIn + c];
    encode_f32(x, g);
    Fwd F;
    forward_f32(P, g, F);
#pragma unroll
    for (int e = 0; e < 3; ++e) out[r * 3 + e] = F.o[e];
}

__device__ inline float sigmoid_exact(float v) { return 1.0f / (1.0f + expf(-v)); }

// log(1 + u) for u in [0, 1] in FP32 only: with w = 1 + u rounded, the ratio
// u / (w - 1) corrects the rounding of w (Goldberg, "What every computer
// scientist should know about floating-point arithmetic", 1991, Thm. 4), so
// logf(w) suffices; the library's log1pf would bring an FP64 instruction in.
__device__ inline float log1p_unit(float u)
{
    const float w = 1.0f + u;
    return w == 1.0f ? u : logf(w) * (u / (w - 1.0f));
}

__global__ __launch_bounds__(kBlock) void mlp_grad_rays_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                               const float* __restrict__ Y, const int32_t* __restrict__ idx,
                                                               int64_t n, int64_t ld, float inv_n, float* __restrict__ ws)
{
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= ld) return;
    const bool live = r < n;
    if (!live) {
        // padding columns: zero, so that the weight gradient may sum whole chunks
        for (int f = 0; f < kRows; ++f) ws[f * ld + r] = 0.0f;
        return;
    }
    const int64_t row = idx ? (int64_t)idx[r] : r;
    float x[kMlpIn], g[kMlpPE];
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) x[c] = X[row * kMlpIn + c];
    const float y0 = Y[row * 3], y1 = Y[row * 3 + 1], y2 = Y[row * 3 + 2];
    encode_f32(x, g);
#pragma unroll
    for (int k = 0; k < kMlpPE; ++k) ws[(kRowG + k) * ld + r] = g[k];
    Fwd F;
    forward_f32(P, g, F);
#pragma unroll
    for (int k = 0; k < kMlpH; ++k) {
        ws[(kRowA1 + k) * ld + r] = F.a1[k];
        ws[(kRowA2 + k) * ld + r] = F.a2[k];
    }
    // loss and dL/do: logistic loss on the hit logit, pinball on the sigmoid
    // of the interval outputs for rays that hit
    const float o0 = F.o[0];
    float loss = fmaxf(o0, 0.0f) - y0 * o0 + log1p_unit(expf(-fabsf(o0)));
    float go[3];
    go[0] = sigmoid_exact(o0) - y0;
    const bool hit = y0 > 0.5f;
    const float yy[2] = {y1, y2};
    const float qq[2] = {kQIn, kQOut};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float s = sigmoid_exact(F.o[1 + e]);
        const float u = yy[e] - s;
        const float w = qq[e] - (u < 0.0f ? 1.0f : 0.0f);
        loss += hit ? u * w : 0.0f;
        go[1 + e] = hit ? -w * s * (1.0f - s) : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        go[e] *= inv_n;
        ws[(kRowGO + e) * ld + r] = go[e];
    }
    ws[kRowLoss * ld + r] = loss * inv_n;
    // deltas: d2 = (W3 go) . [z2 > 0]; d1 = (W2 d2) . [z1 > 0]
    float d2[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float v = 0.0f;
#pragma unroll
        for (int e = 0; e < 3; ++e) v = fmaf(go[e], P[kP3 + j * 3 + e], v);
        d2[j] = ((F.m2 >> j) & 1) ? v : 0.0f;
        ws[(kRowD2 + j) * ld + r] = d2[j];
    }
    for (int k = 0; k < kMlpH; ++k) {
        float v = 0.0f;
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) v = fmaf(d2[j], P[kP2 + k * kMlpH + j], v);
        ws[(kRowD1 + k) * ld + r] = ((F.m1 >> k) & 1) ? v : 0.0f;
    }
}

// Tile table of the weight gradient: (layer, k-tile, j-tile).  Layer L's
// matrix has K_in + 1 rows (the last is the bias, input 1) and J columns.
struct WTile {
    int base, J, K1, xrow, drow, kt, jt;
};

__device__ inline WTile wtile(int t)
{
    // layer 1: 6 x 4 tiles, layer 2: 5 x 4, layer 3: 5 x 1
    if (t < 24) return {kP1, kMlpH, kMlpPE + 1, kRowG, kRowD1, t / 4, t % 4};
    if (t < 44) return {kP2, kMlpH, kMlpH + 1, kRowA1, kRowD2, (t - 24) / 4, (t - 24) % 4};
    return {kP3, 3, kMlpH + 1, kRowA2, kRowGO, t - 44, 0};
}
constexpr int kWTiles = 49;

__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float* __restrict__ ws, int64_t ld,
                                                        float* __restrict__ part)
{
    __shared__ float xs[16][kChunk + 1];
    __shared__ float ds[16][kChunk + 1];
    const WTile T = wtile(blockIdx.x);
    const int tk = threadIdx.x >> 4, tj = threadIdx.x & 15;
    const int k = T.kt * 16 + tk, j = T.jt * 16 + tj;
    const int64_t r0 = (int64_t)blockIdx.y * kSplit;
    const int64_t r1 = min(r0 + kSplit, ld);
    float acc = 0.0f;
    for (int64_t c0 = r0; c0 < r1; c0 += kChunk) {
        // stage 16 input rows and 16 delta rows of this chunk
        for (int e = threadIdx.x; e < 16 * kChunk; e += 256) {
            const int rr = e / kChunk, cc = e % kChunk;
            const int kk = T.kt * 16 + rr, jj = T.jt * 16 + rr;
            float xv = 0.0f, dv = 0.0f;
            if (kk < T.K1 - 1) xv = ws[(int64_t)(T.xrow + kk) * ld + c0 + cc];
            else if (kk == T.K1 - 1) xv = 1.0f;
            if (jj < T.J) dv = ws[(int64_t)(T.drow + jj) * ld + c0 + cc];
            xs[rr][cc] = xv;
            ds[rr][cc] = dv;
        }
        __syncthreads();
#pragma unroll 16
        for (int cc = 0; cc < kChunk; ++cc) acc = fmaf(xs[tk][cc], ds[tj][cc], acc);
        __syncthreads();
    }
    if (k < T.K1 && j < T.J) part[(int64_t)blockIdx.y * kParamsPad + T.base + k * T.J + j] = acc;
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part, int n_split,
                                                         const float* __restrict__ loss_row, int64_t ld,
                                                         float* __restrict__ grad, float* __restrict__ loss)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x < gridDim.x - 1) {
        if (i < FPO_MLP_N_PARAMS) {
            float s = 0.0f;
            for (int sp = 0; sp < n_split; ++sp) s += part[(int64_t)sp * kParamsPad + i];
            grad[i] += s;
        }
        return;
    }
    __shared__ float red[256];
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < ld; r += 256) s += loss_row[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] += red[0];
}

// ---------------------------------------------------------------------------
// FP16 fragments and matrix-core inference
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float* __restrict__ P, unsigned char* __restrict__ out)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id < kFrags * 64) {
        const int fi = id / 64, ln = id % 64;
        const int m = ln & 15, q = ln >> 4;
        _Float16 h[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float v = 0.0f;
            if (fi < kFrag2) {                       // A = W1^T: [64 out][96 features]
                const int mt = fi / 6, kb = fi % 6;
                const int row = 16 * mt + m, k = 16 * kb + 4 * q + e;
                if (k < kMlpPE) v = P[kP1 + k * kMlpH + row];
            } else if (fi < kFrag3) {                // A = W2^T
                const int g = fi - kFrag2, mt = g / 4, kb = g % 4;
                const int row = 16 * mt + m, k = 16 * kb + 4 * q + e;
                v = P[kP2 + k * kMlpH + row];
            } else {                                 // A = W3^T, rows 0..2 of 16
                const int kb = fi - kFrag3;
                const int k = 16 * kb + 4 * q + e;
                if (m < 3) v = P[kP3 + k * 3 + m];
            }
            h[e] = (_Float16)v;
        }
        reinterpret_cast<f16x4*>(out)[id] = f16x4{h[0], h[1], h[2], h[3]};
        return;
    }
    const int b = id - kFrags * 64;
    float* bias = reinterpret_cast<float*>(out + kPackedBias);
    if (b < 64) bias[b] = P[kP1 + kMlpPE * kMlpH + b];
    else if (b < 128) bias[b] = P[kP2 + kMlpH * kMlpH + (b - 64)];
    else if (b < 131) bias[b] = P[kP3 + kMlpH * 3 + (b - 128)];
    else if (b == 131) bias[b] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void mlp_infer_kernel(const unsigned char* __restrict__ packed,
                                                           const float* __restrict__ X, int64_t n,
                                                           float* __restrict__ out)
{
    const int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) & ~(int64_t)63;
    if (base >= n) return;                      // whole waves only
    const int64_t r = base + (threadIdx.x & 63);
    const bool live = r < n;
    float x[kMlpIn];
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) x[c] = live ? X[r * kMlpIn + c] : 0.0f;
    float o[3];
    mlp_infer_wave(reinterpret_cast<const uint2*>(packed), reinterpret_cast<const float*>(packed + kPackedBias), x, o);
    if (live)
#pragma unroll
        for (int e = 0; e < 3; ++e) out[r * 3 + e] = o[e];
}

}  // namespace dev
}  // namespace fpo

using namespace fpo;

static int64_t mlp_ld(int64_t n) { return (n + dev::kChunk - 1) / dev::kChunk * dev::kChunk; }
static int64_t mlp_splits(int64_t n) { return (mlp_ld(n) + dev::kSplit - 1) / dev::kSplit; }

extern "C" int64_t fpo_mlp_workspace_floats(int64_t n)
{
    ApiRange api_range_("fpo_mlp_workspace_floats");
    if (n < 1) return 0;
    return (int64_t)dev::kRows * mlp_ld(n) + mlp_splits(n) * dev::kParamsPad;
}

template <int MODE>
static void launch_labels(const dev::LabelLaunch& a, int64_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(dev::labels_kernel<MODE>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s, a);
}

extern "C" fpo_status fpo_ray_labels(const fpo_tree_view* tree, const float* o, const float* d, const int32_t* t_idx,
                                     const float* basis, const float* tau, int32_t n_t, int64_t n_rays,
                                     const fpo_render_opts* opts, float* labels, float* inputs, void* stream)
{
    ApiRange api_range_("fpo_ray_labels");
    fpo_status st = check_tree(tree, opts == nullptr || opts->snapshot == nullptr);
    if (st != FPO_OK) return st;
    if ((st = check_opts(opts, tree)) != FPO_OK) return st;
    if (n_rays < 0) return fail(FPO_E_INVALID, "n_rays < 0");
    if (n_rays == 0) return FPO_OK;
    if (!o || !d || !t_idx || !basis || !tau || !labels || !inputs) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (n_rays > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many rays");
    dev::LabelLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.tree = dev::tree_dev(tree);
    a.o = o; a.d = d; a.t_idx = t_idx; a.basis = basis; a.tau = tau; a.n_t = n_t; a.n = n_rays;
    a.snap = opts->snapshot;
    a.snap_stride = opts->snapshot_cam_stride;
    a.stop_T = opts->stop_T;
    a.labels = labels;
    a.inputs = inputs;
    const int64_t grid = (n_rays + dev::kBlock - 1) / dev::kBlock;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int mode = opts->snapshot ? 16 + (int)opts->snapshot_dtype : (int)tree->dtype;
    switch (mode) {
        case FPO_F32: launch_labels<FPO_F32>(a, grid, s); break;
        case FPO_BF16: launch_labels<FPO_BF16>(a, grid, s); break;
        case FPO_FP8_E4M3: launch_labels<FPO_FP8_E4M3>(a, grid, s); break;
        case dev::kSnapF32: launch_labels<dev::kSnapF32>(a, grid, s); break;
        case dev::kSnapBF16: launch_labels<dev::kSnapBF16>(a, grid, s); break;
        default: return fail(FPO_E_INVALID, "unknown render mode");
    }
    return launch_status("fpo_ray_labels");
}

extern "C" fpo_status fpo_mlp_forward(const float* params, const float* inputs, int64_t n, float* out, void* stream)
{
    ApiRange api_range_("fpo_mlp_forward");
    if (n < 0) return fail(FPO_E_INVALID, "n < 0");
    if (n == 0) return FPO_OK;
    if (!params || !inputs || !out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "n too large");
    const int64_t grid = (n + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::mlp_forward_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0,
                       static_cast<hipStream_t>(stream), params, inputs, n, out);
    return launch_status("fpo_mlp_forward");
}

extern "C" fpo_status fpo_mlp_loss_grad(const float* params, const float* inputs, const float* labels,
                                        const int32_t* idx, int64_t n, float* workspace, float* grad, float* loss,
                                        void* stream)
{
    ApiRange api_range_("fpo_mlp_loss_grad");
    if (n < 1) return fail(FPO_E_INVALID, "n must be >= 1");
    if (!params || !inputs || !labels || !workspace || !grad || !loss) return fail(FPO_E_INVALID, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(workspace) & 15) != 0) return fail(FPO_E_INVALID, "workspace must be 16-byte aligned");
    const int64_t ld = mlp_ld(n);
    const int64_t n_split = mlp_splits(n);
    if (ld > (int64_t)1 << 30) return fail(FPO_E_INVALID, "batch too large");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* part = workspace + (int64_t)dev::kRows * ld;
    const int64_t g1 = (ld + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::mlp_grad_rays_kernel, dim3((unsigned)g1), dim3(dev::kBlock), 0, s, params, inputs, labels,
                       idx, n, ld, 1.0f / (float)n, workspace);
    fpo_status st = launch_status("fpo_mlp_loss_grad (rays)");
    if (st != FPO_OK) return st;
    hipLaunchKernelGGL(dev::mlp_wgrad_kernel, dim3(dev::kWTiles, (unsigned)n_split), dim3(256), 0, s, workspace, ld, part);
    if ((st = launch_status("fpo_mlp_loss_grad (weights)")) != FPO_OK) return st;
    const int g3 = (FPO_MLP_N_PARAMS + 255) / 256 + 1;
    hipLaunchKernelGGL(dev::mlp_reduce_kernel, dim3(g3), dim3(256), 0, s, part, (int)n_split,
                       workspace + (int64_t)dev::kRowLoss * ld, ld, grad, loss);
    return launch_status("fpo_mlp_loss_grad (reduce)");
}

extern "C" fpo_status fpo_mlp_pack(const float* params, void* packed_out, void* stream)
{
    ApiRange api_range_("fpo_mlp_pack");
    if (!params || !packed_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(packed_out) & 15) != 0) return fail(FPO_E_INVALID, "packed_out must be 16-byte aligned");
    const int n = dev::kFrags * 64 + 132;
    hipLaunchKernelGGL(dev::mlp_pack_kernel, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                       params, static_cast<unsigned char*>(packed_out));
    return launch_status("fpo_mlp_pack");
}

extern "C" fpo_status fpo_mlp_infer(const void* packed, const float* inputs, int64_t n, float* out, void* stream)
{
    ApiRange api_range_("fpo_mlp_infer");
    if (n < 0) return fail(FPO_E_INVALID, "n < 0");
    if (n == 0) return FPO_OK;
    if (!packed || !inputs || !out) return fail(FPO_E_INVALID, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(packed) & 15) != 0) return fail(FPO_E_INVALID, "packed must be 16-byte aligned");
    if (n > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "n too large");
    const int64_t grid = (n + dev::kBlock - 1) / dev::kBlock;
    hipLaunchKernelGGL(dev::mlp_infer_kernel, dim3((unsigned)grid), dim3(dev::kBlock), 0, static_cast<hipStream_t>(stream),
                       static_cast<const unsigned char*>(packed), inputs, n, out);
    return launch_status("fpo_mlp_infer");
}
