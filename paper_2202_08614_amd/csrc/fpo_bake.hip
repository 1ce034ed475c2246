// libfpo precision entry points: per-leaf-scaled BF16 / FP8 (E4M3FN)
// quantisation of the coefficient store, and the MFMA time bake.
//
// Bake (Eq. 7 and Eq. 9 evaluated at many times): for every leaf l and time t
//     out[t][0][l]         = s_l * sum_{i<31} B[t][i] q_l[i]
//     out[t][1 + m][l]     = s_l * sum_{i<5}  B[t][i] q_l[31 + 5 m + i],  m < 27
// with B the FP32 basis of Eq. 8 and q_l the stored (dequantised up to the
// scale s_l) coefficients.  Each 16 x 16 (times x leaves) output tile is a
// v_mfma_f32_16x16x16_bf16 contraction.  BF16 operands carry only 8
// significant bits, so every FP32 operand is split exactly into hi + lo BF16
// parts (x = hi + lo + O(2^-16 x)) and the K dimension holds the three
// products hi*hi + lo*hi + hi*lo: for the sigma row K = 3 x 32 = 96
// (6 MFMAs of K = 16), for an SH row K = 3 x 5 = 15 (one MFMA, padded).
// Stored BF16 and FP8 codes are exact in BF16, so their lo part is zero.
// The kernel is bound by the output writes (n_t x 28 values per leaf), not by
// the MFMA pipes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "fpo.h"
#include "fpo_device.h"
#include "fpo_internal.h"

namespace fpo {
namespace dev {

// ---------------------------------------------------------------------------
// quantisation
// ---------------------------------------------------------------------------

// Round-to-nearest-even FP32 -> BF16 bit pattern (finite inputs).
__device__ inline uint32_t f32_to_bf16_rne(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// Round-to-nearest-even FP32 -> OCP E4M3FN code, saturating at 448.
__device__ inline uint32_t f32_to_e4m3_rne(float y)
{
    const uint32_t sign = (__float_as_uint(y) >> 24) & 0x80u;
    const float a = fabsf(y);
    uint32_t code;
    if (!(a < 448.0f)) {
        code = 0x7Eu;
    } else if (a < 0x1p-6f) {                       // subnormal range: steps of 2^-9
        code = (uint32_t)rintf(a * 0x1p9f);          // 0 .. 8 (8 = smallest normal)
    } else {
        int e;
        const float f = frexpf(a, &e);               // a = f 2^e, f in [0.5, 1)
        // a = (1 + m/8) 2^(e-1): m = rint((2f - 1) 8), exact scaling then RNE
        uint32_t m = (uint32_t)rintf((2.0f * f - 1.0f) * 8.0f);
        int be = e - 1 + 7;
        if (m == 8u) { m = 0u; ++be; }
        code = ((uint32_t)be << 3) | m;
        if (code > 0x7Eu) code = 0x7Eu;
    }
    return code | sign;
}

// One thread per leaf: scale = max|k| (BF16) or max|k| / 448 (FP8), 1 for an
// all-zero leaf; code = RNE(k / scale).  Reads the F32 packed planes, writes
// the quantised packed planes and the scale.
template <int DT>
__global__ __launch_bounds__(kBlock) void quantize_kernel(const float4* src, int64_t n_leaves, int64_t stride,
                                                          uint4* dst, float* scale)
{
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= stride) return;
    constexpr int kSrcWords = (FPO_N_COEFF + 3) / 4;     // 42
    constexpr int W = Pack<DT>::W;                        // 8 or 16 codes per word
    constexpr int kDstWords = (FPO_N_COEFF + W - 1) / W;
    if (l >= n_leaves) {
        for (int g = 0; g < kDstWords; ++g) dst[(int64_t)g * stride + l] = make_uint4(0, 0, 0, 0);
        scale[l] = 1.0f;
        return;
    }
    float mx = 0.0f;
    for (int g = 0; g < kSrcWords; ++g) {
        const float4 w = src[(int64_t)g * stride + l];
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(w.x), fabsf(w.y)), fmaxf(fabsf(w.z), fabsf(w.w))));
    }
    float s = (DT == FPO_BF16) ? mx : mx / 448.0f;
    if (mx == 0.0f) s = 1.0f;
    scale[l] = s;
    for (int g = 0; g < kDstWords; ++g) {
        uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const int q = g * W + e;
            float x = 0.0f;
            if (q < FPO_N_COEFF) {
                const float4 w = src[(int64_t)(q >> 2) * stride + l];
                const float c[4] = {w.x, w.y, w.z, w.w};
                x = c[q & 3];
            }
            const float y = x / s;
            if (DT == FPO_BF16) {
                v[e >> 1] |= f32_to_bf16_rne(y) << (16 * (e & 1));
            } else {
                v[e >> 2] |= f32_to_e4m3_rne(y) << (8 * (e & 3));
            }
        }
        dst[(int64_t)g * stride + l] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// ---------------------------------------------------------------------------
// MFMA bake
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Exact split x = hi + lo (+ residual of relative size 2^-16): hi is x
// truncated to BF16, lo the BF16 rounding of the remainder.
__device__ inline void split_bf16(float x, uint16_t& hi, uint16_t& lo)
{
    const uint32_t hb = __float_as_uint(x) & 0xFFFF0000u;
    hi = (uint16_t)(hb >> 16);
    lo = (uint16_t)f32_to_bf16_rne(x - __uint_as_float(hb));
}

constexpr int kBakeLeaves = 16;           // leaves per wave (one MFMA N tile)
constexpr int kBakeWaves = kBlock / kWave;
constexpr int kKSig = 96;                 // 3 x 32
constexpr int kKZ = 16;                   // 3 x 5, padded

struct BakeLaunch {
    TreeDev tree;
    const float* basis;    // [n_t][32]
    int32_t n_t;
    int32_t dtype;         // coefficient store dtype
    int32_t out_bf16;
    int64_t n_leaves;
    void* out;             // [n_t][28][stride]
};

// Coefficients of the wave's 16 leaves as BF16 hi / lo, [leaf][168].
struct BakeLds {
    uint16_t hi[kBakeWaves][kBakeLeaves][168];
    uint16_t lo[kBakeWaves][kBakeLeaves][168];
    uint16_t bhi[16][32];   // basis of the current 16-time tile
    uint16_t blo[16][32];
};

template <int DT>
__device__ inline void stage_leaf_coeffs(const BakeLaunch& a, BakeLds& L, int wv, int ln, int64_t leaf0)
{
    constexpr int W = Pack<DT>::W;
    constexpr int kWords = (FPO_N_COEFF + W - 1) / W;
    // lane -> (leaf, word) pairs; 16 leaves x kWords words
    for (int idx = ln; idx < kBakeLeaves * kWords; idx += kWave) {
        const int li = idx % kBakeLeaves;
        const int g = idx / kBakeLeaves;
        const int64_t leaf = leaf0 + li;
        float v[W];
        if (leaf < a.n_leaves) {
            const uint4 w = a.tree.planes[(int64_t)g * a.tree.stride + leaf];
            Pack<DT>::unpack(w, v);
        } else {
#pragma unroll
            for (int e = 0; e < W; ++e) v[e] = 0.0f;
        }
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const int q = g * W + e;
            if (q < 168) {
                uint16_t h, l;
                split_bf16(q < FPO_N_COEFF ? v[e] : 0.0f, h, l);
                L.hi[wv][li][q] = h;
                L.lo[wv][li][q] = l;
            }
        }
    }
}

__device__ inline void store_tile(const BakeLaunch& a, const f32x4& acc, int row, int t0, int ln, int64_t leaf0,
                                  float s)
{
    const int64_t leaf = leaf0 + (ln & 15);
    if (leaf >= a.n_leaves) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = t0 + 4 * (ln >> 4) + r;
        if (t >= a.n_t) continue;
        const float v = acc[r] * s;
        const int64_t off = ((int64_t)t * FPO_N_BAKED + row) * a.tree.stride + leaf;
        if (a.out_bf16)
            static_cast<uint16_t*>(a.out)[off] = (uint16_t)f32_to_bf16_rne(v);
        else
            static_cast<float*>(a.out)[off] = v;
    }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void bake_kernel(BakeLaunch a)
{
    __shared__ BakeLds L;
    const int wv = threadIdx.x / kWave;
    const int ln = threadIdx.x % kWave;
    const int64_t leaf0 = ((int64_t)blockIdx.x * kBakeWaves + wv) * kBakeLeaves;
    stage_leaf_coeffs<DT>(a, L, wv, ln, leaf0);
    const int64_t my_leaf = leaf0 + (ln & 15);
    float s = 1.0f;
    if (DT != FPO_F32 && my_leaf < a.n_leaves) s = a.tree.scale[my_leaf];
    const int n = ln & 15;      // MFMA row of A / column of B and D
    const int kg = ln >> 4;     // k group: k = 4 kg .. 4 kg + 3

    for (int t0 = 0; t0 < a.n_t; t0 += 16) {
        __syncthreads();
        // basis tile for times t0 .. t0 + 15, split into hi / lo
        for (int idx = threadIdx.x; idx < 16 * 32; idx += kBlock) {
            const int tt = idx / 32, i = idx % 32;
            const float v = (t0 + tt < a.n_t) ? a.basis[(int64_t)(t0 + tt) * FPO_BASIS_STRIDE + i] : 0.0f;
            uint16_t h, l;
            split_bf16(i < FPO_N_SIGMA ? v : 0.0f, h, l);
            L.bhi[tt][i] = h;
            L.blo[tt][i] = l;
        }
        __syncthreads();

        // sigma row: K = [hi | lo | hi] (basis) x [hi ; hi ; lo] (coefficients)
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < kKSig / 16; ++kk) {
            bf16x4 av, bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = kk * 16 + 4 * kg + e;       // 0 .. 95
                const int part = k / 32, i = k % 32;
                av[e] = (short)(part == 1 ? L.blo[n][i] : L.bhi[n][i]);
                bv[e] = (short)(part == 2 ? L.lo[wv][n][i] : L.hi[wv][n][i]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
        store_tile(a, acc, 0, t0, ln, leaf0, s);

        // SH rows: K = 15 (+1 padding) per row
        bf16x4 az;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * kg + e;                       // 0 .. 15
            const int part = k / 5, i = k % 5;
            az[e] = (short)(k >= 15 ? 0 : (part == 1 ? L.blo[n][i] : L.bhi[n][i]));
        }
        for (int m = 0; m < 27; ++m) {
            bf16x4 bz;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 4 * kg + e;
                const int part = k / 5, i = k % 5;
                const int q = FPO_N_SIGMA + FPO_N_SH_FOURIER * m + i;
                bz[e] = (short)(k >= 15 ? 0 : (part == 2 ? L.lo[wv][n][q] : L.hi[wv][n][q]));
            }
            f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
            z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(az, bz, z, 0, 0, 0);
            store_tile(a, z, 1 + m, t0, ln, leaf0, s);
        }
    }
}

}  // namespace dev
}  // namespace fpo

using namespace fpo;

extern "C" fpo_status fpo_quantize(const float* coeffs, int64_t n_leaves, int64_t leaf_stride, fpo_dtype dtype,
                                   void* q_out, float* scale_out, void* stream)
{
    if (!coeffs || !q_out || !scale_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (dtype != FPO_BF16 && dtype != FPO_FP8_E4M3) return fail(FPO_E_INVALID, "dtype must be BF16 or FP8_E4M3");
    if (n_leaves < 1 || leaf_stride < n_leaves) return fail(FPO_E_INVALID, "bad n_leaves / leaf_stride");
    if (leaf_stride > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many leaves");
    const int64_t grid = (leaf_stride + dev::kBlock - 1) / dev::kBlock;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == FPO_BF16)
        hipLaunchKernelGGL(dev::quantize_kernel<FPO_BF16>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s,
                           reinterpret_cast<const float4*>(coeffs), n_leaves, leaf_stride,
                           static_cast<uint4*>(q_out), scale_out);
    else
        hipLaunchKernelGGL(dev::quantize_kernel<FPO_FP8_E4M3>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s,
                           reinterpret_cast<const float4*>(coeffs), n_leaves, leaf_stride,
                           static_cast<uint4*>(q_out), scale_out);
    return launch_status("fpo_quantize");
}

extern "C" fpo_status fpo_bake_times(const fpo_tree_view* tree, const float* basis, int32_t n_t,
                                     fpo_dtype out_dtype, void* out, void* stream)
{
    fpo_status st = check_tree(tree, true);
    if (st != FPO_OK) return st;
    if (!basis || !out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (out_dtype != FPO_F32 && out_dtype != FPO_BF16) return fail(FPO_E_INVALID, "out_dtype must be F32 or BF16");
    const int64_t per_block = (int64_t)dev::kBakeWaves * dev::kBakeLeaves;
    const int64_t grid = (tree->n_leaves + per_block - 1) / per_block;
    if (grid > INT32_MAX) return fail(FPO_E_INVALID, "too many leaves");
    dev::BakeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.tree = dev::tree_dev(tree);
    a.basis = basis;
    a.n_t = n_t;
    a.dtype = tree->dtype;
    a.out_bf16 = out_dtype == FPO_BF16;
    a.n_leaves = tree->n_leaves;
    a.out = out;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (tree->dtype) {
        case FPO_F32:
            hipLaunchKernelGGL(dev::bake_kernel<FPO_F32>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s, a);
            break;
        case FPO_BF16:
            hipLaunchKernelGGL(dev::bake_kernel<FPO_BF16>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s, a);
            break;
        default:
            hipLaunchKernelGGL(dev::bake_kernel<FPO_FP8_E4M3>, dim3((unsigned)grid), dim3(dev::kBlock), 0, s, a);
            break;
    }
    return launch_status("fpo_bake_times");
}
