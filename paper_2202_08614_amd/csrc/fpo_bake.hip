// libfpo precision entry points: per-leaf-scaled BF16 / FP8 (E4M3FN)
// quantisation of the coefficient store, and the MFMA time bake.
//
// Bake (Eq. 7 and Eq. 9 evaluated at many times): for every leaf l and time t
//     out[t][l][0]         = s_l * sum_{i<31} B[t][i] q_l[i]
//     out[t][l][1 + m]     = s_l * sum_{i<5}  B[t][i] q_l[31 + 5 m + i],  m < 27
// with B the FP32 basis of Eq. 8, q_l the stored coefficients and s_l the
// leaf scale (1 for FP32 stores).  A wave takes 16 leaves; for each tile of
// 16 times it forms every output row as a 16 x 16 (times x leaves) tile with
// v_mfma_f32_16x16x4f32 (FP32 operands, FP32 accumulate): the density row
// contracts K = 32 (8 MFMAs), each of the 27 SH rows K = 8 (5 used, 2 MFMAs).
// With all 28 rows of a tile in registers, each lane holds four complete
// (time, leaf) records; a per-wave LDS transpose turns them into whole-line
// stores, so the output (the dominant traffic: n_t x 128 or 64 bytes per
// leaf) streams out in full cache lines.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

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

// One thread per leaf slot: scale = max|k| (BF16) or max|k| / 448 (FP8), 1 for
// an all-zero leaf; code = RNE(k / scale).  Reads the F32 records of the
// layout (n1, n2) twice (the maximum, then the codes word by word, so that
// even 328 coefficients never sit in registers), writes the quantised records
// and the scale.
template <int DT, int N1, int N2>
__global__ __launch_bounds__(kBlock) void quantize_kernel(const float4* src, int64_t n_leaves, int64_t stride,
                                                          uint4* dst, float* scale)
{
    using RS = Rec<FPO_F32, N1, N2>;
    using RQ = Rec<DT, N1, N2>;
    constexpr int kCoeff = RS::kCoeff;
    constexpr int W = Pack<DT>::W;                        // 8 or 16 codes per word
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= stride) return;
    uint4* out = dst + l * RQ::R;
    if (l >= n_leaves) {
        for (int g = 0; g < RQ::R; ++g) out[g] = make_uint4(0, 0, 0, 0);
        scale[l] = 1.0f;
        return;
    }
    const float4* in = src + l * RS::R;
    float mx = 0.0f;
#pragma unroll 4
    for (int g = 0; g < (kCoeff + 3) / 4; ++g) {
        const float4 w = in[g];
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(w.x), fabsf(w.y)), fmaxf(fabsf(w.z), fabsf(w.w))));
    }
    float s = (DT == FPO_BF16) ? mx : mx / 448.0f;
    if (mx == 0.0f) s = 1.0f;
    scale[l] = s;
    for (int g = 0; g < RQ::R; ++g) {
        uint32_t v[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e4 = 0; e4 < W / 4; ++e4) {
            const int q0 = g * W + 4 * e4;
            if (q0 >= kCoeff) break;
            const float4 w = in[q0 / 4];
            const float x[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = 4 * e4 + u;
                if (q0 + u >= kCoeff) continue;
                const float y = x[u] / s;
                if (DT == FPO_BF16)
                    v[e >> 1] |= f32_to_bf16_rne(y) << (16 * (e & 1));
                else
                    v[e >> 2] |= f32_to_e4m3_rne(y) << (8 * (e & 3));
            }
        }
        out[g] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// ---------------------------------------------------------------------------
// MFMA bake
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values -> one word of two BF16 (round to nearest even, one
// v_cvt_pk_bf16_f32 on gfx950; denormals are kept).
__device__ inline uint32_t pack_bf16x2(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

// The density value a snapshot record holds, as FP32: itself for F32
// records, its BF16 rounding (the same RNE conversion) for BF16 records.
template <int OUT_BF16>
__device__ inline float stored_sigma(float v)
{
    if constexpr (OUT_BF16) return __uint_as_float(pack_bf16x2(v, 0.0f) << 16);
    else return v;
}

constexpr int kBakeLeaves = 16;           // leaves per wave group (one MFMA N tile)
constexpr int kBakeWaves = kBlock / kWave;
constexpr int kCoefPad = 169;             // LDS row stride, F32 rows (odd: spreads banks)
constexpr int kCoefPad16 = 170;           // LDS row stride, BF16 rows (85 words: odd)

struct BakeLaunch {
    TreeDev tree;
    const float* basis;    // [n_t][32]
    int32_t n_t;
    int64_t n_leaves;
    void* out;             // [n_t][stride][32] records
    float* sigma;          // [n_t][stride] value 0 of each record as FP32, or null
};

// One wave per group of 16 leaves.  The 16 records (pad words included:
// whole lines) are decoded into LDS rows coef[leaf][q]; for every tile of 16
// times lane (kq, n) feeds A[t0 + n][k] (basis, through the cache) and
// B[k][leaf n] (LDS), ending with D[t0 + 4 kq + r][leaf n] for all 28 rows and
// r < 4: four whole records.  For each r the wave parks its 64 records
// (scaled, and converted when the output is BF16) in LDS as [kq][leaf][word]
// (word w of leaf n at slot w ^ (n & (words - 1)), so that record writes and
// row reads spread over the banks) and writes them back out as 16 consecutive
// records per time: lane L writes word L of each 64-word run, whole lines.
// The waves of a block share nothing and never wait for each other.
template <int DT, int OUT_BF16>
__global__ __launch_bounds__(kBlock, (DT != FPO_F32 && OUT_BF16) ? 3 : 2) void bake_kernel(BakeLaunch a)
{
    constexpr int W = Pack<DT>::W;                            // codes per 16-byte word
    constexpr int R = Pack<DT>::R;                            // words per record
    constexpr int kWords = (FPO_N_COEFF + W - 1) / W;         // words holding the 166 codes
    constexpr int kPf = kBakeLeaves * R / kWave;              // record words per lane
    static_assert(kBakeLeaves * R % kWave == 0, "whole records per wave");
    constexpr int kOut = OUT_BF16 ? 4 : 8;                    // 16-byte words per output record
    constexpr int kRunsPerTime = kOut / 4;                    // 64-word store runs per time row
    // BF16 and FP8 codes are exact in BF16: their rows are kept as BF16 bit
    // patterns, which halves the LDS per wave (three blocks per CU)
    constexpr bool kHalf = DT != FPO_F32;
    constexpr int kPad = kHalf ? kCoefPad16 : kCoefPad;
    using CoefT = std::conditional_t<kHalf, uint16_t, float>;
    __shared__ CoefT coef[kBakeWaves][kBakeLeaves][kPad];
    __shared__ uint4 stage[kBakeWaves][4][kBakeLeaves][kOut];
    auto coef_at = [&](const CoefT* row, int q) -> float {
        if constexpr (kHalf) return __uint_as_float((uint32_t)row[q] << 16);
        else return row[q];
    };
    const int wv = threadIdx.x / kWave;
    const int ln = threadIdx.x % kWave;
    const int n = ln & 15;      // A row (time) / B and D column (leaf)
    const int kq = ln >> 4;     // k index inside a K = 4 step; D rows 4 kq .. 4 kq + 3
    const int64_t grp = (int64_t)blockIdx.x * kBakeWaves + wv;
    if (grp * kBakeLeaves >= a.n_leaves) return;
    const int64_t row = a.tree.stride * kOut;                 // output words per time row
    {
        uint4 pf[kPf];
        const uint4* src = a.tree.recs + grp * kBakeLeaves * R + ln;
        const int n_words = (int)min<int64_t>(kBakeLeaves, a.n_leaves - grp * kBakeLeaves) * R;
#pragma unroll
        for (int p = 0; p < kPf; ++p) pf[p] = p * kWave + ln < n_words ? src[p * kWave] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int p = 0; p < kPf; ++p) {
            const int idx = p * kWave + ln;
            const int li = idx / R;
            const int g = idx - li * R;
            if (g >= kWords) continue;
            float v[W];
            Pack<DT>::unpack(pf[p], v);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int q = g * W + e;
                if (q >= kPad) continue;
                const float x = q < FPO_N_COEFF ? v[e] : 0.0f;
                if constexpr (kHalf) coef[wv][li][q] = (uint16_t)(__float_as_uint(x) >> 16);
                else coef[wv][li][q] = x;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
        const int64_t leaf0 = grp * kBakeLeaves;
        const int64_t my_leaf = leaf0 + n;
        const float s = (DT != FPO_F32 && my_leaf < a.n_leaves) ? a.tree.scale[my_leaf] : 1.0f;
        const int n_valid = (int)min<int64_t>(kBakeLeaves, a.n_leaves - leaf0);
        const CoefT* cf = coef[wv][n];
        uint4* dst = static_cast<uint4*>(a.out) + leaf0 * kOut + ln;

        for (int t0 = 0; t0 < a.n_t; t0 += 16) {
            // re-read the B operands from LDS every tile rather than hold 62
            // of them in registers across the loop
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int ta = t0 + n;
            const bool ta_ok = ta < a.n_t;
            const float* brow = a.basis + (int64_t)(ta_ok ? ta : 0) * FPO_BASIS_STRIDE;
            f32x4 acc[FPO_N_BAKED];
            // density row: K = 32 (k = 31 is padding: zero basis)
            acc[0] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = 4 * kk + kq;
                const float av = (ta_ok && k < FPO_N_SIGMA) ? brow[k] : 0.0f;
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, coef_at(cf, k), acc[0], 0, 0, 0);
            }
            // SH rows: K = 5 (padded to 8)
            const float a0 = ta_ok ? brow[kq] : 0.0f;
            const float a1 = (ta_ok && kq == 0) ? brow[4] : 0.0f;
#pragma unroll
            for (int m = 0; m < FPO_N_BAKED - 1; ++m) {
                const int q = FPO_N_SIGMA + FPO_N_SH_FOURIER * m;
                const float b0 = coef_at(cf, q + kq);
                const float b1 = kq == 0 ? coef_at(cf, q + 4) : 0.0f;
                f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                z = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, z, 0, 0, 0);
                z = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, z, 0, 0, 0);
                acc[1 + m] = z;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v[32];
#pragma unroll
                for (int q = 0; q < 32; ++q) v[q] = q < FPO_N_BAKED ? acc[q][r] * s : 0.0f;
                if (a.sigma) {
                    const int t = t0 + 4 * kq + r;
                    if (t < a.n_t && n < n_valid) a.sigma[t * a.tree.stride + my_leaf] = stored_sigma<OUT_BF16>(v[0]);
                }
                uint4* st = stage[wv][kq][n];
                if constexpr (OUT_BF16) {
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        st[w ^ (n & 3)] = make_uint4(pack_bf16x2(v[8 * w], v[8 * w + 1]),
                                                     pack_bf16x2(v[8 * w + 2], v[8 * w + 3]),
                                                     pack_bf16x2(v[8 * w + 4], v[8 * w + 5]),
                                                     pack_bf16x2(v[8 * w + 6], v[8 * w + 7]));
                } else {
#pragma unroll
                    for (int w = 0; w < 8; ++w)
                        st[w ^ (n & 7)] = make_uint4(__float_as_uint(v[4 * w]), __float_as_uint(v[4 * w + 1]),
                                                     __float_as_uint(v[4 * w + 2]), __float_as_uint(v[4 * w + 3]));
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // 4 times x 16 leaves x kOut words, in runs of 64 consecutive words
#pragma unroll
                for (int it = 0; it < kOut; ++it) {
                    const int tq = it / kRunsPerTime;
                    const int run = it % kRunsPerTime;
                    const int li = run * (kWave / kOut) + ln / kOut;
                    const int w = ln % kOut;
                    const int t = t0 + 4 * tq + r;
                    if (t < a.n_t && li < n_valid)
                        dst[t * row + run * kWave] = stage[wv][tq][li][w ^ (li & (kOut - 1))];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
}

// Few time points (a per-frame decode) from a quantised store: one thread per
// leaf, the 28 dot products of Eq. 7 / Eq. 9 in FP32 FMAs, one output record
// per time.  With n_t < 4 there is no dense contraction for the matrix cores
// to exploit; the kernel streams the records in and the snapshots out (BF16
// and FP8 records are small enough that per-thread reads stream well).
template <int DT, int OUT_BF16>
__global__ __launch_bounds__(kBlock) void eval_times_kernel(TreeDev tree, const float* basis, int32_t n_t,
                                                            int64_t n_leaves, void* out, float* sigma)
{
    constexpr int W = Pack<DT>::W;
    constexpr int R = Pack<DT>::R;
    constexpr int kWords = (FPO_N_COEFF + W - 1) / W;
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n_leaves) return;
    float k[kWords * W];
    const uint4* rec = tree.recs + l * R;
#pragma unroll
    for (int g = 0; g < kWords; ++g) Pack<DT>::unpack(rec[g], k + g * W);
    const float s = (DT == FPO_F32) ? 1.0f : tree.scale[l];
    for (int t = 0; t < n_t; ++t) {
        const float* b = basis + (int64_t)t * FPO_BASIS_STRIDE;
        float v[32];
        float sg = 0.0f;
#pragma unroll
        for (int i = 0; i < FPO_N_SIGMA; ++i) sg = fmaf(k[i], b[i], sg);
        v[0] = sg * s;
#pragma unroll
        for (int m = 0; m < FPO_N_BAKED - 1; ++m) {
            float z = 0.0f;
#pragma unroll
            for (int i = 0; i < FPO_N_SH_FOURIER; ++i) z = fmaf(k[FPO_N_SIGMA + FPO_N_SH_FOURIER * m + i], b[i], z);
            v[1 + m] = z * s;
        }
        v[28] = v[29] = v[30] = v[31] = 0.0f;
        const int64_t r = (int64_t)t * tree.stride + l;
        if (sigma) sigma[r] = stored_sigma<OUT_BF16>(v[0]);
        if (OUT_BF16) {
            uint4* o = static_cast<uint4*>(out) + r * 4;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                uint32_t u[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    u[e] = pack_bf16x2(v[8 * w + 2 * e], v[8 * w + 2 * e + 1]);
                o[w] = make_uint4(u[0], u[1], u[2], u[3]);
            }
        } else {
            float4* o = static_cast<float4*>(out) + r * 8;
#pragma unroll
            for (int w = 0; w < 8; ++w) o[w] = make_float4(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]);
        }
    }
}

// Few time points from the F32 store (the decode path's per-time IDFT pass):
// the same dot products, with the 768-byte records read as whole lines.  A
// wave takes 16 leaves: their records come in as whole lines into LDS rows,
// lane (n, g) then forms output row group g of leaf n (g = 0: density, 31
// terms; g = 1..3: nine SH rows of 5 terms), and the 16 output records leave
// through LDS as whole lines.
constexpr int kEvalOutPad = 33;           // LDS floats per staged output record (odd stride)

template <int OUT_BF16>
__global__ __launch_bounds__(kBlock) void eval_times_f32_kernel(TreeDev tree, const float* basis, int32_t n_t,
                                                                int64_t n_leaves, void* out, float* sigma)
{
    constexpr int DT = FPO_F32;
    constexpr int W = Pack<DT>::W;
    constexpr int R = Pack<DT>::R;
    constexpr int kWords = (FPO_N_COEFF + W - 1) / W;
    constexpr int kPf = kBakeLeaves * R / kWave;              // record words per lane
    constexpr int kOut = OUT_BF16 ? 4 : 8;                    // 16-byte words per output record
    __shared__ float coef[kBakeWaves][kBakeLeaves][kCoefPad];
    __shared__ float res[kBakeWaves][kBakeLeaves][kEvalOutPad];
    const int wv = threadIdx.x / kWave;
    const int ln = threadIdx.x % kWave;
    const int64_t leaf0 = ((int64_t)blockIdx.x * kBakeWaves + wv) * kBakeLeaves;
    if (leaf0 >= n_leaves) return;
    const int n_valid = (int)min<int64_t>(kBakeLeaves, n_leaves - leaf0);
    {
        uint4 pf[kPf];
        const uint4* src = tree.recs + leaf0 * R + ln;
#pragma unroll
        for (int p = 0; p < kPf; ++p) pf[p] = p * kWave + ln < n_valid * R ? src[p * kWave] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int p = 0; p < kPf; ++p) {
            const int idx = p * kWave + ln;
            const int li = idx / R;
            const int g = idx - li * R;
            if (g >= kWords) continue;
            float v[W];
            Pack<DT>::unpack(pf[p], v);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int q = g * W + e;
                if (q < kCoefPad) coef[wv][li][q] = q < FPO_N_COEFF ? v[e] : 0.0f;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int n = ln & 15;           // leaf of the wave's group
    const int g = ln >> 4;           // output row group
    const float* k = coef[wv][n];
    float* rs = res[wv][n];
    for (int t = 0; t < n_t; ++t) {
        const float* b = basis + (int64_t)t * FPO_BASIS_STRIDE;
        if (g == 0) {
            float sg = 0.0f;
#pragma unroll
            for (int i = 0; i < FPO_N_SIGMA; ++i) sg = fmaf(k[i], b[i], sg);
            rs[0] = sg;
            if (sigma && n < n_valid) sigma[(int64_t)t * tree.stride + leaf0 + n] = stored_sigma<OUT_BF16>(sg);
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int m = 9 * (g - 1) + q;
                float z = 0.0f;
#pragma unroll
                for (int i = 0; i < FPO_N_SH_FOURIER; ++i) z = fmaf(k[FPO_N_SIGMA + FPO_N_SH_FOURIER * m + i], b[i], z);
                rs[1 + m] = z;
            }
            if (g == 3) rs[28] = rs[29] = rs[30] = rs[31] = 0.0f;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // 16 records x kOut words, lane L writing word L of each 64-word run
#pragma unroll
        for (int it = 0; it < kOut / 4; ++it) {
            const int idx = it * kWave + ln;
            const int li = idx / kOut;
            const int w = idx % kOut;
            if (li >= n_valid) continue;
            const float* v = res[wv][li];
            const int64_t rec = (int64_t)t * tree.stride + leaf0 + li;
            if constexpr (OUT_BF16) {
                static_cast<uint4*>(out)[rec * 4 + w] =
                    make_uint4(pack_bf16x2(v[8 * w], v[8 * w + 1]), pack_bf16x2(v[8 * w + 2], v[8 * w + 3]),
                               pack_bf16x2(v[8 * w + 4], v[8 * w + 5]), pack_bf16x2(v[8 * w + 6], v[8 * w + 7]));
            } else {
                static_cast<float4*>(out)[rec * 8 + w] = make_float4(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Per-time evaluation for the other coefficient layouts (n1 density and n2 SH
// Fourier terms; F32, BF16 or FP8 store), one thread per leaf: word by word,
// every coefficient q goes to its one output (sigma for q < n1, else z_m with
// m = (q - n1) / n2 and basis index (q - n1) % n2), so every layout shares one
// loop without index tables; quantised stores scale the sums by the leaf's
// scale, as the default layout's kernels do.  (The compiler issues a record's
// loads together: the widest F32 layouts run at one wave per SIMD, and still
// stream at 5 TB/s.)
template <int DT, int N1, int N2, int OUT_BF16>
__global__ __launch_bounds__(kBlock) void eval_times_layout_kernel(TreeDev tree, const float* basis, int32_t n_t,
                                                                   int64_t n_leaves, void* out, float* sigma)
{
    using RC = Rec<DT, N1, N2>;
    constexpr int W = Pack<DT>::W;
    constexpr int kWords = (RC::kCoeff + W - 1) / W;
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n_leaves) return;
    const uint4* rec = tree.recs + l * RC::R;
    const float sc = (DT == FPO_F32) ? 1.0f : tree.scale[l];
    for (int t = 0; t < n_t; ++t) {
        const float* b = basis + (int64_t)t * FPO_BASIS_STRIDE;
        float v[32];
#pragma unroll
        for (int e = 0; e < 32; ++e) v[e] = 0.0f;
#pragma unroll
        for (int g = 0; g < kWords; ++g) {
            float k[W];
            Pack<DT>::unpack(rec[g], k);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int q = W * g + e;
                if (q < N1) v[0] = fmaf(k[e], b[q], v[0]);
                else if (q < RC::kCoeff) v[1 + (q - N1) / N2] = fmaf(k[e], b[(q - N1) % N2], v[1 + (q - N1) / N2]);
            }
        }
        if constexpr (DT != FPO_F32) {
#pragma unroll
            for (int e = 0; e < FPO_N_BAKED; ++e) v[e] *= sc;
        }
        const int64_t r = (int64_t)t * tree.stride + l;
        if (sigma) sigma[r] = stored_sigma<OUT_BF16>(v[0]);
        if constexpr (OUT_BF16) {
            uint4* o = static_cast<uint4*>(out) + r * 4;
#pragma unroll
            for (int w = 0; w < 4; ++w)
                o[w] = make_uint4(pack_bf16x2(v[8 * w], v[8 * w + 1]), pack_bf16x2(v[8 * w + 2], v[8 * w + 3]),
                                  pack_bf16x2(v[8 * w + 4], v[8 * w + 5]), pack_bf16x2(v[8 * w + 6], v[8 * w + 7]));
        } else {
            float4* o = static_cast<float4*>(out) + r * 8;
#pragma unroll
            for (int w = 0; w < 8; ++w) o[w] = make_float4(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]);
        }
    }
}

}  // namespace dev
}  // namespace fpo

using namespace fpo;

// Below this many time points the contraction is a matrix-vector product and
// the streaming FMA kernel is used; from here on the MFMA tiles pay off.
static constexpr int32_t kMfmaMinTimes = 4;

extern "C" fpo_status fpo_quantize(const float* coeffs, int64_t n_leaves, int64_t leaf_stride,
                                   const fpo_layout* layout, fpo_dtype dtype, void* q_out, float* scale_out,
                                   void* stream)
{
    ApiRange api_range_("fpo_quantize");
    if (!coeffs || !q_out || !scale_out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (dtype != FPO_BF16 && dtype != FPO_FP8_E4M3) return fail(FPO_E_INVALID, "dtype must be BF16 or FP8_E4M3");
    if (n_leaves < 1 || leaf_stride < n_leaves) return fail(FPO_E_INVALID, "bad n_leaves / leaf_stride");
    if (leaf_stride > (int64_t)INT32_MAX * dev::kBlock) return fail(FPO_E_INVALID, "too many leaves");
    const int n1 = layout ? layout->n_sigma : FPO_N_SIGMA;
    const int n2 = layout ? layout->n_sh_fourier : FPO_N_SH_FOURIER;
    const int64_t grid = (leaf_stride + dev::kBlock - 1) / dev::kBlock;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float4* src = reinterpret_cast<const float4*>(coeffs);
    uint4* dst = static_cast<uint4*>(q_out);
    const bool bf = dtype == FPO_BF16;
    switch (n1 * 100 + n2) {
#define FPO_Q(A, B) case A * 100 + B:                                                                           \
        if (bf) hipLaunchKernelGGL((dev::quantize_kernel<FPO_BF16, A, B>), dim3((unsigned)grid), dim3(dev::kBlock), \
                                   0, s, src, n_leaves, leaf_stride, dst, scale_out);                          \
        else hipLaunchKernelGGL((dev::quantize_kernel<FPO_FP8_E4M3, A, B>), dim3((unsigned)grid),              \
                                dim3(dev::kBlock), 0, s, src, n_leaves, leaf_stride, dst, scale_out);          \
        break
        FPO_Q(31, 5); FPO_Q(11, 5); FPO_Q(21, 5); FPO_Q(11, 11); FPO_Q(21, 11); FPO_Q(31, 11);
#undef FPO_Q
        default: return fail(FPO_E_UNSUPPORTED, "layout (n1, n2) not compiled");
    }
    return launch_status("fpo_quantize");
}

extern "C" fpo_status fpo_bake_times(const fpo_tree_view* tree, const float* basis, int32_t n_t,
                                     fpo_dtype out_dtype, void* out, float* sigma_out, void* stream)
{
    ApiRange api_range_("fpo_bake_times");
    fpo_status st = check_tree(tree, true, true);
    if (st != FPO_OK) return st;
    if (!basis || !out) return fail(FPO_E_INVALID, "NULL device pointer");
    if (n_t < 1) return fail(FPO_E_INVALID, "n_t must be >= 1");
    if (out_dtype != FPO_F32 && out_dtype != FPO_BF16) return fail(FPO_E_INVALID, "out_dtype must be F32 or BF16");
    if (!default_layout(tree->layout)) {
        const dev::TreeDev td = dev::tree_dev(tree);
        const int64_t g1 = (tree->n_leaves + dev::kBlock - 1) / dev::kBlock;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int bfo = out_dtype == FPO_BF16 ? 1 : 0;
        const int key = (tree->layout.n_sigma * 100 + tree->layout.n_sh_fourier) * 100 + (int)tree->dtype * 10 + bfo;
        switch (key) {
#define FPO_EVL1(A, B, DT, BF) case (A * 100 + B) * 100 + DT * 10 + BF:                                         \
            hipLaunchKernelGGL((dev::eval_times_layout_kernel<DT, A, B, BF>), dim3((unsigned)g1), dim3(dev::kBlock), \
                               0, s, td, basis, n_t, tree->n_leaves, out, sigma_out); break
#define FPO_EVL(A, B) FPO_EVL1(A, B, 0, 0); FPO_EVL1(A, B, 0, 1); FPO_EVL1(A, B, 1, 0); FPO_EVL1(A, B, 1, 1); \
            FPO_EVL1(A, B, 2, 0); FPO_EVL1(A, B, 2, 1)
            FPO_EVL(11, 5); FPO_EVL(21, 5); FPO_EVL(11, 11); FPO_EVL(21, 11); FPO_EVL(31, 11);
#undef FPO_EVL
#undef FPO_EVL1
            default: return fail(FPO_E_UNSUPPORTED, "layout (n1, n2) not compiled");
        }
        return launch_status("fpo_bake_times");
    }
    const int64_t per_block = (int64_t)dev::kBakeWaves * dev::kBakeLeaves;
    const int64_t grid = (tree->n_leaves + per_block - 1) / per_block;
    if (grid > INT32_MAX) return fail(FPO_E_INVALID, "too many leaves");
    dev::BakeLaunch a;
    std::memset(&a, 0, sizeof(a));
    a.tree = dev::tree_dev(tree);
    a.basis = basis;
    a.n_t = n_t;
    a.n_leaves = tree->n_leaves;
    a.out = out;
    a.sigma = sigma_out;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool bf = out_dtype == FPO_BF16;
    if (n_t < kMfmaMinTimes) {
        const dev::TreeDev td = dev::tree_dev(tree);
        if (tree->dtype == FPO_F32) {
            const int64_t g16 = (tree->n_leaves + per_block - 1) / per_block;
            if (bf)
                hipLaunchKernelGGL((dev::eval_times_f32_kernel<1>), dim3((unsigned)g16), dim3(dev::kBlock), 0, s, td,
                                   basis, n_t, tree->n_leaves, out, sigma_out);
            else
                hipLaunchKernelGGL((dev::eval_times_f32_kernel<0>), dim3((unsigned)g16), dim3(dev::kBlock), 0, s, td,
                                   basis, n_t, tree->n_leaves, out, sigma_out);
            return launch_status("fpo_bake_times");
        }
        const int64_t g1 = (tree->n_leaves + dev::kBlock - 1) / dev::kBlock;
#define FPO_EVAL(DT, BF)                                                                                   \
    hipLaunchKernelGGL((dev::eval_times_kernel<DT, BF>), dim3((unsigned)g1), dim3(dev::kBlock), 0, s, td,  \
                       basis, n_t, tree->n_leaves, out, sigma_out)
        switch (tree->dtype) {
            case FPO_BF16: if (bf) FPO_EVAL(FPO_BF16, 1); else FPO_EVAL(FPO_BF16, 0); break;
            default: if (bf) FPO_EVAL(FPO_FP8_E4M3, 1); else FPO_EVAL(FPO_FP8_E4M3, 0); break;
        }
#undef FPO_EVAL
        return launch_status("fpo_bake_times");
    }
#define FPO_BAKE(DT, BF) \
    hipLaunchKernelGGL((dev::bake_kernel<DT, BF>), dim3((unsigned)grid), dim3(dev::kBlock), 0, s, a)
    switch (tree->dtype) {
        case FPO_F32: if (bf) FPO_BAKE(FPO_F32, 1); else FPO_BAKE(FPO_F32, 0); break;
        case FPO_BF16: if (bf) FPO_BAKE(FPO_BF16, 1); else FPO_BAKE(FPO_BF16, 0); break;
        default: if (bf) FPO_BAKE(FPO_FP8_E4M3, 1); else FPO_BAKE(FPO_FP8_E4M3, 0); break;
    }
#undef FPO_BAKE
    return launch_status("fpo_bake_times");
}
