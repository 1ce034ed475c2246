// Device code of the learned proposal (not part of the paper): the coarse
// occupancy scan that makes empty-space skipping exact, and the wave-wide
// FP16 matrix-core inference of the proposal MLP.
//
// Proposal MLP.  Inputs per ray: the entry point into the unit cube (3), the
// unit direction (3) and tau = t / T mod 1 (1).  Positional encoding
// gamma(x) = (sin 2^f pi x, cos 2^f pi x), f < 6, feature 12 c + 2 f + {0:
// sin, 1: cos}; layers 84 -> 64 -> 64 -> 3 with ReLU on the hidden layers.
// Outputs: hit logit, and logits of s_in / s_out, the first entry into and
// last exit from contributing leaves as fractions of the chord in the cube.
//
// Parameters (FP32 master copy, FPO_MLP_N_PARAMS floats): three row-major
// matrices [85][64], [65][64], [65][3] (input index major), the last row of
// each holding the layer's bias.
//
// Coarse occupancy: a 64^3 bit grid over the unit cube, bit (z 64 + y) 64 + x,
// set where a leaf overlaps the cell or one of its 26 neighbours (dilated by
// one cell).  A scan through it that finds only clear cells proves that the
// ray passes no leaf there: the dilation margin (1/64) dwarfs the FP32 error
// of the scan.
#pragma once

#include "fpo.h"
#include "fpo_device.h"

namespace fpo {
namespace dev {

constexpr int kMlpIn = FPO_MLP_N_IN;
constexpr int kMlpPE = FPO_MLP_N_PE;
constexpr int kMlpH = FPO_MLP_HIDDEN;
constexpr int kP1 = 0;                          // [85][64]
constexpr int kP2 = (kMlpPE + 1) * kMlpH;       // [65][64]
constexpr int kP3 = kP2 + (kMlpH + 1) * kMlpH;  // [65][3]
static_assert(kP3 + (kMlpH + 1) * 3 == FPO_MLP_N_PARAMS, "parameter layout");

// Packed inference weights: 44 A-operand fragments of v_mfma_f32_16x16x16f16
// ([fragment][lane] x 4 FP16 = 8 bytes), then FP32 biases b1[64], b2[64], b3[4].
constexpr int kFrag1 = 0;    // layer 1: fragment mt * 6 + kb (features padded to 96)
constexpr int kFrag2 = 24;   // layer 2: 24 + mt * 4 + kb
constexpr int kFrag3 = 40;   // layer 3: 40 + kb (output rows 0..2 of 16)
constexpr int kFrags = 44;
constexpr int kPackedBias = kFrags * 64 * 8;
static_assert(kPackedBias + (64 + 64 + 4) * 4 == FPO_MLP_PACKED_BYTES, "packed layout");

constexpr int kCoarse = FPO_COARSE_RES;

typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Distance along the unit direction dv from p to the entry of the first set
// coarse cell, or t_max when no set cell starts before t_max (an
// Amanatides-Woo scan over the 64^3 grid).
__device__ inline float coarse_scan(const uint32_t* __restrict__ bits, const float* p, const float* dv,
                                    float t_max)
{
    const float fN = (float)kCoarse;
    const float h = 1.0f / fN;
    int c[3], st[3];
    float tm[3], td[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int v = (int)floorf(p[a] * fN);
        c[a] = min(max(v, 0), kCoarse - 1);
        const float inv = 1.0f / dv[a];
        if (dv[a] > 0.0f) {
            st[a] = 1;
            tm[a] = ((float)(c[a] + 1) * h - p[a]) * inv;
            td[a] = h * inv;
        } else if (dv[a] < 0.0f) {
            st[a] = -1;
            tm[a] = ((float)c[a] * h - p[a]) * inv;
            td[a] = -h * inv;
        } else {
            st[a] = 0;
            tm[a] = __builtin_inff();
            td[a] = __builtin_inff();
        }
    }
    float t = 0.0f;
    for (int it = 0; it < 3 * kCoarse + 1; ++it) {
        const int idx = (c[2] * kCoarse + c[1]) * kCoarse + c[0];
        if ((bits[idx >> 5] >> (idx & 31)) & 1u) return fmaxf(t, 0.0f);
        const int ax = tm[0] <= tm[1] ? (tm[0] <= tm[2] ? 0 : 2) : (tm[1] <= tm[2] ? 1 : 2);
        t = tm[ax];
        if (t >= t_max) return t_max;
        c[ax] += st[ax];
        if ((unsigned)c[ax] >= (unsigned)kCoarse) return t_max;
        tm[ax] += td[ax];
    }
    return t_max;
}

// Inputs of one ray: entry point, unit direction, tau.
__device__ inline void proposal_inputs(const Ray& r, float tau, float* x)
{
    x[0] = r.o[0]; x[1] = r.o[1]; x[2] = r.o[2];
    x[3] = r.d[0]; x[4] = r.d[1]; x[5] = r.d[2];
    x[6] = tau;
}

__device__ inline f16x4 frag_load(const uint2* F, int frag, int ln)
{
    const uint2 w = F[frag * 64 + ln];
    return __builtin_bit_cast(f16x4, w);
}

__device__ inline f16x4 relu_h(f32x4 v)
{
    f16x4 o;
    o[0] = (_Float16)fmaxf(v[0], 0.0f);
    o[1] = (_Float16)fmaxf(v[1], 0.0f);
    o[2] = (_Float16)fmaxf(v[2], 0.0f);
    o[3] = (_Float16)fmaxf(v[3], 0.0f);
    return o;
}

// Wave-wide inference: every lane of the wave must call this together.  x is
// this lane's 7 inputs; out receives this lane's 3 outputs.  Features are the
// rows (M) of each product and the wave's 64 rays its columns (N), so each
// layer's accumulator tile is, lane for lane, the next layer's B operand.
// F: the 44 fragments ([fragment][lane]); bias: the 132 FP32 biases (either
// may point to global memory or to an LDS copy).
__device__ inline void mlp_infer_wave(const uint2* F, const float* bias, const float* x, float* out)
{
    const int ln = threadIdx.x & 63;
    const int q = ln >> 4;
    const int j = ln & 15;

    // inputs of the rays 16 nt + j this lane supplies B-operand values for
    float xin[4][kMlpIn];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c) xin[nt][c] = __shfl(x[c], 16 * nt + j, 64);

    f32x4 acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const float4 b4 = *reinterpret_cast<const float4*>(bias + 16 * mt + 4 * q);
        const f32x4 b = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = b;
    }
    // layer 1: K = 96 encoded features (84 used), six K-blocks of 16.  Lane
    // (q, j) supplies features 16 kb + 4 q .. + 3: one input component c and
    // the sin / cos pair of two consecutive frequencies.
#pragma unroll
    for (int kb = 0; kb < 6; ++kb) {
        const int F0 = 16 * kb + 4 * q;
        const int c_lo = (16 * kb) / 12;
        const bool hi = F0 >= 12 * (c_lo + 1);
        const int c = c_lo + (hi ? 1 : 0);
        const int f0 = (F0 - 12 * c) >> 1;                  // 0, 2 or 4
        const float rev = (float)(1 << f0) * 0.5f;          // revolutions per unit x at frequency f0
        f16x4 B[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const float lo_v = xin[nt][c_lo < kMlpIn ? c_lo : kMlpIn - 1];
            const float hi_v = xin[nt][c_lo + 1 < kMlpIn ? c_lo + 1 : kMlpIn - 1];
            const float xv = hi ? hi_v : lo_v;
            const float a0 = xv * rev;
            const float a1 = a0 * 2.0f;
            f16x4 v;
            v[0] = (_Float16)__builtin_amdgcn_sinf(a0);
            v[1] = (_Float16)__builtin_amdgcn_cosf(a0);
            v[2] = (_Float16)__builtin_amdgcn_sinf(a1);
            v[3] = (_Float16)__builtin_amdgcn_cosf(a1);
            const f16x4 zero = {0, 0, 0, 0};
            B[nt] = F0 < kMlpPE ? v : zero;
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f16x4 A = frag_load(F, kFrag1 + mt * 6 + kb, ln);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16f16(A, B[nt], acc[mt][nt], 0, 0, 0);
        }
    }
    f16x4 H[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) H[mt][nt] = relu_h(acc[mt][nt]);
    // layer 2
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const float4 b4 = *reinterpret_cast<const float4*>(bias + 64 + 16 * mt + 4 * q);
        const f32x4 b = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = b;
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f16x4 A = frag_load(F, kFrag2 + mt * 4 + kb, ln);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16f16(A, H[kb][nt], acc[mt][nt], 0, 0, 0);
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) H[mt][nt] = relu_h(acc[mt][nt]);
    // layer 3: output rows 0..2 live in lanes q = 0
    f32x4 o[4];
    {
        const float4 b4 = *reinterpret_cast<const float4*>(bias + 128);
        const f32x4 b = {b4.x, b4.y, b4.z, 0.0f};
        const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) o[nt] = q == 0 ? b : z;
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const f16x4 A = frag_load(F, kFrag3 + kb, ln);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) o[nt] = __builtin_amdgcn_mfma_f32_16x16x16f16(A, H[kb][nt], o[nt], 0, 0, 0);
    }
    // ray ln's outputs sit in lane ln & 15 of column tile ln >> 4
    const int src = ln & 15;
    const int tile = ln >> 4;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const float v0 = __shfl(o[0][e], src, 64);
        const float v1 = __shfl(o[1][e], src, 64);
        const float v2 = __shfl(o[2][e], src, 64);
        const float v3 = __shfl(o[3][e], src, 64);
        out[e] = tile == 0 ? v0 : tile == 1 ? v1 : tile == 2 ? v2 : v3;
    }
}

}  // namespace dev
}  // namespace fpo
