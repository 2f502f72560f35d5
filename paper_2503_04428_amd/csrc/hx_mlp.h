// Learned slope limiter: 4 -> 32 -> 32 -> 1 MLP (tanh-GELU hidden layers, phi = 2 sigmoid(z))
// evaluated with BF16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation).
//
// A wave evaluates 16 stencils per tile in the transposed form, so that every layer's output
// already sits in the lanes the next layer's operand needs:
//   layer 1: H1^T (32 x 16) = [W1 b1 0] (32 x 16) . [X 1 0]^T (16 x 16)     -> 2 MFMAs
//            (the bias rides in the padded K dimension: input 4 is the constant 1)
//   layer 2: H2^T (32 x 16) = W2 (32 x 32) . GELU(H1^T)                     -> 4 MFMAs
//   layer 3: z = w3 . GELU(H2^T) + b3 on the VALU, reduced over the 4 lanes of a stencil.
// Operand layout of the 16x16x16 MFMA: lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and
// D[4(l/16)+j][l%16], j = 0..3.  All 1249 parameters are used as BF16 values (weights in the MFMA
// operands as BF16, biases and w3 as the FP32 images of their BF16 roundings).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hx {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int MLP_NPARAM = 1249;
constexpr int MLP_W1 = 0, MLP_B1 = 128, MLP_W2 = 160, MLP_B2 = 1184, MLP_W3 = 1216, MLP_B3 = 1248;

// round-to-nearest-even FP32 -> BF16 bits (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ short bf16_bits(float f)
{
    return __builtin_bit_cast(short, (__bf16)f);
}
__device__ __forceinline__ float bf16_round(float f)
{
    return __uint_as_float(((uint32_t)(uint16_t)bf16_bits(f)) << 16);
}

// tanh-form GELU: 0.5 z (1 + tanh(k (z + 0.044715 z^3))) = z / (1 + exp(-2 k (z + 0.044715 z^3))),
// k = sqrt(2/pi); the exponent is folded into z (G1 + G3 z^2) in base 2
__device__ __forceinline__ float gelu_f(float z)
{
    constexpr float G1 = (float)(-2.0 * 0.7978845608028654 * 1.4426950408889634);
    constexpr float G3 = (float)(-2.0 * 0.7978845608028654 * 0.044715 * 1.4426950408889634);
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * (G1 + G3 * z * z)));
}

// per-lane constant operands of the network
struct MlpLane {
    bf16x4_t a1[2];     // [W1 b1] rows 16t + l%16, columns 4(l/16)+j (column 4 = b1, zero beyond)
    bf16x4_t a2[2][2];  // W2 rows 16u + l%16, columns 16t + 4(l/16) + j
    f32x4_t b2[2];      // b2 rows 16u + 4(l/16) + j
    f32x4_t w3[2];
    float b3;
};

// operands of one lane (lane = index within the wave), from the FP32 parameter vector
__device__ __forceinline__ void mlp_load(const float* __restrict__ w, int lane, MlpLane& m)
{
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; t++) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = 4 * q + j;
            m.a1[t][j] = k < 4    ? bf16_bits(w[MLP_W1 + (16 * t + r) * 4 + k])
                         : k == 4 ? bf16_bits(w[MLP_B1 + 16 * t + r])
                                  : (short)0;
            m.b2[t][j] = bf16_round(w[MLP_B2 + 16 * t + 4 * q + j]);
            m.w3[t][j] = bf16_round(w[MLP_W3 + 16 * t + 4 * q + j]);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int t = 0; t < 2; t++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                m.a2[u][t][j] = bf16_bits(w[MLP_W2 + (16 * u + r) * 32 + 16 * t + 4 * q + j]);
    m.b3 = bf16_round(w[MLP_B3]);
}

// One LDS copy per block of what MlpLane holds per lane (the b2 and w3 vectors depend on l/16 only).
struct MlpShared {
    bf16x4_t a1[2][64];
    bf16x4_t a2[2][2][64];
    f32x4_t b2[2][4], w3[2][4];
    float b3;
};

// filled by threads tid = 0..nthreads-1 of the block (a barrier must follow before use)
__device__ __forceinline__ void mlp_fill_shared(const float* __restrict__ w, int tid, int nthreads, MlpShared& s)
{
    for (int l = tid; l < 64; l += nthreads) {
        MlpLane m;
        mlp_load(w, l, m);
        const int q = l >> 4;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            s.a1[t][l] = m.a1[t];
#pragma unroll
            for (int u = 0; u < 2; u++)
                s.a2[u][t][l] = m.a2[u][t];
            if ((l & 15) == 0) {
                s.b2[t][q] = m.b2[t];
                s.w3[t][q] = m.w3[t];
            }
        }
        if (l == 0)
            s.b3 = m.b3;
    }
}

__device__ __forceinline__ void mlp_lane_from_shared(const MlpShared& s, int lane, MlpLane& m)
{
    const int q = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; t++) {
        m.a1[t] = s.a1[t][lane];
#pragma unroll
        for (int u = 0; u < 2; u++)
            m.a2[u][t] = s.a2[u][t][lane];
        m.b2[t] = s.b2[t][q];
        m.w3[t] = s.w3[t][q];
    }
    m.b3 = s.b3;
}

// phi for the 16 stencils of a tile.  xb: lanes 0..15 carry the 4 normalised inputs of stencil
// l (BF16); what the other lanes pass is ignored.  Lanes 0..15 return phi of stencil l (the other
// lanes return partial sums).  Must be called by the whole wave in uniform control flow.
__device__ __forceinline__ float mlp_tile(const MlpLane& m, bf16x4_t xb)
{
    const int lane = __lane_id();
    const bf16x4_t one = {(short)0x3f80, 0, 0, 0}, zero = {0, 0, 0, 0};  // BF16 1.0 = 0x3f80
    const bf16x4_t xin = lane < 16 ? xb : (lane < 32 ? one : zero);
    const f32x4_t c0 = {0.0f, 0.0f, 0.0f, 0.0f};
    bf16x4_t hb[2];
#pragma unroll
    for (int t = 0; t < 2; t++) {
        f32x4_t h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(m.a1[t], xin, c0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; j++)
            hb[t][j] = bf16_bits(gelu_f(h[j]));
    }
    float part = 0.0f;
#pragma unroll
    for (int u = 0; u < 2; u++) {
        f32x4_t c = m.b2[u];
#pragma unroll
        for (int t = 0; t < 2; t++)
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(m.a2[u][t], hb[t], c, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; j++)
            part += m.w3[u][j] * gelu_f(c[j]);
    }
    // sum over the four lane groups of a stencil: lanes 0..31 add lanes 32..63 (second result of
    // the 32-lane swap), then lanes 0..15 add lanes 16..31 (second result of the row swap)
    const auto s32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(part), __float_as_uint(part), false, false);
    part += __uint_as_float(s32[1]);
    const auto s16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(part), __float_as_uint(part), false, false);
    part += __uint_as_float(s16[1]);
    const float z = part + m.b3;
    return 2.0f * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

__device__ __forceinline__ bf16x4_t pack_x(float x0, float x1, float x2, float x3)
{
    bf16x4_t v;
    v[0] = bf16_bits(x0);
    v[1] = bf16_bits(x1);
    v[2] = bf16_bits(x2);
    v[3] = bf16_bits(x3);
    return v;
}

}  // namespace hx
