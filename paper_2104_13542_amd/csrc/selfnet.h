// Device helpers of the learned self-collision network (Sec. 3.2, Eq. 13,
// the jointNERF form) on the matrix cores: MFMA operand types, the LDS row
// layout of the activations and the fragment loads / activation stores of a
// 16 x 16 tile.
//
// Precision.  The weights are FP16 values (the context rejects weights that
// FP16 cannot hold exactly), and every activation a that feeds a matrix
// product is carried as two FP16 values, hi = fp16(a) and lo = fp16(a - hi),
// kept side by side in its LDS row.  A product is W hi + W lo, two FP16 MFMAs
// into one FP32 accumulator; each FP16 x FP16 product is exact in FP32, so
// the result matches an FP32 evaluation of the layer up to the lo rounding
// (about 2^-22 relative to a) and the FP32 accumulation order.
#pragma once

#include "storm_internal.h"

namespace storm {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// LDS row strides: the first two hidden layers' rows hold [hi (width) | lo
// (width) | pad] in halves, the last hidden layer's FP32 values; padded so
// that the 16 rows of an operand tile fall in different banks.
constexpr int kNetA1 = 2 * kNetH1 + 8;
constexpr int kNetA2 = 2 * kNetH2 + 8;
constexpr int kNetA3 = kNetH3 + 4;

// MFMA operands, lane l (both layouts checked on the device):
//   v_mfma_f32_16x16x16_f16 (layer 1, k = 16)
//     A (16 x 16, rows x k):    A[l % 16][4 (l / 16) + j], j < 4
//     B (16 x 16, k x columns): B[4 (l / 16) + j][l % 16]
//   v_mfma_f32_16x16x32_f16 (layers 2 and 3, twice the k per instruction)
//     A (16 x 32):              A[l % 16][8 (l / 16) + j], j < 8
//     B (32 x 16):              B[8 (l / 16) + j][l % 16]
//   D (16 x 16), both:          D[4 (l / 16) + j][l % 16]
__device__ __forceinline__ half4_t net_load_a(const _Float16 *s, int stride, int m, int ks, int lane)
{
    return *reinterpret_cast<const half4_t *>(s + (16 * m + (lane & 15)) * stride + 16 * ks + 4 * (lane >> 4));
}

__device__ __forceinline__ half8_t net_load_a8(const _Float16 *s, int stride, int m, int ks, int lane)
{
    return *reinterpret_cast<const half8_t *>(s + (16 * m + (lane & 15)) * stride + 32 * ks + 8 * (lane >> 4));
}

// The FP16 pair (hi, lo) of a: hi = fp16(a), lo = fp16(a - hi).
__device__ __forceinline__ void split_half(float a, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)a;
    lo = (_Float16)(a - (float)hi);
}

// D tile (row block m, column block n) + bias, ReLU, stored as the (hi, lo)
// pairs of the next layer's input rows (lo `width` halves after hi).
__device__ __forceinline__ void net_store_relu_h(_Float16 *s, int stride, int width, int m, int n, int lane,
                                                 float4_t d, float bias)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        _Float16 hi, lo;
        split_half(fmaxf(d[j] + bias, 0.0f), hi, lo);
        _Float16 *r = s + (16 * m + 4 * (lane >> 4) + j) * stride + 16 * n + (lane & 15);
        r[0] = hi;
        r[width] = lo;
    }
}

// Same, FP32 rows (the last hidden layer, read by the output dot product).
__device__ __forceinline__ void net_store_relu_f(float *s, int stride, int m, int n, int lane, float4_t d,
                                                 float bias)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) s[(16 * m + 4 * (lane >> 4) + j) * stride + 16 * n + (lane & 15)] = fmaxf(d[j] + bias, 0.0f);
}

// Layer 2 column block n (16 units) for all 64 rows: 8 k-steps of 32 over
// the 256 first-layer outputs in LDS, each taken as hi and as lo.
__device__ __forceinline__ void net_layer2(const _Float16 *s_a1, _Float16 *s_a2, const half8_t b2[8], float bias2,
                                           int n, int lane)
{
    float4_t d[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) d[m] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int m = 0; m < 4; ++m)
        {
            d[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(net_load_a8(s_a1, kNetA1, m, s, lane), b2[s], d[m], 0, 0, 0);
            d[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(net_load_a8(s_a1 + kNetH1, kNetA1, m, s, lane), b2[s], d[m],
                                                          0, 0, 0);
        }
#pragma unroll
    for (int m = 0; m < 4; ++m) net_store_relu_h(s_a2, kNetA2, kNetH2, m, n, lane, d[m], bias2);
}

// Layer 3 column block n, row blocks m0 and m0 + 1: 4 k-steps of 32 over
// the 128 second-layer outputs, each taken as hi and as lo.
__device__ __forceinline__ void net_layer3(const _Float16 *s_a2, float *s_a3, const half8_t b3[4], float bias3, int n,
                                           int m0, int lane)
{
    float4_t d[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) d[r] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r = 0; r < 2; ++r)
        {
            d[r] = __builtin_amdgcn_mfma_f32_16x16x32_f16(net_load_a8(s_a2, kNetA2, m0 + r, s, lane), b3[s], d[r], 0,
                                                          0, 0);
            d[r] = __builtin_amdgcn_mfma_f32_16x16x32_f16(net_load_a8(s_a2 + kNetH2, kNetA2, m0 + r, s, lane), b3[s],
                                                          d[r], 0, 0, 0);
        }
#pragma unroll
    for (int r = 0; r < 2; ++r) net_store_relu_f(s_a3, kNetA3, m0 + r, n, lane, d[r], bias3);
}

// Output layer for row `lane`: d = b4 + w4 . a3[lane].
__device__ __forceinline__ float net_output(const float *s_a3, const float *__restrict__ bias, int lane)
{
    float dist = bias[kNetBias4];
    const float *a3 = s_a3 + lane * kNetA3;
#pragma unroll
    for (int k = 0; k < kNetH3; k += 4) {
        const float4 v = *reinterpret_cast<const float4 *>(a3 + k);
        dist = fmaf(bias[kNetW4 + k], v.x, dist);
        dist = fmaf(bias[kNetW4 + k + 1], v.y, dist);
        dist = fmaf(bias[kNetW4 + k + 2], v.z, dist);
        dist = fmaf(bias[kNetW4 + k + 3], v.w, dist);
    }
    return dist;
}

}  // namespace storm
