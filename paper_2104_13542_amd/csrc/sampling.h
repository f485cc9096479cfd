// Device helpers shared by the rollout and adjoint kernels: counter-based
// Gaussian noise (Sec. 3.3 sampling) and wavefront segmented scans over the
// steps of one particle (the triangular sums of Sec. 3.1, Eq. 7).
#pragma once

#include "storm_internal.h"

namespace storm {
namespace {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products with the Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Box-Muller on 24-bit uniforms u1 in (0, 1], u2 in [0, 1).
__device__ __forceinline__ void box_muller(uint32_t x0, uint32_t x1, float &zc, float &zs)
{
    const float u1 = (float)((x0 >> 8) + 1u) * 0x1.0p-24f;
    const float u2 = (float)(x1 >> 8) * 0x1.0p-24f;
    const float r = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    zc = r * c;
    zs = r * s;
}

// Lane move through DPP: lane l receives x from the lane that `kCtrl` names
// (row shifts, row broadcasts); lanes whose source is outside the row, or
// in a row that kRowMask leaves out, receive 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_or_zero(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, kRowMask, 0xf, true));
}

// Inclusive prefix sum over the lanes of one particle (lanes p*H .. p*H+H-1;
// h = step index of this lane), without LDS traffic: a Kogge-Stone scan
// inside each 16-lane row (DPP row shifts by 1, 2, 4, 8, each term taken
// only from the lane's own segment and row), then the two row broadcasts
// that carry the sums of rows 0 and 2 into rows 1 and 3, and of rows 0-1
// into rows 2-3, each taken only by lanes whose particle began before the
// source lane.  Segments of the padding lanes past the last particle are
// scanned the same way.
__device__ __forceinline__ float segmented_scan(float x, int h, int H)
{
    (void)H;
    const int lane = threadIdx.x & (kLanes - 1);
    const int in_row = lane & 15;
    const int reach = h < in_row ? h : in_row;  // lanes back to the row or segment start
    float y;
    y = dpp_or_zero<0x111, 0xf>(x);  // row_shr:1
    x += reach >= 1 ? y : 0.0f;
    y = dpp_or_zero<0x112, 0xf>(x);  // row_shr:2
    x += reach >= 2 ? y : 0.0f;
    y = dpp_or_zero<0x114, 0xf>(x);  // row_shr:4
    x += reach >= 4 ? y : 0.0f;
    y = dpp_or_zero<0x118, 0xf>(x);  // row_shr:8
    x += reach >= 8 ? y : 0.0f;
    y = dpp_or_zero<0x142, 0xa>(x);  // row_bcast:15 -> rows 1, 3
    x += h > in_row ? y : 0.0f;
    y = dpp_or_zero<0x143, 0xc>(x);  // row_bcast:31 -> rows 2, 3
    x += (lane >= 32 && h > lane - 32) ? y : 0.0f;
    return x;
}

__device__ __forceinline__ float hinge_box(float x, float lo, float hi)
{
    return fmaxf(lo - x, 0.0f) + fmaxf(x - hi, 0.0f);
}

// Inclusive suffix sum over the lanes of one particle (the transpose of
// segmented_scan, used by the reverse pass).
__device__ __forceinline__ float segmented_suffix_scan(float x, int h, int H)
{
    for (int off = 1; off < H; off <<= 1) {
        const float y = __shfl_down(x, (unsigned)off, kLanes);
        if (h + off < H) x += y;
    }
    return x;
}

// Comb-filtered noise of one joint at step h (Sec. 3.3), from that joint's
// row of standard noise over the tile's lanes: the filter's recursion in
// step order written as its convolution, sum over k <= h of g_k e_{h-k},
// with the response g in the tables; e_{h-k} is the lane k below, in the
// same particle.
__device__ __forceinline__ float comb_noise(const float *row, int lane, int h, int H,
                                            const float *__restrict__ tab)
{
    // eight terms per batch, every read of a batch in flight at once (the
    // response is zero past H, and within the table's kMaxH entries)
    float acc = 0.0f;
    for (int k0 = 0; k0 < H; k0 += 8) {
        float g[8], e[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            g[m] = tab[kTabComb + k0 + m];
            e[m] = k0 + m <= h ? row[lane - k0 - m] : 0.0f;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) acc = fmaf(g[m], e[m], acc);
    }
    return acc;
}

// Standard noise of joints 4k..4k+3 for one (particle, step) point from the
// override, the Halton table or Philox (k = 0 or 1).
__device__ __forceinline__ void standard_noise4(const ProblemDev &P, const float *__restrict__ noise, int k, int i,
                                                int h, uint32_t counter, float e[4])
{
    const int j0 = 4 * k;
    if (noise != nullptr) {
#pragma unroll
        for (int m = 0; m < 4; ++m) e[m] = j0 + m < kDof ? noise[((size_t)(j0 + m) * P.N + i) * P.H + h] : 0.0f;
    } else if (i < P.n_halton) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
            e[m] = j0 + m < kDof ? P.halton[((size_t)(j0 + m) * P.n_halton + i) * P.H + h] : 0.0f;
    } else {
        uint32_t c0 = (uint32_t)i, c1 = (uint32_t)h, c2 = (uint32_t)k, c3 = counter;
        philox4x32_10(c0, c1, c2, c3, P.seed_lo, P.seed_hi);
        box_muller(c0, c1, e[0], e[1]);
        box_muller(c2, c3, e[2], e[3]);
    }
}

// Standard noise of joints 4k + 2 half and 4k + 2 half + 1 for one (particle,
// step) point: the same values as standard_noise4's e[2 half], e[2 half + 1]
// (the Philox call of k, then the Box-Muller transform of its half).
__device__ __forceinline__ void standard_noise2(const ProblemDev &P, const float *__restrict__ noise, int k, int half,
                                                int i, int h, uint32_t counter, float e[2])
{
    const int j0 = 4 * k + 2 * half;
    if (noise != nullptr) {
#pragma unroll
        for (int m = 0; m < 2; ++m) e[m] = j0 + m < kDof ? noise[((size_t)(j0 + m) * P.N + i) * P.H + h] : 0.0f;
    } else if (i < P.n_halton) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
            e[m] = j0 + m < kDof ? P.halton[((size_t)(j0 + m) * P.n_halton + i) * P.H + h] : 0.0f;
    } else {
        uint32_t c0 = (uint32_t)i, c1 = (uint32_t)h, c2 = (uint32_t)k, c3 = counter;
        philox4x32_10(c0, c1, c2, c3, P.seed_lo, P.seed_hi);
        if (half == 0)
            box_muller(c0, c1, e[0], e[1]);
        else
            box_muller(c2, c3, e[0], e[1]);
    }
}

}  // namespace
}  // namespace storm
