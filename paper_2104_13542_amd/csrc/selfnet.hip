// Learned self-collision term (Sec. 3.2, Eq. 13, the jointNERF form) on the
// matrix cores.  The network maps the encoding [sin q, cos q] through ReLU
// layers of 256, 128 and 64 units to one output d, the predicted closest
// distance between the links (positive when they penetrate); the term is
// max(0, d).
//
// One workgroup (8 waves) per 64-lane tile of the rollout (the same
// (particle, step) rows): the three hidden layers are 64-row GEMMs on
// v_mfma_f32_16x16x16_f16 (layer 1) and v_mfma_f32_16x16x32_f16 (FP16
// weights, activations as FP16 (hi, lo) pairs, FP32 accumulation), with
// the activations staged in LDS between layers and the weights read as
// pre-packed per-lane fragments (one coalesced 512-byte load per wave and
// fragment).  The output layer is a 64-term dot product per row on the
// vector units; the term then joins the running cost (weight a_coll, as the
// sphere model's) and, through a segmented scan over the steps, the horizon
// cost C_i that the rollout kernel wrote.
#include "sampling.h"
#include "selfnet.h"
#include "storm_internal.h"

namespace storm {

namespace {

constexpr int kNetWaves = 8;
constexpr int kNetThreads = kNetWaves * kLanes;
constexpr int kIn = 16;      // 14 inputs padded to one k-step
constexpr int kX = 2 * kIn;  // LDS row stride of the encoding in halves: hi (16), lo (16)
// LDS: encoding, first and second hidden layers; the last hidden layer's
// FP32 rows reuse the first layer's space (dead once layer 2 has run)
constexpr int kOffA1 = 64 * kX * 2;
constexpr int kOffA2 = kOffA1 + 64 * kNetA1 * 2;
constexpr int kNetLds = kOffA2 + 64 * kNetA2 * 2;
static_assert(64 * kNetA3 * 4 <= 64 * kNetA1 * 2, "last hidden layer fits in the first layer's space");

__global__ __launch_bounds__(kNetThreads) void selfnet_kernel(ProblemDev P, const _Float16 *__restrict__ frag,
                                                              const float *__restrict__ bias, StepOut out)
{
    __shared__ __attribute__((aligned(16))) unsigned char s_lds[kNetLds];
    _Float16 *s_x = reinterpret_cast<_Float16 *>(s_lds);
    _Float16 *s_a1 = reinterpret_cast<_Float16 *>(s_lds + kOffA1);
    _Float16 *s_a2 = reinterpret_cast<_Float16 *>(s_lds + kOffA2);
    float *s_a3 = reinterpret_cast<float *>(s_lds + kOffA1);

    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = blockIdx.x;
    const int N = P.N, H = P.H;

    // row `lane` of the tile; wave j < 7 encodes joint j of every row.  Its
    // position is loaded first, so that waiting for it does not wait for the
    // weight loads behind it (an invalid row reads particle 0 and is ignored).
    const int pl = lane / H;
    const int h = lane - pl * H;
    const int i = tile * P.ppt + pl;
    const bool valid = pl < P.ppt && i < N;
    const int jq = wave < kDof ? wave : 0;
    const float qv = P.qbuf[((size_t)jq * N + (valid ? i : 0)) * H + h];
    __builtin_amdgcn_sched_barrier(0);  // keep that load ahead of the weight loads

    // every weight fragment this wave uses, loaded up front (52 VGPRs)
    // (in the order of use, each layer's biases with its fragments)
    const half4_t *F1 = reinterpret_cast<const half4_t *>(frag + kNetFrag1);
    const half8_t *F2 = reinterpret_cast<const half8_t *>(frag + kNetFrag2);
    const half8_t *F3 = reinterpret_cast<const half8_t *>(frag + kNetFrag3);
    half4_t b1[2];
    half8_t b2[8], b3[4];
#pragma unroll
    for (int t = 0; t < 2; ++t) b1[t] = F1[(2 * wave + t) * kLanes + lane];
    const float bias1[2] = {bias[kNetBias1 + 16 * (2 * wave) + (lane & 15)],
                            bias[kNetBias1 + 16 * (2 * wave + 1) + (lane & 15)]};
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 8; ++s) b2[s] = F2[(wave * 8 + s) * kLanes + lane];
    const float bias2 = bias[kNetBias2 + 16 * wave + (lane & 15)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) b3[s] = F3[((wave >> 1) * 4 + s) * kLanes + lane];
    const float bias3 = bias[kNetBias3 + 16 * (wave >> 1) + (lane & 15)];

    // encoding [sin q, cos q, 0, 0] of the 64 rows, as (hi, lo) pairs
    if (wave < kDof) {
        float sn, cs;
        sincosf(valid ? qv : 0.0f, &sn, &cs);
        _Float16 *r = s_x + lane * kX;
        split_half(sn, r[wave], r[kIn + wave]);
        split_half(cs, r[kDof + wave], r[kIn + kDof + wave]);
    } else if (wave == kDof) {
        _Float16 *r = s_x + lane * kX;
        r[14] = r[15] = r[kIn + 14] = r[kIn + 15] = (_Float16)0.0f;
    }
    __syncthreads();

    // layer 1: 64 x 16 by 16 x 256 for hi and for lo; wave w: columns
    // 32 w .. 32 w + 31
    {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const half4_t ahi = net_load_a(s_x, kX, m, 0, lane);
            const half4_t alo = net_load_a(s_x + kIn, kX, m, 0, lane);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                float4_t d = {0.0f, 0.0f, 0.0f, 0.0f};
                d = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, b1[t], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x16f16(alo, b1[t], d, 0, 0, 0);
                net_store_relu_h(s_a1, kNetA1, kNetH1, m, 2 * wave + t, lane, d, bias1[t]);
            }
        }
    }
    __syncthreads();

    // layer 2: 64 x 256 by 256 x 128; wave w: columns 16 w .. 16 w + 15
    net_layer2(s_a1, s_a2, b2, bias2, wave, lane);
    __syncthreads();

    // layer 3: 64 x 128 by 128 x 64; wave w: columns 16 (w / 2) .., rows 32
    // (w % 2) ..; its FP32 output rows go where layer 1's were
    net_layer3(s_a2, s_a3, b3, bias3, wave >> 1, 2 * (wave & 1), lane);
    __syncthreads();

    // output layer, cost term and horizon cost (wave 0, lane = row)
    if (wave == 0) {
        const float dist = net_output(s_a3, bias, lane);
        const float term = fmaxf(dist, 0.0f);  // Eq. 13
        const float dc = P.a_coll * term;
        const float added = segmented_scan(P.tables[kTabHw + h] * dc, h, H);
        if (valid) {
            if (out.terms) out.terms[((size_t)6 * N + i) * H + h] = term;
            if (out.c) out.c[(size_t)i * H + h] += dc;
            if (h == H - 1) {
                const float C = P.C[i] + added;
                P.C[i] = C;
                if (out.C) out.C[i] = C;
            }
        }
    }
}

}  // namespace

hipError_t launch_selfnet(const ProblemDev &P, const _Float16 *frag, const float *bias, const StepOut &out,
                          hipStream_t stream)
{
    hipLaunchKernelGGL(selfnet_kernel, dim3((unsigned)P.n_tiles), dim3(kNetThreads), 0, stream, P, frag, bias, out);
    return hipGetLastError();
}

bool selfnet_weights_fp16(const float *prm)
{
    const float *W1 = prm, *W2 = W1 + kNetH1 * kNetIn + kNetH1, *W3 = W2 + kNetH2 * kNetH1 + kNetH2;
    auto exact = [](const float *W, int n) {
        for (int k = 0; k < n; ++k)
            if ((float)(_Float16)W[k] != W[k]) return false;
        return true;
    };
    return exact(W1, kNetH1 * kNetIn) && exact(W2, kNetH2 * kNetH1) && exact(W3, kNetH3 * kNetH2);
}

// Pack the network's parameters (weights [out][in], FP32 holding FP16
// values) into the per-lane FP16 fragments the kernel loads, and the biases
// and output weights (FP32).
void pack_selfnet(const float *prm, std::vector<_Float16> &frag, std::vector<float> &bias)
{
    const float *W1 = prm, *b1 = W1 + kNetH1 * kNetIn;
    const float *W2 = b1 + kNetH1, *b2 = W2 + kNetH2 * kNetH1;
    const float *W3 = b2 + kNetH2, *b3 = W3 + kNetH3 * kNetH2;
    const float *w4 = b3 + kNetH3, *b4 = w4 + kNetH3;
    frag.assign((size_t)kNetFragHalves, (_Float16)0.0f);
    // fragment (column block t, k-step s) of B = W^T with `per` halves per
    // lane (k-steps of 4 per): lane l, element j is
    // W[16 t + l % 16][4 per s + per (l / 16) + j]
    auto put = [&](int base, const float *W, int n_in, int n_tiles, int n_steps, int per) {
        for (int t = 0; t < n_tiles; ++t)
            for (int s = 0; s < n_steps; ++s)
                for (int l = 0; l < kLanes; ++l)
                    for (int j = 0; j < per; ++j) {
                        const int o = 16 * t + (l & 15), k = 4 * per * s + per * (l >> 4) + j;
                        frag[(size_t)base + (((size_t)t * n_steps + s) * kLanes + l) * per + j] =
                            (_Float16)(k < n_in ? W[o * n_in + k] : 0.0f);
                    }
    };
    put(kNetFrag1, W1, kNetIn, kNetH1 / 16, 1, 4);
    put(kNetFrag2, W2, kNetH1, kNetH2 / 16, kNetH1 / 32, 8);
    put(kNetFrag3, W3, kNetH2, kNetH3 / 16, kNetH2 / 32, 8);
    bias.assign((size_t)kNetBiasSize, 0.0f);
    for (int k = 0; k < kNetH1; ++k) bias[kNetBias1 + k] = b1[k];
    for (int k = 0; k < kNetH2; ++k) bias[kNetBias2 + k] = b2[k];
    for (int k = 0; k < kNetH3; ++k) bias[kNetBias3 + k] = b3[k];
    for (int k = 0; k < kNetH3; ++k) bias[kNetW4 + k] = w4[k];
    bias[kNetBias4] = b4[0];
}

}  // namespace storm
