// Kernel U: exponentiated-cost policy update of STORM (Sec. 3, Eq. 4-6),
// followed by the next command and the warm-start shift of Alg. 1.
//
//   w_i     = exp(-(C_i - min C) / beta) / sum_k exp(-(C_k - min C) / beta)
//   mu'     = mu + alpha_mu sum_i w_i d_i,          d_i = u_i - mu
//   sigma2' = (1 - alpha_sigma) sigma2
//             + alpha_sigma mean_h sum_i w_i (u_ih - mu'_h)^2   (per joint)
//
// One workgroup of 1024 threads per problem.  Weights are staged in LDS in
// chunks.  Two wavefronts per joint stream that joint's controls u[j][*][*]
// in contiguous rows of H floats, sixteen loads in flight per lane, and
// accumulate per step; the partial sums are merged in a fixed order.  The variance about
// the new mean comes from the moments about the old one,
// sum w (d - delta)^2 = S2/S0 - 2 delta S1/S0 + delta^2, in one pass.  Every
// sum has a fixed order (results are bitwise reproducible); no atomics on
// floating-point data and no cross-workgroup synchronisation.
#include "storm_internal.h"

namespace storm {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / kLanes;
constexpr int kUnroll = 16;    // independent loads in flight per lane

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kLanes);
    return x;
}

__device__ __forceinline__ float wave_min(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fminf(x, __shfl_xor(x, off, kLanes));
    return x;
}

// Two ways to form the moments, chosen by the number M of particles whose
// weight is not exactly zero (with beta small against the spread of C, most
// weights underflow to 0 and contribute nothing):
//  - sparse (M <= kList): the nonzero weights and their particle indices are
//    compacted in ascending order into LDS; thread rows of each (joint, step)
//    column take list entries r, r + R, ... and only those rows of u are read;
//  - dense: two wavefronts per joint stream u[j] in contiguous rows of H
//    floats (two particles per load when H <= 32), sixteen loads in flight
//    per lane.
// Both add in a fixed order, so results are bitwise reproducible.
constexpr int kList = 4096;

__device__ __forceinline__ void update_problem(const ProblemDev &P, float *__restrict__ mean_out,
                                               float *__restrict__ sigma2_out, float *__restrict__ cmd, int shift)
{
    __shared__ float s_buf[2 * kList];  // sparse: indices then weights; dense: a chunk of weights
    __shared__ float s_part[2][kWaves][kLanes];
    __shared__ float s_red[2 * kThreads];
    __shared__ float s_wave[kWaves];
    __shared__ int s_count[kWaves];
    __shared__ float s_mu[kDof * kMaxH];
    __shared__ float s_v[kDof * kMaxH];

    const int t = threadIdx.x;
    const int lane = t & (kLanes - 1), wave = t / kLanes;
    const int N = P.N, H = P.H;
    const int ncol = kDof * H;
    const float beta = P.beta;
    const float *__restrict__ C = P.C;
    int *s_idx = reinterpret_cast<int *>(s_buf);
    float *s_wl = s_buf + kList;

    // min C over all particles, and whether any C is not finite
    float cmin = INFINITY;
    int nonfinite = 0;
    for (int i = t; i < N; i += kThreads) {
        const float c = C[i];
        nonfinite |= !isfinite(c);
        cmin = fminf(cmin, c);
    }
    cmin = wave_min(cmin);
    const int any_nonfinite = __syncthreads_or(nonfinite);
    if (lane == 0) s_wave[wave] = cmin;
    __syncthreads();
    cmin = s_wave[0];
    for (int k = 1; k < kWaves; ++k) cmin = fminf(cmin, s_wave[k]);
    __syncthreads();

    // weights: sum (per thread in stride order, then per wave, then waves in
    // order) and the compacted list of the nonzero ones
    float sw = 0.0f;
    int base = 0;
    for (int c0 = 0; c0 < N; c0 += kThreads) {
        const int i = c0 + t;
        const float w = i < N ? expf(-(C[i] - cmin) / beta) : 0.0f;
        sw += w;
        const bool nz = w > 0.0f;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(nz);
        const int before = __builtin_popcountll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_count[wave] = __builtin_popcountll(bal);
        __syncthreads();
        int off = 0, total = 0;
        for (int k = 0; k < kWaves; ++k) {
            const int c = s_count[k];
            off += k < wave ? c : 0;
            total += c;
        }
        const int pos = base + off + before;
        if (nz && pos < kList) {
            s_idx[pos] = i;
            s_wl[pos] = w;
        }
        base += total;
        __syncthreads();
    }
    sw = wave_sum(sw);
    if (lane == 0) s_wave[wave] = sw;
    __syncthreads();
    float S0 = 0.0f;
    for (int k = 0; k < kWaves; ++k) S0 += s_wave[k];
    const bool ok = !any_nonfinite && S0 > 0.0f && isfinite(S0);
    const int M = base;

    if (M <= kList) {
        // ---- sparse moments over the compacted list -------------------------
        const int rows = kThreads / ncol;  // >= 2 for H <= 64
        const int r = t / ncol, col = t - r * ncol;
        float a1 = 0.0f, a2 = 0.0f;
        if (r < rows && ok) {
            const int j = col / H, h = col - j * H;
            const float mu = P.mean[h * kDof + j];
            const float *__restrict__ U = P.u + (size_t)j * N * H + h;
            int k = r;
            for (; k + 3 * rows < M; k += 4 * rows) {
                float d[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) d[m] = U[(size_t)s_idx[k + m * rows] * H] - mu;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float wd = s_wl[k + m * rows] * d[m];
                    a1 += wd;
                    a2 = fmaf(wd, d[m], a2);
                }
            }
            for (; k < M; k += rows) {
                const float d = U[(size_t)s_idx[k] * H] - mu;
                const float wd = s_wl[k] * d;
                a1 += wd;
                a2 = fmaf(wd, d, a2);
            }
        }
        s_red[t] = a1;
        s_red[kThreads + t] = a2;
        __syncthreads();
        for (int c = t; c < ncol; c += kThreads) {
            float x1 = 0.0f, x2 = 0.0f;
            for (int k = 0; k < rows; ++k) {
                x1 += s_red[k * ncol + c];
                x2 += s_red[kThreads + k * ncol + c];
            }
            s_red[c] = x1;  // rows were read above by this thread only for column c
            s_v[c] = x2;
        }
    } else {
        // ---- dense moments --------------------------------------------------
        const int per = H <= 32 ? 2 : 1;
        const int seg = H <= 32 ? 32 : 64;
        const int slot = lane / seg, h = lane - slot * seg;
        const bool lane_ok = h < H;
        const int groups = (N + per - 1) / per;
        const int j = wave >> 1, half = wave & 1;
        const bool wave_ok = wave < 2 * kDof;
        const int g_lo = half ? groups / 2 : 0, g_hi = half ? groups : groups / 2;
        const float mu = (wave_ok && lane_ok) ? P.mean[h * kDof + j] : 0.0f;
        const float *__restrict__ U = P.u + (size_t)(wave_ok ? j : 0) * N * H;
        float s1 = 0.0f, s2 = 0.0f;
        for (int c0 = 0; c0 < N; c0 += 2 * kList) {
            const int nc = min(2 * kList, N - c0);
            __syncthreads();
            for (int k = t; k < nc; k += kThreads) s_buf[k] = expf(-(C[c0 + k] - cmin) / beta);
            __syncthreads();
            if (!(wave_ok && lane_ok && ok)) continue;
            const int ga = max(g_lo, (c0 + per - 1) / per), gb = min(g_hi, (c0 + nc + per - 1) / per);
            int g = ga;
            for (; g + kUnroll <= gb; g += kUnroll) {
                float uv[kUnroll];
#pragma unroll
                for (int m = 0; m < kUnroll; ++m) {
                    const int i = (g + m) * per + slot;
                    uv[m] = i < N ? U[(size_t)i * H + h] : mu;
                }
#pragma unroll
                for (int m = 0; m < kUnroll; ++m) {
                    const int i = (g + m) * per + slot;
                    const float d = uv[m] - mu;
                    const float wd = (i < N ? s_buf[i - c0] : 0.0f) * d;
                    s1 += wd;
                    s2 = fmaf(wd, d, s2);
                }
            }
            for (; g < gb; ++g) {
                const int i = g * per + slot;
                if (i < N) {
                    const float d = U[(size_t)i * H + h] - mu;
                    const float wd = s_buf[i - c0] * d;
                    s1 += wd;
                    s2 = fmaf(wd, d, s2);
                }
            }
        }
        s_part[0][wave][lane] = s1;
        s_part[1][wave][lane] = s2;
        __syncthreads();
        for (int c = t; c < ncol; c += kThreads) {
            const int jj = c / H, hh = c - jj * H;
            float x1 = 0.0f, x2 = 0.0f;
            for (int w = 2 * jj; w < 2 * jj + 2; ++w)
                for (int sl = 0; sl < per; ++sl) {
                    x1 += s_part[0][w][sl * seg + hh];
                    x2 += s_part[1][w][sl * seg + hh];
                }
            s_red[c] = x1;
            s_v[c] = x2;
        }
    }
    __syncthreads();
    for (int c = t; c < ncol; c += kThreads) {
        const int jj = c / H, hh = c - jj * H;
        const float muo = P.mean[hh * kDof + jj];
        const float m1 = s_red[c] / S0, m2 = s_v[c] / S0;
        const float delta = P.alpha_mu * m1;
        s_mu[c] = ok ? muo + delta : muo;
        s_v[c] = fmaxf(fmaf(delta, delta - 2.0f * m1, m2), 0.0f);  // weighted variance about mu'
    }
    __syncthreads();
    if (t < kDof) {
        float acc = 0.0f;
        for (int k = 0; k < H; ++k) acc += s_v[t * H + k];
        const float old = P.sigma2[t];
        float s2n = old;
        if (ok) s2n = fmaxf(fmaf(P.alpha_sigma, acc / (float)H - old, old), P.sigma2_min);
        P.sigma2[t] = s2n;
        if (sigma2_out) sigma2_out[t] = s2n;
        cmd[t] = s_mu[t * H];
    }
    for (int c = t; c < ncol; c += kThreads) {
        const int jj = c / H, hh = c - jj * H;
        if (mean_out) mean_out[hh * kDof + jj] = s_mu[c];
        P.mean[hh * kDof + jj] = shift ? (hh + 1 < H ? s_mu[c + 1] : 0.0f) : s_mu[c];
    }
    if (t == 0) {
        *P.step = *P.step + 1u;
        if (!ok) atomicOr(P.status, any_nonfinite ? STORM_FLAG_NONFINITE_COST : STORM_FLAG_ZERO_WEIGHT);
    }
}

__global__ __launch_bounds__(kThreads) void update_kernel(ProblemDev P, float *__restrict__ mean_out,
                                                          float *__restrict__ sigma2_out, float *__restrict__ cmd,
                                                          int shift)
{
    update_problem(P, mean_out, sigma2_out, cmd, shift);
}

// One workgroup per problem of a batch; commands go to cmd[p][7].
__global__ __launch_bounds__(kThreads) void update_batch_kernel(const ProblemDev *__restrict__ probs,
                                                                float *__restrict__ cmd, int shift)
{
    const ProblemDev P = load_uniform(probs + blockIdx.x);
    update_problem(P, nullptr, nullptr, cmd + (size_t)blockIdx.x * kDof, shift);
}

}  // namespace

hipError_t launch_update_batch(const ProblemDev *probs, int n_problems, float *cmd, int shift, hipStream_t stream)
{
    hipLaunchKernelGGL(update_batch_kernel, dim3((unsigned)n_problems), dim3(kThreads), 0, stream, probs, cmd,
                       shift);
    return hipGetLastError();
}

hipError_t launch_update(const ProblemDev &P, float *mean_out, float *sigma2_out, float *cmd, int shift,
                         hipStream_t stream)
{
    hipLaunchKernelGGL(update_kernel, dim3(1), dim3(kThreads), 0, stream, P, mean_out, sigma2_out, cmd, shift);
    return hipGetLastError();
}

}  // namespace storm
