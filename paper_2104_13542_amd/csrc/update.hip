// Kernel U: exponentiated-cost policy update of STORM (Sec. 3, Eq. 4-6),
// followed by the next command and the warm-start shift of Alg. 1.
//
//   w_i     = exp(-(C_i - min C) / beta) / sum_k exp(-(C_k - min C) / beta)
//   mu'     = mu + alpha_mu sum_i w_i d_i,          d_i = u_i - mu
//   sigma2' = (1 - alpha_sigma) sigma2
//             + alpha_sigma mean_h sum_i w_i (u_ih - mu'_h)^2   (per joint)
//
// One workgroup of 1024 threads per problem.  Weights are staged in LDS in
// chunks; threads are laid out (row r, column (j, h)) and row r accumulates
// the particles r, r + R, ... of its column with four independent partial
// sums, so that each thread keeps four loads in flight.  The variance about
// the new mean comes from the moments about the old one,
// sum w (d - delta)^2 = S2/S0 - 2 delta S1/S0 + delta^2, in one pass.  Every
// sum has a fixed order (results are bitwise reproducible); no atomics on
// floating-point data and no cross-workgroup synchronisation.
#include "storm_internal.h"

namespace storm {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / kLanes;
constexpr int kWChunk = 8192;  // weights staged in LDS per chunk of particles

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

__global__ __launch_bounds__(kThreads) void update_kernel(ProblemDev P, float *__restrict__ mean_out,
                                                          float *__restrict__ sigma2_out, float *__restrict__ cmd,
                                                          int shift)
{
    __shared__ float s_w[kWChunk];
    __shared__ float s_red[2 * kThreads];
    __shared__ float s_wave[kWaves];
    __shared__ float s_mu[kDof * kMaxH];
    __shared__ float s_v[kDof * kMaxH];

    const int t = threadIdx.x;
    const int lane = t & (kLanes - 1), wave = t / kLanes;
    const int N = P.N, H = P.H;
    const int ncol = kDof * H;
    const float beta = P.beta;
    const float *__restrict__ C = P.C;

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

    // weight sum: per-thread sequential, then per wave, then over waves in order
    float sw = 0.0f;
    for (int i = t; i < N; i += kThreads) sw += expf(-(C[i] - cmin) / beta);
    sw = wave_sum(sw);
    if (lane == 0) s_wave[wave] = sw;
    __syncthreads();
    float S0 = 0.0f;
    for (int k = 0; k < kWaves; ++k) S0 += s_wave[k];
    const bool ok = !any_nonfinite && S0 > 0.0f && isfinite(S0);

    // weighted first and second moments of d = u - mu per (joint, step) column
    const int rows = kThreads / ncol;  // >= 2 for H <= 64
    const int r = t / ncol, col = t - r * ncol;
    const bool act = r < rows;
    const int j = col / H, h = col - j * H;
    const float mu = act ? P.mean[h * kDof + j] : 0.0f;
    const float *__restrict__ U = P.u + (size_t)j * N * H + h;
    float a1[4] = {0.0f, 0.0f, 0.0f, 0.0f}, a2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int c0 = 0; c0 < N; c0 += kWChunk) {
        const int nc = min(kWChunk, N - c0);
        __syncthreads();
        for (int k = t; k < nc; k += kThreads) s_w[k] = expf(-(C[c0 + k] - cmin) / beta);
        __syncthreads();
        if (act && ok) {
            int k = r;
            for (; k + 3 * rows < nc; k += 4 * rows) {
                float d[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) d[m] = U[(size_t)(c0 + k + m * rows) * H] - mu;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const float wd = s_w[k + m * rows] * d[m];
                    a1[m] += wd;
                    a2[m] = fmaf(wd, d[m], a2[m]);
                }
            }
            for (; k < nc; k += rows) {
                const float d = U[(size_t)(c0 + k) * H] - mu;
                const float wd = s_w[k] * d;
                a1[0] += wd;
                a2[0] = fmaf(wd, d, a2[0]);
            }
        }
    }
    s_red[t] = (a1[0] + a1[1]) + (a1[2] + a1[3]);
    s_red[kThreads + t] = (a2[0] + a2[1]) + (a2[2] + a2[3]);
    __syncthreads();
    if (t < ncol) {
        float s1 = 0.0f, s2 = 0.0f;
        for (int k = 0; k < rows; ++k) {
            s1 += s_red[k * ncol + t];
            s2 += s_red[kThreads + k * ncol + t];
        }
        const float muo = P.mean[h * kDof + j];
        const float m1 = s1 / S0, m2 = s2 / S0;
        const float delta = P.alpha_mu * m1;
        s_mu[t] = ok ? muo + delta : muo;
        s_v[t] = fmaxf(fmaf(delta, delta - 2.0f * m1, m2), 0.0f);  // weighted variance about mu'
    }
    __syncthreads();
    if (t < kDof) {
        float acc = 0.0f;
        for (int k = 0; k < H; ++k) acc += s_v[t * H + k];
        const float old = P.sigma2[t];
        float s2 = old;
        if (ok) s2 = fmaxf(fmaf(P.alpha_sigma, acc / (float)H - old, old), P.sigma2_min);
        P.sigma2[t] = s2;
        if (sigma2_out) sigma2_out[t] = s2;
        cmd[t] = s_mu[t * H];
    }
    if (t < ncol) {
        if (mean_out) mean_out[h * kDof + j] = s_mu[t];
        P.mean[h * kDof + j] = shift ? (h + 1 < H ? s_mu[t + 1] : 0.0f) : s_mu[t];
    }
    if (t == 0) {
        *P.step = *P.step + 1u;
        if (!ok) atomicOr(P.status, any_nonfinite ? STORM_FLAG_NONFINITE_COST : STORM_FLAG_ZERO_WEIGHT);
    }
}

}  // namespace

hipError_t launch_update(const ProblemDev &P, float *mean_out, float *sigma2_out, float *cmd, int shift,
                         hipStream_t stream)
{
    hipLaunchKernelGGL(update_kernel, dim3(1), dim3(kThreads), 0, stream, P, mean_out, sigma2_out, cmd, shift);
    return hipGetLastError();
}

}  // namespace storm
