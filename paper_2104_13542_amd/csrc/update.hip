// Kernel U: exponentiated-cost policy update of STORM (Sec. 3, Eq. 4-6),
// followed by the next command and the warm-start shift of Alg. 1.
//
// One workgroup per joint j (grid = 7).  Each recomputes min C and the weight
// sum over all N particles (cheap, and it keeps the joints independent), then
// reduces the H weighted moments of its joint's controls u[j][*][*]:
//   mean:       mu'_h = (1 - alpha_mu) mu_h + alpha_mu sum_i w_i u_ih
//   covariance: sigma2' = (1 - alpha_sigma) sigma2
//                         + alpha_sigma mean_h sum_i w_i (u_ih - mu'_h)^2
// with w_i = exp(-(C_i - min C) / beta) / sum_k exp(-(C_k - min C) / beta).
// Threads are laid out (row r, step h): row r sums particles r, r + rows, ...
// so a row reads one contiguous H-float segment per particle.  Every sum has
// a fixed order (per-thread sequential, then a fixed tree or row order), so
// results are bitwise reproducible; no floating-point atomics.
#include "storm_internal.h"

namespace storm {
namespace {

constexpr int kThreads = 256;
constexpr int kWChunk = 4096;  // weights staged in LDS per chunk of particles

__device__ __forceinline__ float block_reduce_sum(float x, float *s_red)
{
    const int t = threadIdx.x;
    __syncthreads();
    s_red[t] = x;
    __syncthreads();
    for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
        if (t < stride) s_red[t] += s_red[t + stride];
        __syncthreads();
    }
    const float r = s_red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ float block_reduce_min(float x, float *s_red)
{
    const int t = threadIdx.x;
    __syncthreads();
    s_red[t] = x;
    __syncthreads();
    for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
        if (t < stride) s_red[t] = fminf(s_red[t], s_red[t + stride]);
        __syncthreads();
    }
    const float r = s_red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kThreads) void update_kernel(ProblemDev P, float *__restrict__ mean_out,
                                                          float *__restrict__ sigma2_out, float *__restrict__ cmd,
                                                          int shift)
{
    __shared__ float s_w[kWChunk];
    __shared__ float s_red[kThreads];
    __shared__ float s_mu[kMaxH];
    __shared__ int s_bad;

    const int j = blockIdx.x;
    const int t = threadIdx.x;
    const int N = P.N, H = P.H;
    const float beta = P.beta;
    const float *__restrict__ C = P.C;
    const float *__restrict__ U = P.u + (size_t)j * N * H;

    if (t == 0) s_bad = 0;
    __syncthreads();
    float cmin = INFINITY;
    bool nonfinite = false;
    for (int i = t; i < N; i += kThreads) {
        const float c = C[i];
        nonfinite |= !isfinite(c);
        cmin = fminf(cmin, c);
    }
    if (nonfinite) atomicOr(&s_bad, 1);
    cmin = block_reduce_min(cmin, s_red);
    float sw = 0.0f;
    for (int i = t; i < N; i += kThreads) sw += expf(-(C[i] - cmin) / beta);
    sw = block_reduce_sum(sw, s_red);
    const bool bad = s_bad != 0;
    const bool ok = !bad && sw > 0.0f && isfinite(sw);

    const int rows = kThreads / H;
    const int r = t / H;
    const int hh = t - r * H;
    const bool act = r < rows;

    // Mean (Eq. 4).
    float acc = 0.0f;
    if (ok) {
        for (int c0 = 0; c0 < N; c0 += kWChunk) {
            const int nc = min(kWChunk, N - c0);
            __syncthreads();
            for (int k = t; k < nc; k += kThreads) s_w[k] = expf(-(C[c0 + k] - cmin) / beta);
            __syncthreads();
            if (act)
                for (int k = r; k < nc; k += rows) acc = fmaf(s_w[k], U[(size_t)(c0 + k) * H + hh], acc);
        }
    }
    __syncthreads();
    s_red[t] = act ? acc : 0.0f;
    __syncthreads();
    if (t < H) {
        float s = 0.0f;
        for (int k = 0; k < rows; ++k) s += s_red[k * H + t];
        const float mu_old = P.mean[t * kDof + j];
        s_mu[t] = ok ? fmaf(P.alpha_mu, s / sw - mu_old, mu_old) : mu_old;
    }
    __syncthreads();

    // Covariance about the updated mean (Eq. 5), diagonal and shared over h.
    float acc2 = 0.0f;
    if (ok) {
        const float mu = act ? s_mu[hh] : 0.0f;
        for (int c0 = 0; c0 < N; c0 += kWChunk) {
            const int nc = min(kWChunk, N - c0);
            __syncthreads();
            for (int k = t; k < nc; k += kThreads) s_w[k] = expf(-(C[c0 + k] - cmin) / beta);
            __syncthreads();
            if (act)
                for (int k = r; k < nc; k += rows) {
                    const float d = U[(size_t)(c0 + k) * H + hh] - mu;
                    acc2 = fmaf(s_w[k] * d, d, acc2);
                }
        }
    }
    __syncthreads();
    s_red[t] = act ? acc2 : 0.0f;
    __syncthreads();
    if (t < H) {
        float s = 0.0f;
        for (int k = 0; k < rows; ++k) s += s_red[k * H + t];
        s_w[t] = s;  // per-step weighted second moment (unnormalised)
    }
    __syncthreads();
    if (t == 0) {
        float s = 0.0f;
        for (int k = 0; k < H; ++k) s += s_w[k];
        const float old = P.sigma2[j];
        float s2 = old;
        if (ok) s2 = fmaxf(fmaf(P.alpha_sigma, (s / sw) / (float)H - old, old), P.sigma2_min);
        P.sigma2[j] = s2;
        if (sigma2_out) sigma2_out[j] = s2;
        cmd[j] = s_mu[0];
        if (j == 0) {
            *P.step = *P.step + 1u;
            if (!ok) atomicOr(P.status, bad ? STORM_FLAG_NONFINITE_COST : STORM_FLAG_ZERO_WEIGHT);
        }
    }
    if (t < H) {
        if (mean_out) mean_out[t * kDof + j] = s_mu[t];
        const float next = shift ? (t + 1 < H ? s_mu[t + 1] : 0.0f) : s_mu[t];
        P.mean[t * kDof + j] = next;
    }
}

}  // namespace

hipError_t launch_update(const ProblemDev &P, float *mean_out, float *sigma2_out, float *cmd, int shift,
                         hipStream_t stream)
{
    hipLaunchKernelGGL(update_kernel, dim3(kDof), dim3(kThreads), 0, stream, P, mean_out, sigma2_out, cmd, shift);
    return hipGetLastError();
}

}  // namespace storm
