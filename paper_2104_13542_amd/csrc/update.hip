// Kernel U: exponentiated-cost policy update of STORM (Sec. 3, Eq. 4-6),
// followed by the next command and the warm-start shift of Alg. 1.
//
//   w_i     = exp(-(C_i - min C) / beta) / sum_k exp(-(C_k - min C) / beta)
//   mu'     = mu + alpha_mu sum_i w_i d_i,          d_i = u_i - mu
//   sigma2' = (1 - alpha_sigma) sigma2
//             + alpha_sigma mean_h sum_i w_i (u_ih - mu'_h)^2   (per joint)
//
// One 1024-thread workgroup per (problem, joint): a joint's new mean and
// variance depend only on the weights and on that joint's controls, so the
// seven joints need no synchronisation with each other; every workgroup
// recomputes min C and the weights of all particles (N exponentials).  The
// joint's H columns are read by rows of threads, row r taking particles r,
// r + R, ... with eight loads in flight per thread.  When few weights are not
// exactly zero (beta small against the spread of C) only those particles are
// gathered, from a list compacted in ascending order.  The variance about the
// new mean comes from the moments about the old one,
// sum w (d - delta)^2 = S2/S0 - 2 delta S1/S0 + delta^2, in one pass.  Every
// sum has a fixed order, so results are bitwise reproducible; there is no
// floating-point atomic and no synchronisation between workgroups.
#include "storm_internal.h"

namespace storm {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / kLanes;
constexpr int kList = 4096;   // capacity of the nonzero-weight list
constexpr int kChunk = 8192;  // weights staged in LDS per chunk (dense path)
constexpr int kUnroll = 8;    // independent loads in flight per thread

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

__device__ __forceinline__ void update_joint(const ProblemDev &P, const int j, float *__restrict__ mean_out,
                                             float *__restrict__ sigma2_out, float *__restrict__ cmd, int shift)
{
    __shared__ float s_buf[kChunk];  // sparse: indices, then weights; dense: a chunk of weights
    __shared__ float s_red[2 * kThreads];
    __shared__ float s_wave[kWaves];
    __shared__ int s_count[kWaves];
    __shared__ float s_mu[kMaxH];
    __shared__ float s_var[kMaxH];

    const int t = threadIdx.x;
    const int lane = t & (kLanes - 1), wave = t / kLanes;
    const int N = P.N, H = P.H;
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

    // weight sum (per thread in stride order, per wave, waves in order) and
    // the list of nonzero weights in ascending particle order
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

    // moments of d = u - mu over the particles, per step h of joint j
    const int rows = kThreads / H;
    const int r = t / H, h = t - r * H;
    const bool act = r < rows && ok;
    const float mu = r < rows ? P.mean[h * kDof + j] : 0.0f;
    const float *__restrict__ U = P.u + (size_t)j * N * H + h;
    float a1[kUnroll], a2[kUnroll];
#pragma unroll
    for (int m = 0; m < kUnroll; ++m) a1[m] = a2[m] = 0.0f;
    if (M <= kList) {
        if (act) {
            int k = r;
            for (; k + (kUnroll - 1) * rows < M; k += kUnroll * rows) {
                float d[kUnroll];
#pragma unroll
                for (int m = 0; m < kUnroll; ++m) d[m] = U[(size_t)s_idx[k + m * rows] * H] - mu;
#pragma unroll
                for (int m = 0; m < kUnroll; ++m) {
                    const float wd = s_wl[k + m * rows] * d[m];
                    a1[m] += wd;
                    a2[m] = fmaf(wd, d[m], a2[m]);
                }
            }
            for (; k < M; k += rows) {
                const float d = U[(size_t)s_idx[k] * H] - mu;
                const float wd = s_wl[k] * d;
                a1[0] += wd;
                a2[0] = fmaf(wd, d, a2[0]);
            }
        }
    } else {
        for (int c0 = 0; c0 < N; c0 += kChunk) {
            const int nc = min(kChunk, N - c0);
            __syncthreads();
            for (int k = t; k < nc; k += kThreads) s_buf[k] = expf(-(C[c0 + k] - cmin) / beta);
            __syncthreads();
            if (!act) continue;
            int k = r;
            for (; k + (kUnroll - 1) * rows < nc; k += kUnroll * rows) {
                float d[kUnroll];
#pragma unroll
                for (int m = 0; m < kUnroll; ++m) d[m] = U[(size_t)(c0 + k + m * rows) * H] - mu;
#pragma unroll
                for (int m = 0; m < kUnroll; ++m) {
                    const float wd = s_buf[k + m * rows] * d[m];
                    a1[m] += wd;
                    a2[m] = fmaf(wd, d[m], a2[m]);
                }
            }
            for (; k < nc; k += rows) {
                const float d = U[(size_t)(c0 + k) * H] - mu;
                const float wd = s_buf[k] * d;
                a1[0] += wd;
                a2[0] = fmaf(wd, d, a2[0]);
            }
        }
    }
    float x1 = 0.0f, x2 = 0.0f;
#pragma unroll
    for (int m = 0; m < kUnroll; ++m) {
        x1 += a1[m];
        x2 += a2[m];
    }
    s_red[t] = x1;
    s_red[kThreads + t] = x2;
    __syncthreads();
    if (t < H) {
        float s1 = 0.0f, s2 = 0.0f;
        for (int k = 0; k < rows; ++k) {
            s1 += s_red[k * H + t];
            s2 += s_red[kThreads + k * H + t];
        }
        const float muo = P.mean[t * kDof + j];
        const float m1 = s1 / S0, m2 = s2 / S0;
        const float delta = P.alpha_mu * m1;
        s_mu[t] = ok ? muo + delta : muo;
        s_var[t] = fmaxf(fmaf(delta, delta - 2.0f * m1, m2), 0.0f);  // weighted variance about mu'
    }
    __syncthreads();
    if (t == 0) {
        float acc = 0.0f;
        for (int k = 0; k < H; ++k) acc += s_var[k];
        const float old = P.sigma2[j];
        float s2n = old;
        if (ok) s2n = fmaxf(fmaf(P.alpha_sigma, acc / (float)H - old, old), P.sigma2_min);
        P.sigma2[j] = s2n;
        if (sigma2_out) sigma2_out[j] = s2n;
        cmd[j] = s_mu[0];
        if (j == 0) {
            *P.step = *P.step + 1u;
            if (!ok) atomicOr(P.status, any_nonfinite ? STORM_FLAG_NONFINITE_COST : STORM_FLAG_ZERO_WEIGHT);
        }
    }
    if (t < H) {
        if (mean_out) mean_out[t * kDof + j] = s_mu[t];
        P.mean[t * kDof + j] = shift ? (t + 1 < H ? s_mu[t + 1] : 0.0f) : s_mu[t];
    }
}

__global__ __launch_bounds__(kThreads) void update_kernel(ProblemDev P, float *__restrict__ mean_out,
                                                          float *__restrict__ sigma2_out, float *__restrict__ cmd,
                                                          int shift)
{
    update_joint(P, blockIdx.x, mean_out, sigma2_out, cmd, shift);
}

// Workgroup (p, j) of a batch; commands go to cmd[p][7].
__global__ __launch_bounds__(kThreads) void update_batch_kernel(const ProblemDev *__restrict__ probs,
                                                                float *__restrict__ cmd, int shift)
{
    const int p = blockIdx.x / kDof, j = blockIdx.x - p * kDof;
    const ProblemDev P = load_uniform(probs + p);
    update_joint(P, j, nullptr, nullptr, cmd + (size_t)p * kDof, shift);
}

}  // namespace

hipError_t launch_update_batch(const ProblemDev *probs, int n_problems, float *cmd, int shift, hipStream_t stream)
{
    hipLaunchKernelGGL(update_batch_kernel, dim3((unsigned)(n_problems * kDof)), dim3(kThreads), 0, stream, probs,
                       cmd, shift);
    return hipGetLastError();
}

hipError_t launch_update(const ProblemDev &P, float *mean_out, float *sigma2_out, float *cmd, int shift,
                         hipStream_t stream)
{
    hipLaunchKernelGGL(update_kernel, dim3(kDof), dim3(kThreads), 0, stream, P, mean_out, sigma2_out, cmd, shift);
    return hipGetLastError();
}

}  // namespace storm
