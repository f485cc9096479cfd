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
// r + R, ...  Three ways to gather them:
//   registers  (N <= 32 R): every thread loads its up to 32 controls at the
//              start, together with the costs, so the only global-memory
//              latency on the path is the first one;
//   list       (at most 4096 weights not exactly zero, beta small against the
//              spread of C): only those particles, from a list compacted in
//              ascending order;
//   dense      otherwise: all particles, weights staged in LDS by chunks,
//              eight loads in flight per thread.
// The variance about the new mean comes from the moments about the old one,
// sum w (d - delta)^2 = S2/S0 - 2 delta S1/S0 + delta^2, in one pass.  Wave
// reductions use DPP lane moves; every sum has a fixed order, so results are
// bitwise reproducible; there is no floating-point atomic and no
// synchronisation between workgroups.
#include "storm_internal.h"

namespace storm {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / kLanes;
constexpr int kList = 4096;   // capacity of the nonzero-weight list
constexpr int kChunk = 8192;  // weights staged in LDS per chunk (dense path)
constexpr int kUnroll = 8;    // independent loads in flight per thread
constexpr int kRegU = 32;     // most controls per thread held in registers (register path)

// Full-wave reductions through DPP lane moves (quad permutes, half-row and
// row mirrors, then the row broadcasts that carry each row's result into the
// next); lane 63, which every step feeds, holds the result, read back into
// an SGPR.  The order of the operations is fixed.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_move(int x)
{
    return __builtin_amdgcn_mov_dpp(x, kCtrl, kRowMask, 0xf, false);
}

__device__ __forceinline__ float wave_sum(float x)
{
    x += __int_as_float(dpp_move<0xb1, 0xf>(__float_as_int(x)));
    x += __int_as_float(dpp_move<0x4e, 0xf>(__float_as_int(x)));
    x += __int_as_float(dpp_move<0x141, 0xf>(__float_as_int(x)));
    x += __int_as_float(dpp_move<0x140, 0xf>(__float_as_int(x)));
    x += __int_as_float(dpp_move<0x142, 0xa>(__float_as_int(x)));
    x += __int_as_float(dpp_move<0x143, 0xc>(__float_as_int(x)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// IEEE bits mapped so that signed-integer order is float order (negative
// values have their magnitude bits flipped); the map is its own inverse.
__device__ __forceinline__ int ordered(int b) { return b ^ (int)((uint32_t)(b >> 31) >> 1); }

__device__ __forceinline__ float wave_min(float x)
{
    int b = ordered(__float_as_int(x));
    b = min(b, dpp_move<0xb1, 0xf>(b));
    b = min(b, dpp_move<0x4e, 0xf>(b));
    b = min(b, dpp_move<0x141, 0xf>(b));
    b = min(b, dpp_move<0x140, 0xf>(b));
    b = min(b, dpp_move<0x142, 0xa>(b));
    b = min(b, dpp_move<0x143, 0xc>(b));
    return __int_as_float(ordered(__builtin_amdgcn_readlane(b, 63)));
}

// x moved into VGPRs at this point (a wave-uniform value the compiler
// would otherwise keep, or reload, as a scalar).
template <typename T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// The same for a pointer, kept a global-memory pointer so that accesses
// through it stay global (not flat) instructions.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ global_ptr<T> global_in_vgpr(T *p)
{
    global_ptr<T> g = (global_ptr<T>)p;
    asm volatile("" : "+v"(g));
    return g;
}

// Minimum of v over the workgroup (all threads get it).
__device__ __forceinline__ float block_min(float v, float *s_wave, int lane, int wave)
{
    v = wave_min(v);
    if (lane == 0) s_wave[wave] = v;
    __syncthreads();
    float m = s_wave[0];
    for (int k = 1; k < kWaves; ++k) m = fminf(m, s_wave[k]);
    __syncthreads();
    return m;
}

// Workgroup LDS of the update, declared once per kernel.
struct UpdateLds {
    float buf[kChunk];  // register path: weights; list: indices, then weights; dense: a chunk
    float red[2 * kThreads];
    float wave[kWaves];
    float wsum[kWaves];
    int count[kWaves];
    float mold[kMaxH];
};

// Controls per thread of the register path for N particles over `rows`
// rows: the smallest of 8, 16 and 32 that holds them (0: other paths).
__host__ __device__ inline int update_slots(int N, int H)
{
    const int rows = kThreads / H;
    if (N > 2 * kThreads) return 0;
    for (int k = 8; k <= kRegU; k *= 2)
        if (N <= k * rows && k * rows <= kChunk) return k;
    return 0;
}

// `cov` is P.cov_step, passed apart so that the plain kernel can fix it at
// compile time; kSlots the register path's controls per thread
// (update_slots), 32 when that path is not taken.
template <int kSlots>
__device__ __forceinline__ void update_joint(const ProblemDev &P, const int j, float *__restrict__ mean_out,
                                             float *__restrict__ sigma2_out, float *__restrict__ cmd, int shift,
                                             const bool cov, const float alpha_mu, const float alpha_sigma,
                                             const float sigma2_min, UpdateLds &L)
{
    float *s_buf = L.buf;
    float *s_red = L.red;
    float *s_wave = L.wave;
    float *s_wsum = L.wsum;
    int *s_count = L.count;
    float *s_mold = L.mold;

    const int t = threadIdx.x;
    const int lane = t & (kLanes - 1), wave = __builtin_amdgcn_readfirstlane(t / kLanes);
    const int N = P.N, H = P.H;
    const float beta = P.beta;
    const float *__restrict__ C = P.C;
    int *s_idx = reinterpret_cast<int *>(s_buf);
    float *s_wl = s_buf + kList;

    // thread (r, h): step h of particles r, r + rows, ...
    const int rows = kThreads / H;
    const int r = t / H, h = t - r * H;
    const bool in_rows = r < rows;
    const float *__restrict__ U = P.u + (size_t)j * N * H + h;
    const bool regs = N <= kSlots * rows && N <= 2 * kThreads && kSlots * rows <= kChunk;
    const float nib = -1.0f / beta;

    // register path: the costs, then every control load, all in flight at
    // once.  The controls come through a buffer resource bounded by the
    // joint's N H values: slots past the last particle read 0 and cost no
    // address arithmetic (the load returns the raw 32 bits).
    float c0 = INFINITY, c1 = INFINITY;
    float uu[kSlots];
    if (regs) {
        if (t < N) c0 = C[t];
        if (t + kThreads < N) c1 = C[t + kThreads];
        const __amdgpu_buffer_rsrc_t ub = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(P.u + (size_t)j * N * H), (short)0, N * H * (int)sizeof(float), 0x00020000);
        const int stride = rows * H * (int)sizeof(float);
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            uu[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ub, t * 4 + k * stride, 0, 0));
    }
    const float mu = in_rows ? P.mean[h * kDof + j] : 0.0f;
    // What the tail reads is fetched now, with the first loads, since each
    // would add a memory round trip to the tail: the old variances and the
    // noise counter through vector loads (waited for only where they are
    // used); the scalars go into VGPRs, because the kernel runs at its SGPR
    // limit and the compiler would otherwise reload each from the kernel
    // arguments there, one scalar-memory round trip after another.
    const float sig_old = cov ? (t < H ? vector_load_f32(P.sigma2 + t * kDof + j) : 0.0f) : vector_load_f32(P.sigma2 + j);
    const float sig_init = cov && shift ? vector_load_f32(P.tables + kTabSig0 + j) : 0.0f;
    const uint32_t step0 = vector_load_u32(P.step);
    const global_ptr<float> mean_p = global_in_vgpr(P.mean), sigma2_p = global_in_vgpr(P.sigma2);
    const global_ptr<float> cmd_p = global_in_vgpr(cmd), mean_out_p = global_in_vgpr(mean_out),
                            sigma2_out_p = global_in_vgpr(sigma2_out);
    const global_ptr<uint32_t> step_p = global_in_vgpr(P.step);
    shift = in_vgpr(shift);
    const float a_mu = in_vgpr(alpha_mu), a_sigma = in_vgpr(alpha_sigma), s2_min = in_vgpr(sigma2_min);

    float S0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
    int any_nonfinite = 0;
    bool ok = false;
    if (regs) {
        // min C and the non-finite flag in one exchange, then the weights
        // and their sum in a second (separate LDS slots: no third barrier)
        const bool bad = (t < N && !isfinite(c0)) || (t + kThreads < N && !isfinite(c1));
        const uint64_t bad_lanes = __builtin_amdgcn_ballot_w64(bad);
        const float wmin = wave_min(fminf(c0, c1));
        if (lane == 0) {
            s_wave[wave] = wmin;
            s_count[wave] = bad_lanes != 0;
        }
        __syncthreads();
        float cmin = s_wave[0];
        any_nonfinite = s_count[0];
        for (int k = 1; k < kWaves; ++k) {
            cmin = fminf(cmin, s_wave[k]);
            any_nonfinite |= s_count[k];
        }
        const float w0 = t < N ? expf((c0 - cmin) * nib) : 0.0f;
        const float w1 = t + kThreads < N ? expf((c1 - cmin) * nib) : 0.0f;
        s_buf[t] = w0;
        s_buf[t + kThreads] = w1;
        for (int i = 2 * kThreads + t; i < kSlots * rows; i += kThreads) s_buf[i] = 0.0f;  // slots past N
        const float sw = wave_sum(w0 + w1);
        if (lane == 0) s_wsum[wave] = sw;
        __syncthreads();
        for (int k = 0; k < kWaves; ++k) S0 += s_wsum[k];
        ok = !any_nonfinite && S0 > 0.0f && isfinite(S0);
        // straight-line over the 32 slots (weight 0 and control 0 past the
        // last particle) so that every LDS read is in flight before the first use
        float a1[4] = {0.0f, 0.0f, 0.0f, 0.0f}, a2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (in_rows && ok) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                const float d = uu[k] - mu;
                const float wd = s_buf[r + k * rows] * d;
                a1[k & 3] += wd;
                a2[k & 3] = fmaf(wd, d, a2[k & 3]);
            }
        }
        x1 = (a1[0] + a1[1]) + (a1[2] + a1[3]);
        x2 = (a2[0] + a2[1]) + (a2[2] + a2[3]);
    } else {
        // min C over all particles, and whether any C is not finite
        float cmin = INFINITY;
        int nonfinite = 0;
        for (int i = t; i < N; i += kThreads) {
            const float c = C[i];
            nonfinite |= !isfinite(c);
            cmin = fminf(cmin, c);
        }
        any_nonfinite = __syncthreads_or(nonfinite);
        cmin = block_min(cmin, s_wave, lane, wave);

        // weight sum (per thread in stride order, per wave, waves in order)
        // and the list of nonzero weights in ascending particle order
        float sw = 0.0f;
        int base = 0;
        for (int c0 = 0; c0 < N; c0 += kThreads) {
            const int i = c0 + t;
            const float w = i < N ? expf((C[i] - cmin) * nib) : 0.0f;
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
        for (int k = 0; k < kWaves; ++k) S0 += s_wave[k];
        ok = !any_nonfinite && S0 > 0.0f && isfinite(S0);
        const int M = base;

        // moments of d = u - mu over the particles, per step h of joint j
        const bool act = in_rows && ok;
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
                for (int k = t; k < nc; k += kThreads) s_buf[k] = expf((C[c0 + k] - cmin) * nib);
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
#pragma unroll
        for (int m = 0; m < kUnroll; ++m) {
            x1 += a1[m];
            x2 += a2[m];
        }
    }

    // Wave 0 finishes alone: lane h adds the rows of step h in order (S1, S2),
    // forms the new mean and the variance about it, then one wave sum gives
    // the variance over the horizon; no further workgroup barrier.
    s_red[t] = x1;
    s_red[kThreads + t] = x2;
    if (r == 0) s_mold[h] = mu;  // stored late: an early store would wait for every load in flight
    __syncthreads();
    if (wave == 0) {
        const float inv_S0 = 1.0f / S0;
        float s1 = 0.0f, s2 = 0.0f, muo = 0.0f;
        if (lane < H) {
            for (int k = 0; k < rows; ++k) {
                s1 += s_red[k * H + lane];
                s2 += s_red[kThreads + k * H + lane];
            }
            muo = s_mold[lane];
        }
        const float m1 = s1 * inv_S0, m2 = s2 * inv_S0;
        const float delta = a_mu * m1;
        const float mu_new = ok ? muo + delta : muo;
        const float var = lane < H ? fmaxf(fmaf(delta, delta - 2.0f * m1, m2), 0.0f) : 0.0f;  // about mu'
        const float acc = wave_sum(var);
        // the new mean of step h + 1 (the shifted warm start), 0 past the end
        const float mu_next = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(mu_new), 0x130, 0xf, 0xf,
                                                                         true));  // wave_shl:1
        if (lane == 0) {
            if (j == 0) {
                // the increment here, not at the load (where it would wait for
                // every load in flight), and before the other stores (whose
                // completion a wait for the load would otherwise include)
                uint32_t next = step0;
                asm volatile("" : "+v"(next));
                *step_p = next + 1u;
                if (!ok) atomicOr(P.status, any_nonfinite ? STORM_FLAG_NONFINITE_COST : STORM_FLAG_ZERO_WEIGHT);
            }
            if (!cov) {
                float s2n = sig_old;
                if (ok) s2n = fmaxf(fmaf(a_sigma, acc / (float)H - sig_old, sig_old), s2_min);
                sigma2_p[j] = s2n;
                if (sigma2_out_p) sigma2_out_p[j] = s2n;
            }
            cmd_p[j] = mu_new;
        }
        if (lane < H) {
            if (mean_out_p) mean_out_p[lane * kDof + j] = mu_new;
            mean_p[lane * kDof + j] = shift ? (lane + 1 < H ? mu_next : 0.0f) : mu_new;
        }
        if (cov) {
            // Eq. 5 per step: lane h updates sigma^2[h][j] from the variance at
            // step h; the shift moves it one step, sigma_init^2 appended
            const float old = sig_old;  // sigma^2[lane][j] (0 past H)
            const float s2n = ok ? fmaxf(fmaf(a_sigma, var - old, old), s2_min) : old;
            const float s2_next = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s2n), 0x130, 0xf, 0xf,
                                                                             true));  // wave_shl:1
            if (lane < H) {
                if (sigma2_out_p) sigma2_out_p[lane * kDof + j] = s2n;
                sigma2_p[lane * kDof + j] = shift ? (lane + 1 < H ? s2_next : sig_init) : s2n;
            }
        }
    }
}

// The fields the first loads depend on, and the scalars of the tail, come
// first, as scalar arguments, so that they are preloaded into SGPRs (16
// dwords); the rest of the problem follows in P.  kCov: one variance per
// (step, joint) instead of one per joint.
template <bool kCov, int kSlots>
__global__ __launch_bounds__(kThreads) void update_kernel(float *C, float *u, float *mean, float *sigma2, int32_t N,
                                                          int32_t H, float beta, float alpha_mu, float alpha_sigma,
                                                          float sigma2_min, int shift, ProblemDev P,
                                                          float *__restrict__ mean_out, float *__restrict__ sigma2_out,
                                                          float *__restrict__ cmd)
{
    __shared__ UpdateLds L;
    ProblemDev Q = P;
    Q.C = C;
    Q.u = u;
    Q.mean = mean;
    Q.sigma2 = sigma2;
    Q.N = N;
    Q.H = H;
    Q.beta = beta;
    update_joint<kSlots>(Q, blockIdx.x, mean_out, sigma2_out, cmd, shift, kCov, alpha_mu, alpha_sigma, sigma2_min, L);
}

// Workgroup (p, j) of a batch; commands go to cmd[p][7].
__global__ __launch_bounds__(kThreads) void update_batch_kernel(const ProblemDev *__restrict__ probs,
                                                                float *__restrict__ cmd, int shift)
{
    __shared__ UpdateLds L;
    const int p = blockIdx.x / kDof, j = blockIdx.x - p * kDof;
    const ProblemDev P = load_uniform(probs + p);
    const int slots = update_slots(P.N, P.H);
    float *c = cmd + (size_t)p * kDof;
    if (slots == 8)
        update_joint<8>(P, j, nullptr, nullptr, c, shift, P.cov_step != 0u, P.alpha_mu, P.alpha_sigma, P.sigma2_min,
                          L);
    else if (slots == 16)
        update_joint<16>(P, j, nullptr, nullptr, c, shift, P.cov_step != 0u, P.alpha_mu, P.alpha_sigma, P.sigma2_min,
                          L);
    else
        update_joint<32>(P, j, nullptr, nullptr, c, shift, P.cov_step != 0u, P.alpha_mu, P.alpha_sigma, P.sigma2_min,
                          L);
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
    const int slots = update_slots(P.N, P.H);
    auto kernel = P.cov_step ? (slots == 8    ? update_kernel<true, 8>
                                : slots == 16 ? update_kernel<true, 16>
                                              : update_kernel<true, 32>)
                             : (slots == 8    ? update_kernel<false, 8>
                                : slots == 16 ? update_kernel<false, 16>
                                              : update_kernel<false, 32>);
    hipLaunchKernelGGL(kernel, dim3(kDof), dim3(kThreads), 0, stream, P.C, P.u, P.mean, P.sigma2, P.N, P.H, P.beta,
                       P.alpha_mu, P.alpha_sigma, P.sigma2_min, shift, P, mean_out, sigma2_out, cmd);
    return hipGetLastError();
}

}  // namespace storm
