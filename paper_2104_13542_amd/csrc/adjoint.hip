// Kernel A: reverse-mode gradient of the expected horizon cost
//   J(mu) = (1/N) sum_i C_i(mu + sigma * eps_i),  eps held fixed,
// with respect to the mean control sequence mu [H][7] (not in the paper: the
// differentiable form).  Differentiated terms: pose (Eq. 9), joint and
// velocity limits (Eq. 11 form) and stop (Eq. 10); hinge and norm kinks take
// subgradient 0.  States are recomputed from mu and the noise, never stored.
//
// Per 64-lane tile (ppt particles x H steps), eight wavefronts:
//   A   noise, controls, the forward integrator and sin/cos of q (as kernel R)
//   B   waves 0-2: forward kinematics to LDS, one frame row each; wave 3:
//       limit costs and their gradients with respect to q and v
//   C   wave 0: pose cost and dC/dq through the Jacobian columns,
//       dp/dq_k = z_k x (p - o_k) and dR/dq_k = [z_k]x R; horizon cost
//   D   waves 0-6: the integrator backwards, two segmented suffix sums:
//       dC/dv_k = gv_k + dt_k sum_{h>=k} gq_h,  dC/du_m = dt_m sum_{k>=m} dC/dv_k
//   E   per (joint, step) sum over the tile's particles -> partial gradient
// A second kernel adds the tile partials per (joint, step) in a fixed order
// and, when refining, takes an Adam step (Kingma and Ba, 2015) on mu.
#include "kinematics.h"
#include "sampling.h"

namespace storm {
namespace {

constexpr int kAdjWaves = 8;
constexpr int kRedThreads = 1024;

// Phases A-D for one tile, then the tile's share of the chunk partials:
// acc (thread t < 7H: joint t / H, step t % H) gains the sum over the tile's
// particles of dC/du, cacc (thread 0) the tile's horizon-cost sum.
__device__ __forceinline__ void adjoint_tile(const ProblemDev &P, const RobotDev &R, const int tile,
                                             const float *__restrict__ x0, const float *__restrict__ goal,
                                             const float *__restrict__ mean, const float *__restrict__ noise,
                                             float &acc, float &cacc)
{
    __shared__ float s_eps[8][kLanes];
    __shared__ float s_q[kDof][kLanes];
    __shared__ float s_v[kDof][kLanes];
    __shared__ float s_fr[kFrames * 12][kLanes];
    __shared__ float s_sc[2 * kDof][kLanes];  // sin q_j, cos q_j
    __shared__ float s_gl[kDof][kLanes];  // limit-cost gradient d c / d q
    __shared__ float s_gv[kDof][kLanes];  // limit and stop gradient d c / d v
    __shared__ float s_gq[kDof][kLanes];  // horizon-weighted d C / d q
    __shared__ float s_gu[kDof][kLanes];  // d C / d u
    __shared__ float s_cl[kLanes];        // weighted limit and stop costs
    __shared__ float s_Cp[kLanes];        // horizon cost per particle of the tile

    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = P.N, H = P.H;
    const int pl = lane / H;
    const int h = lane - pl * H;
    const int i = tile * P.ppt + pl;
    const bool valid = pl < P.ppt && i < N;
    const bool live = valid && i < N - P.n_null;
    const uint32_t mask = P.grad_mask;
    const float *__restrict__ tab = P.tables;
    const float dt_h = tab[kTabDt + h];
    const float hw_h = tab[kTabHw + h];

    // ---- A: noise, controls, integrator ---------------------------------------
    if (wave < 2) {
        float e[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (live) standard_noise4(P, noise, wave, i, h, *P.last_step, e);
#pragma unroll
        for (int m = 0; m < 4; ++m) s_eps[4 * wave + m][lane] = e[m];
    }
    __syncthreads();
    if (wave < kDof) {
        const int j = wave;
        float e = s_eps[j][lane];
        // the comb filter on the sampled Gaussian particles' noise, as in kernel R
        const bool comb = P.comb && noise == nullptr && live && i >= P.n_halton;
        if (__builtin_amdgcn_ballot_w64(comb) != 0) {
            const float f = comb_noise(&s_eps[j][0], lane, h, H, tab);
            if (comb) e = f;
        }
        float u = 0.0f;
        if (live) u = fmaf(sqrtf(P.cov_step ? P.sigma2[h * kDof + j] : P.sigma2[j]), e, mean[h * kDof + j]);
        const float v = x0[kDof + j] + segmented_scan(dt_h * u, h, H);
        const float q = x0[j] + segmented_scan(dt_h * v, h, H);
        s_q[j][lane] = q;
        s_v[j][lane] = v;
        float sq, cq;
        sincosf(q, &sq, &cq);
        s_sc[2 * j][lane] = sq;
        s_sc[2 * j + 1][lane] = cq;
    }
    __syncthreads();

    // ---- B: kinematics, one frame row per wave | limit costs and gradients ---
    if (wave < 3) {
        const int row = wave;
        float r[3] = {row == 0 ? 1.0f : 0.0f, row == 1 ? 1.0f : 0.0f, row == 2 ? 1.0f : 0.0f};
        float p = 0.0f;
#pragma unroll
        for (int f = 0; f < kFrames; ++f) {
            float st = 0.0f, ct = 1.0f;
            if (f < kDof) {
                st = s_sc[2 * f][lane];
                ct = s_sc[2 * f + 1][lane];
            }
            dh_step_row(r, p, R.ca[f], R.sa[f], R.a[f], R.d[f], ct, st);
#pragma unroll
            for (int c = 0; c < 3; ++c) s_fr[f * 12 + row * 3 + c][lane] = r[c];
            s_fr[f * 12 + 9 + row][lane] = p;
        }
    } else if (wave == 3) {
        float ej[kDof], ev[kDof], es[kDof];
        float nj = 0.0f, nv = 0.0f, ns = 0.0f;
        const float vs = tab[kTabVstop + h];
#pragma unroll
        for (int j = 0; j < kDof; ++j) {
            const float q = s_q[j][lane], v = s_v[j][lane];
            // signed violations: negative below the band, positive above
            ej[j] = fminf(q - tab[kTabJlo + j], 0.0f) + fmaxf(q - tab[kTabJhi + j], 0.0f);
            ev[j] = fminf(v - tab[kTabVlo + j], 0.0f) + fmaxf(v - tab[kTabVhi + j], 0.0f);
            es[j] = fmaxf(fabsf(v) - vs, 0.0f);
            nj = fmaf(ej[j], ej[j], nj);
            nv = fmaf(ev[j], ev[j], nv);
            ns = fmaf(es[j], es[j], ns);
        }
        nj = (mask & STORM_COST_JOINT) ? fast_sqrt(nj) : 0.0f;
        nv = (mask & STORM_COST_VEL) ? fast_sqrt(nv) : 0.0f;
        ns = (mask & STORM_COST_STOP) ? fast_sqrt(ns) : 0.0f;
        const float kj = nj > 0.0f ? P.a_joint / nj : 0.0f;
        const float kv = nv > 0.0f ? P.a_vel / nv : 0.0f;
        const float ks = ns > 0.0f ? P.a_stop / ns : 0.0f;
#pragma unroll
        for (int j = 0; j < kDof; ++j) {
            const float v = s_v[j][lane];
            s_gl[j][lane] = kj * ej[j];
            s_gv[j][lane] = fmaf(kv, ev[j], ks * es[j] * (v > 0.0f ? 1.0f : -1.0f));
        }
        s_cl[lane] = fmaf(P.a_joint, nj, fmaf(P.a_vel, nv, P.a_stop * ns));
    }
    __syncthreads();

    // ---- C: pose cost and its gradient; horizon cost ------------------------
    if (wave == 0) {
        float gq[kDof];
#pragma unroll
        for (int k = 0; k < kDof; ++k) gq[k] = s_gl[k][lane];
        float cost = s_cl[lane];
        if (mask & STORM_COST_POSE) {
            float Re[9], pe[3];
#pragma unroll
            for (int c = 0; c < 9; ++c) Re[c] = s_fr[7 * 12 + c][lane];
#pragma unroll
            for (int c = 0; c < 3; ++c) pe[c] = s_fr[7 * 12 + 9 + c][lane];
            // position: e = diag(a2) R_g^T (p - p_g), gradient g_p = w_pos R_g diag(a2) e / |e|
            float e[3], pos2 = 0.0f;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                e[r] = P.alpha_pos[r] * fmaf(goal[0 * 3 + r], pe[0] - goal[9],
                                             fmaf(goal[1 * 3 + r], pe[1] - goal[10], goal[2 * 3 + r] * (pe[2] - goal[11])));
                pos2 = fmaf(e[r], e[r], pos2);
            }
            const float pos = fast_sqrt(pos2);
            const float kp = pos > 0.0f ? P.w_pos / pos : 0.0f;
            float gp[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                gp[a] = kp * fmaf(goal[a * 3 + 0], P.alpha_pos[0] * e[0],
                                  fmaf(goal[a * 3 + 1], P.alpha_pos[1] * e[1], goal[a * 3 + 2] * P.alpha_pos[2] * e[2]));
            // rotation: M = diag(a1)(I - R_g^T R), gradient G = -w_rot R_g diag(a1) M / |M|_F
            float M[9], rot2 = 0.0f;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float m = fmaf(goal[0 * 3 + r], Re[0 * 3 + c],
                                         fmaf(goal[1 * 3 + r], Re[1 * 3 + c], goal[2 * 3 + r] * Re[2 * 3 + c]));
                    M[r * 3 + c] = P.alpha_rot[r] * ((r == c ? 1.0f : 0.0f) - m);
                    rot2 = fmaf(M[r * 3 + c], M[r * 3 + c], rot2);
                }
            const float rot = fast_sqrt(rot2);
            const float kr = rot > 0.0f ? -P.w_rot / rot : 0.0f;
            float G[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    G[a * 3 + c] = kr * fmaf(goal[a * 3 + 0], P.alpha_rot[0] * M[0 * 3 + c],
                                             fmaf(goal[a * 3 + 1], P.alpha_rot[1] * M[1 * 3 + c],
                                                  goal[a * 3 + 2] * P.alpha_rot[2] * M[2 * 3 + c]));
            // <G, [z]x R> = z . w with A = R G^T, w = (A12 - A21, A20 - A02, A01 - A10)
            float A[9];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    A[a * 3 + b] = fmaf(Re[a * 3 + 0], G[b * 3 + 0], fmaf(Re[a * 3 + 1], G[b * 3 + 1], Re[a * 3 + 2] * G[b * 3 + 2]));
            const float w0 = A[1 * 3 + 2] - A[2 * 3 + 1];
            const float w1 = A[2 * 3 + 0] - A[0 * 3 + 2];
            const float w2 = A[0 * 3 + 1] - A[1 * 3 + 0];
#pragma unroll
            for (int k = 0; k < kDof; ++k) {
                const float z0 = s_fr[k * 12 + 2][lane], z1 = s_fr[k * 12 + 5][lane], z2 = s_fr[k * 12 + 8][lane];
                const float r0 = pe[0] - s_fr[k * 12 + 9][lane];
                const float r1 = pe[1] - s_fr[k * 12 + 10][lane];
                const float r2 = pe[2] - s_fr[k * 12 + 11][lane];
                // (p - o_k) x g_p
                const float c0 = r1 * gp[2] - r2 * gp[1];
                const float c1 = r2 * gp[0] - r0 * gp[2];
                const float c2 = r0 * gp[1] - r1 * gp[0];
                gq[k] += fmaf(z0, c0 + w0, fmaf(z1, c1 + w1, z2 * (c2 + w2)));
            }
            cost = fmaf(P.w_pos, pos, fmaf(P.w_rot, rot, cost));
        }
#pragma unroll
        for (int k = 0; k < kDof; ++k) s_gq[k][lane] = hw_h * gq[k];
        const float Ci = segmented_scan(hw_h * cost, h, H);
        if (h == H - 1) s_Cp[pl] = valid ? Ci : 0.0f;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int p = 0; p < P.ppt; ++p) cacc += s_Cp[p];

    // ---- D: the integrator backwards -----------------------------------------
    if (wave < kDof) {
        const int j = wave;
        const float Gv = fmaf(dt_h, segmented_suffix_scan(s_gq[j][lane], h, H), hw_h * s_gv[j][lane]);
        const float gu = dt_h * segmented_suffix_scan(Gv, h, H);
        s_gu[j][lane] = live ? gu : 0.0f;
    }
    __syncthreads();

    // ---- E: the tile's partial of dJ/dmu (sum over the tile's particles) -----
    if ((int)threadIdx.x < kDof * H) {
        const int j = threadIdx.x / H, hh = threadIdx.x - j * H;
        for (int p = 0; p < P.ppt; ++p) acc += s_gu[j][p * H + hh];
    }
    __syncthreads();  // LDS is reused by the next tile of the chunk
}

// Chunks of tiles of one problem: min(n_tiles, kAdjChunks), chunk c covering
// tiles [c T / n, (c + 1) T / n); one workgroup per chunk, tiles in order.
__device__ __forceinline__ int adj_chunks(const ProblemDev &P) { return min(P.n_tiles, kAdjChunks); }

__device__ __forceinline__ void adjoint_chunk(const ProblemDev &P, const RobotDev &R, const int c,
                                              const float *__restrict__ x0, const float *__restrict__ goal,
                                              const float *__restrict__ mean, const float *__restrict__ noise)
{
    const int n = adj_chunks(P), T = P.n_tiles;
    const int t0 = (int)((long long)c * T / n), t1 = (int)((long long)(c + 1) * T / n);
    float acc = 0.0f, cacc = 0.0f;
    for (int tile = t0; tile < t1; ++tile) adjoint_tile(P, R, tile, x0, goal, mean, noise, acc, cacc);
    if ((int)threadIdx.x < kDof * P.H) {
        const int j = threadIdx.x / P.H, hh = threadIdx.x - j * P.H;
        P.grad_part[((size_t)c * kDof + j) * kMaxH + hh] = acc;
    }
    if (threadIdx.x == 0) P.cost_part[c] = cacc;
}

// The fields the first loads of a tile depend on come first, as scalar
// arguments, so that they are preloaded into SGPRs; the rest of the problem
// follows in P.
__global__ __launch_bounds__(kAdjWaves *kLanes) void adjoint_kernel(const float *__restrict__ mean, uint32_t *last_step,
                                                                    float *sigma2, const float *halton,
                                                                    const float *tables, int32_t N, int32_t H,
                                                                    int32_t ppt, ProblemDev P, RobotDev R,
                                                                    const float *__restrict__ x0,
                                                                    const float *__restrict__ goal,
                                                                    const float *__restrict__ noise)
{
    ProblemDev Q = P;
    Q.last_step = last_step;
    Q.sigma2 = sigma2;
    Q.halton = halton;
    Q.tables = tables;
    Q.N = N;
    Q.H = H;
    Q.ppt = ppt;
    adjoint_chunk(Q, R, blockIdx.x, x0, goal, mean, noise);
}

// Batched form: workgroup k takes chunk items[k] = (problem, chunk).  At
// most 80 VGPRs (six waves per SIMD), so that three workgroups share a CU
// (3 x 41.5 KB of LDS): the third one's serial phases fill the others'
// stalls (large workload: 2.2 -> 1.65 ms per launch; 88 VGPRs unbounded).
__global__ __launch_bounds__(kAdjWaves *kLanes) __attribute__((amdgpu_waves_per_eu(6))) void adjoint_batch_kernel(const ProblemDev *__restrict__ probs,
                                                                          const int2 *__restrict__ items,
                                                                          RobotDev R, const float *__restrict__ x0s,
                                                                          const float *__restrict__ goals)
{
    const STORM_CONST_AS int32_t *it = uniform_ptr(reinterpret_cast<const int32_t *>(items));
    const int p = it[2 * blockIdx.x], c = it[2 * blockIdx.x + 1];
    const ProblemDev P = load_uniform(probs + p);
    adjoint_chunk(P, R, c, x0s + (size_t)p * 3 * kDof, goals + (size_t)p * 12, P.mean, nullptr);
}

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kLanes);
    return x;
}

// grad[h][j] = (1/N) sum over chunks of the partials, J = (1/N) sum of the
// chunk cost sums; rows of threads take chunks r, r + R, ..., then the rows
// are added in order.
// One Adam step with gradient g on the stored mean, element t (moments
// restart at it == 1).
__device__ __forceinline__ void adam_step(const ProblemDev &P, int t, float g, int it, float lr, float b1, float b2,
                                          float eps)
{
    const float m0 = it == 1 ? 0.0f : P.adam_m[t];
    const float v0 = it == 1 ? 0.0f : P.adam_v[t];
    const float m = fmaf(b1, m0, (1.0f - b1) * g);
    const float v = fmaf(b2, v0, (1.0f - b2) * g * g);
    P.adam_m[t] = m;
    P.adam_v[t] = v;
    const float mh = m / (1.0f - powf(b1, (float)it));
    const float vh = v / (1.0f - powf(b2, (float)it));
    P.mean[t] -= lr * mh / (sqrtf(vh) + eps);
}

// cmd = mu_0, then the warm-start shift of the stored mean (and of a
// per-step variance, sigma_init^2 appended) if requested.
__device__ __forceinline__ void command(const ProblemDev &P, float *__restrict__ cmd, int shift)
{
    __shared__ float s_mu[kDof * kMaxH];
    __shared__ float s_s2[kDof * kMaxH];
    const int t = threadIdx.x;
    const int n = P.H * kDof;
    for (int k = t; k < n; k += blockDim.x) {
        s_mu[k] = P.mean[k];
        if (P.cov_step) s_s2[k] = P.sigma2[k];
    }
    __syncthreads();
    if (t < kDof) cmd[t] = s_mu[t];
    if (shift)
        for (int k = t; k < n; k += blockDim.x) {
            P.mean[k] = k + kDof < n ? s_mu[k + kDof] : 0.0f;
            if (P.cov_step) P.sigma2[k] = k + kDof < n ? s_s2[k + kDof] : P.tables[kTabSig0 + k % kDof];
        }
}

// Gradient of joint j: the chunk partials of (h, j) summed in a fixed order
// (thread (r, h) over chunks r, r + rows, ..., every load in flight at once,
// then wave 0 over the rows), divided by N; joint 0 also sums the chunk
// costs into J.  With it > 0, lane h of wave 0 then takes the Adam step on
// mu[h][j]; with cmd, it writes the command mu[0][j] and the warm-start
// shift of the joint (the next step's value through a DPP wave shift), with
// a per-step variance shifted alike.
__device__ __forceinline__ void grad_step(const ProblemDev &P, int j, float *__restrict__ grad_out,
                                          float *__restrict__ J_out, int it, float lr, float *__restrict__ cmd,
                                          int shift)
{
    constexpr int kMaxPerThread = (kAdjChunks * kMaxH + kRedThreads - 1) / kRedThreads;
    __shared__ float s_red[kRedThreads];
    __shared__ float s_wave[kRedThreads / kLanes];
    const int t = threadIdx.x;
    const int lane = t & (kLanes - 1), wave = t / kLanes;
    const int H = P.H, T = min(P.n_tiles, kAdjChunks);
    const int rows = kRedThreads / H;
    const int r = t / H, h = t - r * H;
    float acc = 0.0f;
    if (r < rows) {
        const float *__restrict__ src = P.grad_part + (size_t)j * kMaxH + h;
        float v[kMaxPerThread];
#pragma unroll
        for (int i = 0; i < kMaxPerThread; ++i) {
            const int k = r + i * rows;
            v[i] = k < T ? src[(size_t)k * kDof * kMaxH] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < kMaxPerThread; ++i) acc += v[i];
    }
    s_red[t] = acc;
    if (j == 0) {
        float cs = 0.0f;
        for (int k = t; k < T; k += kRedThreads) cs += P.cost_part[k];
        cs = wave_sum(cs);
        if (lane == 0) s_wave[wave] = cs;
    }
    __syncthreads();
    if (wave != 0) return;
    const float invN = 1.0f / (float)P.N;
    if (j == 0 && lane == 0 && J_out) {
        float J = 0.0f;
        for (int k = 0; k < kRedThreads / kLanes; ++k) J += s_wave[k];
        *J_out = J * invN;
    }
    float mu = 0.0f;
    if (lane < H) {
        float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        int k = 0;
        for (; k + 3 < rows; k += 4)
#pragma unroll
            for (int m = 0; m < 4; ++m) p4[m] += s_red[(k + m) * H + lane];
#pragma unroll
        for (int m = 0; m < 3; ++m)
            if (k + m < rows) p4[m] += s_red[(k + m) * H + lane];
        const float g = ((p4[0] + p4[1]) + (p4[2] + p4[3])) * invN;
        const int e = lane * kDof + j;
        P.grad[e] = g;
        if (grad_out) grad_out[e] = g;
        if (it > 0) adam_step(P, e, g, it, lr, 0.9f, 0.999f, 1e-8f);
        if (cmd) mu = P.mean[e];
    }
    if (cmd) {
        const float mu_next = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(mu), 0x130, 0xf, 0xf,
                                                                         true));  // wave_shl:1
        if (lane == 0) cmd[j] = mu;
        if (shift && lane < H) P.mean[lane * kDof + j] = lane + 1 < H ? mu_next : 0.0f;
        if (shift && P.cov_step) {
            // a per-step variance moves forward too, sigma_init^2 appended
            const float s2 = lane < H ? P.sigma2[lane * kDof + j] : 0.0f;
            const float s2_next = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s2), 0x130, 0xf, 0xf,
                                                                             true));  // wave_shl:1
            if (lane < H) P.sigma2[lane * kDof + j] = lane + 1 < H ? s2_next : P.tables[kTabSig0 + j];
        }
    }
}

__global__ __launch_bounds__(kRedThreads) void grad_step_kernel(ProblemDev P, float *__restrict__ grad_out,
                                                                float *__restrict__ J_out, int it, float lr,
                                                                float *__restrict__ cmd, int shift)
{
    grad_step(P, blockIdx.x, grad_out, J_out, it, lr, cmd, shift);
}

__global__ void command_kernel(ProblemDev P, float *__restrict__ cmd, int shift) { command(P, cmd, shift); }

// Batched forms: workgroup p * 7 + j serves joint j of problem p.
__global__ __launch_bounds__(kRedThreads) void grad_step_batch_kernel(const ProblemDev *__restrict__ probs, int it,
                                                                      float lr, float *__restrict__ cmd, int shift)
{
    const int p = blockIdx.x / kDof, j = blockIdx.x - p * kDof;
    const ProblemDev P = load_uniform(probs + p);
    grad_step(P, j, nullptr, nullptr, it, lr, cmd ? cmd + (size_t)p * kDof : nullptr, shift);
}

__global__ void command_batch_kernel(const ProblemDev *__restrict__ probs, float *__restrict__ cmd, int shift)
{
    const ProblemDev P = load_uniform(probs + blockIdx.x);
    command(P, cmd + (size_t)blockIdx.x * kDof, shift);
}

}  // namespace

hipError_t launch_grad(const ProblemDev &P, const RobotDev &R, const float *x0, const float *goal, const float *mean,
                       const float *noise, float *grad_out, float *J_out, int it, float lr, float *cmd, int shift,
                       hipStream_t stream)
{
    const int chunks = P.n_tiles < kAdjChunks ? P.n_tiles : kAdjChunks;
    hipLaunchKernelGGL(adjoint_kernel, dim3((unsigned)chunks), dim3(kAdjWaves * kLanes), 0, stream, mean, P.last_step,
                       P.sigma2, P.halton, P.tables, P.N, P.H, P.ppt, P, R, x0, goal, noise);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_step_kernel, dim3(kDof), dim3(kRedThreads), 0, stream, P, grad_out, J_out, it, lr, cmd,
                       shift);
    return hipGetLastError();
}

hipError_t launch_command(const ProblemDev &P, float *cmd, int shift, hipStream_t stream)
{
    hipLaunchKernelGGL(command_kernel, dim3(1), dim3(256), 0, stream, P, cmd, shift);
    return hipGetLastError();
}

hipError_t launch_refine_batch(const ProblemDev *probs, int n_problems, const int2 *items, int n_items,
                               const RobotDev &R, const float *x0s, const float *goals, int iterations, float lr,
                               float *cmd, int shift, hipStream_t stream)
{
    hipError_t e = hipSuccess;
    for (int it = 1; e == hipSuccess && it <= iterations; ++it) {
        hipLaunchKernelGGL(adjoint_batch_kernel, dim3((unsigned)n_items), dim3(kAdjWaves * kLanes), 0, stream,
                           probs, items, R, x0s, goals);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(grad_step_batch_kernel, dim3((unsigned)(n_problems * kDof)), dim3(kRedThreads), 0, stream,
                           probs, it, lr, it == iterations ? cmd : nullptr, shift);
        e = hipGetLastError();
    }
    if (e == hipSuccess && iterations == 0) {
        hipLaunchKernelGGL(command_batch_kernel, dim3((unsigned)n_problems), dim3(256), 0, stream, probs, cmd, shift);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace storm
