// Kernel R: sample -> integrate -> kinematics -> running cost -> horizon cost
// for one MPC problem (STORM, Sec. 3.1-3.3, Eq. 2 and 7-15).
//
// Work decomposition.  A tile is one 64-lane point set holding
// ppt = floor(64 / H) whole particles, lane = particle_in_tile * H + step.
// One workgroup of W wavefronts owns one tile; the waves split the work of
// the tile's 64 (particle, step) points and exchange data through LDS:
//   A0  waves 0-3  standard noise: one Philox4x32-10 call gives four normals
//                  (joints 4k..4k+3), each wave the Box-Muller pair of one
//                  half of a call; or the Halton table; or the override
//   A1  waves 0-6  one joint each: u = mu + sigma eps, then the two
//                  segmented prefix sums of the triple integrator (Eq. 7) as
//                  wavefront DPP scans over the particle's lanes, the joint's
//                  sine and cosine, and its squared joint, velocity and stop
//                  hinges (Eq. 10-11)
//   B   waves 0-2  forward kinematics (Eq. 8), one row of the eight frames
//                  per wave, to LDS
//       wave W-1   the hinge norms over the joints (Eq. 10-11)
//   C   waves 0..W-3  world centres of the body spheres to LDS
//       wave W-2   manipulability (Eq. 12)
//       wave W-1   pose (Eq. 9)
//   D   all waves  environment (spheres x obstacles) split over waves, then
//                  self-collision (sphere pairs) as items taken from a queue,
//                  each behind a broad-phase test
//   E   wave 0     weighted running cost (Eq. 15), horizon sum (Eq. 2) as a
//                  segmented DPP scan
// Obstacle, sphere and pair records are indexed by wave-uniform loop
// counters, so they are fetched with scalar loads into SGPRs; every per-point
// LDS array is [row][lane] (conflict-free), and rows whose lifetimes do not
// overlap share space (about 80 KB per workgroup with 52 spheres, so that the
// batched form holds two workgroups per CU).  Reductions run in a fixed
// order: results are bitwise reproducible.
#include <algorithm>

#include "kinematics.h"
#include "sampling.h"

namespace storm {
namespace {

// Rows of the sphere-centre block, which also holds the noise, sine/cosine
// and hinge rows of phases A0-B (8 + 14 + 21) before the centres exist.
__host__ __device__ constexpr int rollout_cen_rows(int S) { return 3 * S > 43 ? 3 * S : 43; }
static_assert(2 * 16 <= 96, "the collision partials of 16 waves fit over the frame rows");

// Wavefront-wide maximum of a non-negative float: IEEE bit patterns of
// non-negative floats order like unsigned integers, so the maximum runs on
// the bits through DPP lane moves (quad permutes, half-row and row mirrors,
// then the row broadcasts that carry each row's result into the next) and is
// read back from lane 63, the lane every step feeds, into an SGPR.
__device__ __forceinline__ float wave_max_nonneg(float x)
{
    uint32_t b = __float_as_uint(x);
    b = max(b, (uint32_t)__builtin_amdgcn_mov_dpp((int)b, 0xb1, 0xf, 0xf, false));   // quad_perm [1, 0, 3, 2]
    b = max(b, (uint32_t)__builtin_amdgcn_mov_dpp((int)b, 0x4e, 0xf, 0xf, false));   // quad_perm [2, 3, 0, 1]
    b = max(b, (uint32_t)__builtin_amdgcn_mov_dpp((int)b, 0x141, 0xf, 0xf, false));  // row_half_mirror
    b = max(b, (uint32_t)__builtin_amdgcn_mov_dpp((int)b, 0x140, 0xf, 0xf, false));  // row_mirror
    b = max(b, (uint32_t)__builtin_amdgcn_mov_dpp((int)b, 0x142, 0xa, 0xf, false));  // row_bcast:15, rows 1 and 3
    b = max(b, (uint32_t)__builtin_amdgcn_mov_dpp((int)b, 0x143, 0xc, 0xf, false));  // row_bcast:31, rows 2 and 3
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)b, 63));
}

// Candidates of one 64-obstacle chunk above which the environment broad phase
// refines the wave's ball into eight balls of eight lanes (measured: the
// refinement pays for itself from about this many candidates on).
constexpr int kFineCandidates = 8;

// LDS copy of the goal (R row-major, p) and the cost weights, by index.
constexpr int kParArot = 12, kParApos = 15, kParW = 18, kParKm = 25, kParCount = 26;

// Lane 0's value, as a wave-uniform (SGPR) float.
__device__ __forceinline__ float uniform_lane0(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Culling record o, or one that no test can pass for o beyond the scene.
__device__ __forceinline__ float4 load_bound(const float4 *__restrict__ b, int o, int n)
{
    return o < n ? b[o] : make_float4(3.0e38f, 3.0e38f, 3.0e38f, 0.0f);
}

// The ball-on-tray term (appendix on dynamic object balancing), by the pose
// wave: every lane forms the flange frame of the current state q0 and moves
// the ball's world state into it (its z velocity dropped); lane (particle,
// h) takes the in-plane gravity in the flange frame of its rolled-out state
// and the two segmented scans of Eq. 7's scheme give the ball's velocity
// and position; the term is the distance from the tray centre.
__device__ __forceinline__ void ball_term(const ProblemDev &P, const RobotDev &R, const float *__restrict__ x0,
                                          const float *s_fr, float *s_terms, const int lane, const int h,
                                          const int H, const float *__restrict__ tab)
{
    float r0[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f}, p0[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int f = 0; f < kFrames; ++f) {
        float st = 0.0f, ct = 1.0f;
        if (f < kDof) sincosf(x0[f], &st, &ct);
        dh_step(r0, p0, R.ca[f], R.sa[f], R.a[f], R.d[f], ct, st);
    }
    const float bw[3] = {P.ball[0] - p0[0], P.ball[1] - p0[1], P.ball[2] - p0[2]};
    float xb[2], vb[2], ab[2];
    const float *E = s_fr + 7 * 12 * kLanes + lane;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        xb[c] = fmaf(r0[c], bw[0], fmaf(r0[3 + c], bw[1], r0[6 + c] * bw[2]));
        vb[c] = fmaf(r0[c], P.ball[3], fmaf(r0[3 + c], P.ball[4], r0[6 + c] * P.ball[5]));
        ab[c] = fmaf(E[c * kLanes], P.ball_g[0], fmaf(E[(3 + c) * kLanes], P.ball_g[1],
                                                      E[(6 + c) * kLanes] * P.ball_g[2]));
    }
    const float dt_h = tab[kTabDt + h];
    float d2 = 0.0f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const float v = vb[c] + segmented_scan(dt_h * ab[c], h, H);
        const float x = xb[c] + segmented_scan(dt_h * v, h, H);
        const float e = x - P.ball_c[c];
        d2 = fmaf(e, e, d2);
    }
    s_terms[8 * kLanes + lane] = fast_sqrt(d2);
}

// One 64-lane tile of one problem, executed by the W waves of the calling
// workgroup; smem is the workgroup's dynamic LDS (rollout_lds_bytes).
// kTask: the task-space form, which adds the flange velocity and
// acceleration outputs (Eq. 8), the ball-on-tray term and the joint
// positions the learned self-collision network reads.
template <int W, bool kTask = false>
__device__ __forceinline__ void rollout_tile(const ProblemDev &P, const RobotDev &R, const int tile,
                                             const float *__restrict__ x0, const float *__restrict__ goal,
                                             const float *__restrict__ noise, const StepOut &out, float *smem)
{
    // LDS rows of 64 floats, overlaid where their lifetimes do not meet
    // (rollout_lds_bytes), so that two workgroups of the batched form fit on
    // one CU:
    //   frames [96]              B - C,  then the collision partials [2W]  D - E
    //   terms [kTerms]           B - E
    //   |c|^2 [S], centres [3S]  C - D;  before them noise [8] A0 - A1,
    //                            sin/cos [14] and hinges [21] A1 - B
    //   velocities, accelerations [14]  A1 - C (task-space form only)
    const int S = R.n_spheres;
    float *s_fr = smem;                        // [8 frames][12][64]: R row-major, p
    float *s_penv = s_fr;                      // [W][64] (over the frames, after phase C)
    float *s_pself = s_penv + W * kLanes;      // [W][64]
    float *s_terms = s_fr + 96 * kLanes;       // [kTerms][64]
    float *s_cn = s_terms + kTerms * kLanes;   // [S][64]: |c|^2 of the sphere centres
    float *s_cen = s_cn + S * kLanes;          // [S][3][64]
    float *s_eps = s_cen;                      // [8][64] (before the centres)
    float *s_sc = s_eps + 8 * kLanes;          // [7][2][64]: sin q_j, cos q_j
    float *s_lim = s_sc + 14 * kLanes;         // [3][7][64]: squared joint, velocity, stop hinges per joint
    float *s_v = s_cen + rollout_cen_rows(S) * kLanes;  // [7][64] (task-space form only)
    float *s_acc = s_v + kDof * kLanes;                  // [7][64]

    const int lane = threadIdx.x & (kLanes - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int N = P.N, H = P.H;
    const int pl = lane / H;
    const int h = lane - pl * H;
    const int i = tile * P.ppt + pl;
    const bool valid = pl < P.ppt && i < N;
    const bool live = valid && i < N - P.n_null;  // sampled (non-null) particle
    const uint32_t mask = P.cost_mask;
    const float *__restrict__ tab = P.tables;

    // Per-joint inputs of phase A1, loaded up front so that their latency
    // overlaps the noise generation.
    const int jw = wave < kDof ? wave : 0;
    // (vector loads throughout, so that the first barrier waits for none of
    // them: the state and the policy come fresh from the previous kernels)
    const float mu_j = live ? P.mean[h * kDof + jw] : 0.0f;
    const float sig_j = sqrtf(P.cov_step ? P.sigma2[h * kDof + jw] : vector_load_f32(P.sigma2 + jw));
    const float dt_h = tab[kTabDt + h];
    const float vs_h = tab[kTabVstop + h];
    const float q0_j = vector_load_f32(x0 + jw), v0_j = vector_load_f32(x0 + kDof + jw);
    // culling record of obstacle `lane` (first 64 obstacles) for phase D
    const float4 bound0 = (mask & STORM_COST_ENV) ? load_bound(P.obs_bound, lane, P.n_sph_obs + P.n_box_obs)
                                                  : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // the goal and the cost weights that phases C and E read, staged in
    // LDS by the last wave while the noise is drawn (read where they are
    // used, as scalar loads, they would add a memory round trip to those
    // serial phases)
    __shared__ float s_par[kParCount];
    __shared__ int s_self_next;  // head of the self-collision item queue (phase D)
    if (wave == W - 1 && lane == kParCount) s_self_next = 0;
    if (wave == W - 1 && lane < kParCount) {
        const float wts[kParCount - 12] = {P.alpha_rot[0], P.alpha_rot[1], P.alpha_rot[2], P.alpha_pos[0],
                                           P.alpha_pos[1], P.alpha_pos[2], P.w_pos,        P.w_rot,
                                           P.a_joint,      P.a_vel,        P.a_stop,       P.a_manip,
                                           P.a_coll,       P.k_m};
        float v = 0.0f;
#pragma unroll
        for (int k = 0; k < kParCount - 12; ++k) v = lane == 12 + k ? wts[k] : v;
        const float g = goal[lane < 12 ? lane : 0];
        s_par[lane] = lane < 12 ? g : v;
    }

    // ---- A0: standard noise ------------------------------------------------
    // waves 0-3, one per SIMD: wave w makes the normal pair w / 2 of Philox
    // call w % 2, i.e. joints 4 (w % 2) + 2 (w / 2) and the next (the
    // Philox call is repeated by the two waves that share it; its Box-Muller
    // half is not)
    if (wave < 4) {
        const int k = wave & 1, half = wave >> 1;
        const int j0 = 4 * k + 2 * half;
        float e[2] = {0.0f, 0.0f};
        const uint32_t counter = *P.step;
        if (live) standard_noise2(P, noise, k, half, i, h, counter, e);
        s_eps[j0 * kLanes + lane] = e[0];
        s_eps[(j0 + 1) * kLanes + lane] = e[1];
        if (tile == 0 && threadIdx.x == 0) *P.last_step = counter;
    }
    __syncthreads();

    // ---- A1: controls and the triple integrator (Eq. 7) ---------------------
    if (wave < kDof) {
        const int j = wave;
        float e = s_eps[j * kLanes + lane];
        // the comb filter on the sampled Gaussian particles' noise (Sec. 3.3)
        const bool comb = P.comb && noise == nullptr && live && i >= P.n_halton;
        if (__builtin_amdgcn_ballot_w64(comb) != 0) {
            const float f = comb_noise(s_eps + j * kLanes, lane, h, H, tab);
            if (comb) e = f;
        }
        float u = 0.0f;
        if (live) u = fmaf(sig_j, e, mu_j);
        const float v = v0_j + segmented_scan(dt_h * u, h, H);
        const float q = q0_j + segmented_scan(dt_h * v, h, H);
        if (kTask) s_v[j * kLanes + lane] = v;
        // this joint's squared joint, velocity and stop hinges (Eq. 10-11),
        // summed over the joints in phase C
        const float hj = hinge_box(q, tab[kTabJlo + j], tab[kTabJhi + j]);
        const float hv = hinge_box(v, tab[kTabVlo + j], tab[kTabVhi + j]);
        const float hs = fmaxf(fabsf(v) - vs_h, 0.0f);
        s_lim[(0 * kDof + j) * kLanes + lane] = hj * hj;
        s_lim[(1 * kDof + j) * kLanes + lane] = hv * hv;
        s_lim[(2 * kDof + j) * kLanes + lane] = hs * hs;
        float sq, cq;
        sincosf(q, &sq, &cq);
        s_sc[(2 * j) * kLanes + lane] = sq;
        s_sc[(2 * j + 1) * kLanes + lane] = cq;
        if (kTask) s_acc[j * kLanes + lane] = u;
        if (valid) {
            const size_t o = ((size_t)j * N + i) * H + h;
            P.u[o] = u;
            if (kTask && P.qbuf != nullptr) P.qbuf[o] = q;
            if (out.u) out.u[o] = u;
            if (out.q) out.q[o] = q;
            if (out.v) out.v[o] = v;
            if (out.a) out.a[o] = u;
        }
    }
    __syncthreads();

    // ---- B: forward kinematics, one row of the frames per wave ----------------
    if (wave < 3) {
        const int row = wave;
        float r[3] = {row == 0 ? 1.0f : 0.0f, row == 1 ? 1.0f : 0.0f, row == 2 ? 1.0f : 0.0f};
        float p = 0.0f;
#pragma unroll
        for (int f = 0; f < kFrames; ++f) {
            float st = 0.0f, ct = 1.0f;
            if (f < kDof) {
                st = s_sc[(2 * f) * kLanes + lane];
                ct = s_sc[(2 * f + 1) * kLanes + lane];
            }
            dh_step_row(r, p, R.ca[f], R.sa[f], R.a[f], R.d[f], ct, st);
#pragma unroll
            for (int c = 0; c < 3; ++c) s_fr[(f * 12 + row * 3 + c) * kLanes + lane] = r[c];
            s_fr[(f * 12 + 9 + row) * kLanes + lane] = p;
        }
    } else if (wave == W - 1) {
        // Eq. 10-11: norms over the joints of the hinges formed in phase A1
        // (here, so that the hinge rows are free for the centres of phase C)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < kDof; ++j) acc += s_lim[(k * kDof + j) * kLanes + lane];
            s_terms[(2 + k) * kLanes + lane] = fast_sqrt(acc);
        }
    }
    __syncthreads();

    // ---- C: world centres of the body spheres | pose | manipulability --------
    // The last two waves evaluate the pose (Eq. 9) and manipulability
    // (Eq. 12) terms from the frames while the others place the spheres, so
    // that the collision phase is spread evenly over all waves.
    constexpr int WC = W - kPoseWaves;
    if (wave < WC) {
        if (mask & (STORM_COST_SELF | STORM_COST_ENV)) {
            // a contiguous run of spheres per wave (sorted by body): the
            // frame of a body is read from LDS once per run
            const int s0 = wave * S / WC, s1 = (wave + 1) * S / WC;
            const STORM_CONST_AS int32_t *body = uniform_ptr(R.sph_body);
            int fb = -1;
            float F[12];
            for (int s = s0; s < s1; ++s) {
                const STORM_CONST_AS float *sl = uniform_ptr(reinterpret_cast<const float *>(R.sph_local)) + 4 * s;
                const int b = body[s];
                if (b != fb) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) F[c] = s_fr[(b * 12 + c) * kLanes + lane];
                    fb = b;
                }
                float cc[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    cc[c] = fmaf(F[c * 3 + 0], sl[0], fmaf(F[c * 3 + 1], sl[1], fmaf(F[c * 3 + 2], sl[2], F[9 + c])));
                    s_cen[(s * 3 + c) * kLanes + lane] = cc[c];
                }
                s_cn[s * kLanes + lane] = fmaf(cc[0], cc[0], fmaf(cc[1], cc[1], cc[2] * cc[2]));
            }
        }
    } else if (wave == W - 1) {
        if (mask & STORM_COST_POSE) {
            // Eq. 9: rotation error |diag(alpha_rot)(I - R_g^T R)|_F and position
            // error |diag(alpha_pos) R_g^T (p - p_g)|.
            const float *E = s_fr + 7 * 12 * kLanes + lane;
            float Re[9], pe[3];
#pragma unroll
            for (int c = 0; c < 9; ++c) Re[c] = E[c * kLanes];
#pragma unroll
            for (int c = 0; c < 3; ++c) pe[c] = E[(9 + c) * kLanes];
            float rot2 = 0.0f, pos2 = 0.0f;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float m = fmaf(s_par[0 * 3 + r], Re[0 * 3 + c],
                                         fmaf(s_par[1 * 3 + r], Re[1 * 3 + c], s_par[2 * 3 + r] * Re[2 * 3 + c]));
                    const float e = s_par[kParArot + r] * ((r == c ? 1.0f : 0.0f) - m);
                    rot2 = fmaf(e, e, rot2);
                }
                const float l = fmaf(s_par[0 * 3 + r], pe[0] - s_par[9],
                                     fmaf(s_par[1 * 3 + r], pe[1] - s_par[10], s_par[2 * 3 + r] * (pe[2] - s_par[11])));
                const float e = s_par[kParApos + r] * l;
                pos2 = fmaf(e, e, pos2);
            }
            s_terms[0 * kLanes + lane] = fast_sqrt(pos2);
            s_terms[1 * kLanes + lane] = fast_sqrt(rot2);
        }
        if (kTask && (mask & STORM_COST_BALL)) ball_term(P, R, x0, s_fr, s_terms, lane, h, H, tab);
    } else {
        const bool task_out = kTask && (out.xd != nullptr || out.xdd != nullptr);
        if ((mask & STORM_COST_MANIP) || task_out) {
            float z[kDof][3], o[kDof][3], pe[3];
#pragma unroll
            for (int k = 0; k < kDof; ++k) {
                const float *F = s_fr + k * 12 * kLanes + lane;
                z[k][0] = F[2 * kLanes];
                z[k][1] = F[5 * kLanes];
                z[k][2] = F[8 * kLanes];
                o[k][0] = F[9 * kLanes];
                o[k][1] = F[10 * kLanes];
                o[k][2] = F[11 * kLanes];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) pe[c] = s_fr[(7 * 12 + 9 + c) * kLanes + lane];
            if (mask & STORM_COST_MANIP) s_terms[5 * kLanes + lane] = manipulability(z, o, pe);
            if (task_out) {
                float qd[kDof], qdd[kDof], xd[6], xdd[6];
#pragma unroll
                for (int k = 0; k < kDof; ++k) {
                    qd[k] = s_v[k * kLanes + lane];
                    qdd[k] = s_acc[k * kLanes + lane];
                }
                task_space(s_fr + lane, kLanes, qd, qdd, xd, xdd);
                if (valid)
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        const size_t at = ((size_t)c * N + i) * H + h;
                        if (out.xd) out.xd[at] = xd[c];
                        if (out.xdd) out.xdd[at] = xdd[c];
                    }
            }
        }
    }
    __syncthreads();

    // ---- D: collision terms ---------------------------------------------------
    // Environment (spheres round robin over the waves), then self-collision
    // (items from a queue).  Both cull first at the level of the whole wave
    // and take exact distances (and their square roots) only where some lane
    // of the wave may touch; a culled record touches at no lane, so the
    // terms equal the brute-force ones.
    float env = 0.0f, selfpen = 0.0f;
    if (mask & STORM_COST_ENV) {
        const STORM_CONST_AS float *sob = uniform_ptr(reinterpret_cast<const float *>(P.sph_obs));
        const STORM_CONST_AS float *box = uniform_ptr(P.box_obs);
        const STORM_CONST_AS float *sloc = uniform_ptr(reinterpret_cast<const float *>(R.sph_local));
        const int nso = P.n_sph_obs, nobs = P.n_sph_obs + P.n_box_obs;
        for (int s = wave; s < S; s += W) {
            const float x = s_cen[(s * 3 + 0) * kLanes + lane];
            const float y = s_cen[(s * 3 + 1) * kLanes + lane];
            const float z = s_cen[(s * 3 + 2) * kLanes + lane];
            const float rs = sloc[4 * s + 3];
            const float rs2 = rs * rs;
            // Broad phase: the wave's 64 centres of this sphere lie in the
            // ball of radius rad about lane 0's centre; by the triangle
            // inequality an obstacle whose bounding ball is farther than
            // rad + r_s from that point touches the sphere at no lane.  One
            // lane tests one obstacle, and a ballot gives the candidates.  A
            // non-finite centre anywhere in the wave turns the culling off.
            const float rx = uniform_lane0(x), ry = uniform_lane0(y), rz = uniform_lane0(z);
            const float ax = x - rx, ay = y - ry, az = z - rz;
            const float rad = fast_sqrt(wave_max_nonneg(fminf(fmaf(ax, ax, fmaf(ay, ay, az * az)), 1.0e30f)));
            const bool cull = rad < 1.0e6f;
            const float rad_rs = rad + rs;
            float best = 0.0f;
            for (int o0 = 0; o0 < nobs; o0 += kLanes) {
                const float4 bd = o0 == 0 ? bound0 : load_bound(P.obs_bound, o0 + lane, nobs);
                const float dx = bd.x - rx, dy = bd.y - ry, dz = bd.z - rz;
                const float reach = bd.w + rad_rs;
                uint64_t cand = cull ? __builtin_amdgcn_ballot_w64(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < reach * reach)
                                     : __builtin_amdgcn_ballot_w64(o0 + lane < nobs);
                if (cull && __builtin_popcountll(cand) > kFineCandidates) {
                    // Many candidates: trajectories that sweep far over the
                    // horizon make the wave's ball large.  Eight balls of
                    // eight lanes instead (centre: the group's first lane;
                    // radius: the group's largest distance to it); an
                    // obstacle stays a candidate where it reaches one of them.
                    // The centres come through swizzles within each 32-lane
                    // half, the radii through DPP maxima within each group.
                    float gx[8], gy[8], gz[8], gr[8];
                    {
                        const float cx = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x18));
                        const float cy = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(y), 0x18));
                        const float cz = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(z), 0x18));
                        const float bx = x - cx, by = y - cy, bz = z - cz;
                        uint32_t u = __float_as_uint(fmaf(bx, bx, fmaf(by, by, bz * bz)));
                        u = max(u, (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0xb1, 0xf, 0xf, false));
                        u = max(u, (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0x4e, 0xf, 0xf, false));
                        u = max(u, (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0x141, 0xf, 0xf, false));
                        const float r8 = fast_sqrt(__uint_as_float(u)) + rs;
#pragma unroll
                        for (int g = 0; g < 8; ++g) {
                            gx[g] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 8 * g));
                            gy[g] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), 8 * g));
                            gz[g] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z), 8 * g));
                            gr[g] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r8), 8 * g));
                        }
                    }
                    bool hit = false;
#pragma unroll
                    for (int g = 0; g < 8; ++g) {
                        const float ex = bd.x - gx[g], ey = bd.y - gy[g], ez = bd.z - gz[g];
                        const float rg = bd.w + gr[g];
                        hit |= fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < rg * rg;
                    }
                    cand &= __builtin_amdgcn_ballot_w64(hit);
                }
                // Narrow phase over the candidates, in increasing obstacle
                // order (the maximum does not depend on the order).
                while (cand != 0) {
                    const int o = o0 + (int)__builtin_ctzll(cand);
                    cand &= cand - 1;
                    if (o < nso) {
                        // the direct squared distance (no cancellation) against
                        // the squared contact distance, from the obstacle's own
                        // 16-byte record; where a lane touches, the penetration
                        // (r_s + r_o) - |x - c| at every lane (at or below zero
                        // where a lane does not touch)
                        const STORM_CONST_AS float *so = sob + 4 * o;
                        const float dx = x - so[0], dy = y - so[1], dz = z - so[2];
                        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const float rc = rs + so[3];
                        if (__builtin_amdgcn_ballot_w64(d2 < rc * rc) != 0) best = fmaxf(best, rc - fast_sqrt(d2));
                    } else {
                        const STORM_CONST_AS float *bb = box + (size_t)(o - nso) * 16;
                        const float lx = fmaf(bb[0], x, fmaf(bb[1], y, fmaf(bb[2], z, bb[9])));
                        const float ly = fmaf(bb[3], x, fmaf(bb[4], y, fmaf(bb[5], z, bb[10])));
                        const float lz = fmaf(bb[6], x, fmaf(bb[7], y, fmaf(bb[8], z, bb[11])));
                        // excess per axis, clamped to [0, 1 m]: one instruction
                        // with the clamp modifier; body spheres are below 1 m, so
                        // clamping cannot turn a miss into a hit and leaves every
                        // axis of a hit exact
                        const float ox = fminf(fmaxf(fabsf(lx) - bb[12], 0.0f), 1.0f);
                        const float oy = fminf(fmaxf(fabsf(ly) - bb[13], 0.0f), 1.0f);
                        const float oz = fminf(fmaxf(fabsf(lz) - bb[14], 0.0f), 1.0f);
                        const float out2 = fmaf(ox, ox, fmaf(oy, oy, oz * oz));
                        const bool hit = out2 < rs2;
                        if (__builtin_amdgcn_ballot_w64(hit) != 0) {
                            const float qin =
                                fminf(fmaxf(fabsf(lx) - bb[12], fmaxf(fabsf(ly) - bb[13], fabsf(lz) - bb[14])), 0.0f);
                            const float pen = rs - (fast_sqrt(out2) + qin);
                            if (hit) best = fmaxf(best, pen);
                        }
                    }
                }
            }
            env += best;
        }
    }
    if (mask & STORM_COST_SELF) {
        // Pairs by groups of up to four spheres t of one body, held in
        // registers as (-2 c_t, |c_t|^2), against their partners s streamed
        // from LDS, two partners per round.  Per pair, the expanded form
        // a = |c_t|^2 - 2 c_s.c_t (three FMAs) less the pair's threshold;
        // the group's minimum plus |c_s|^2 is negative at a lane where some
        // pair may touch: one compare per partner and one branch per round,
        // no per-pair lane masks.  Only a partner, and then a pair, that some
        // lane passes gets the exact penetration (r_s + r_t) - |c_s - c_t|,
        // at every lane: a lane whose pair fails the expanded test is apart
        // by more than the contact distance plus the rounding, so its
        // penetration is negative and leaves the maximum unchanged.  Unused
        // slots of a short group repeat its last sphere against a threshold
        // of -1e30, and the round after the last partner of an odd count
        // repeats that partner.
        //
        // Work comes as items (one group against the spheres of one partner
        // body) from a queue in LDS, so that waves done early with the
        // environment term take more.  Broad phase per item: one sphere of
        // each side (the anchors) with the radius about it that holds all of
        // that side's spheres; where the anchors are farther apart than the
        // two radii at every lane, no pair of the item touches and the item
        // is skipped (its penetrations are all negative: the maximum is the
        // same).
        const STORM_CONST_AS int32_t *items = uniform_ptr(R.self_items);
        const STORM_CONST_AS float *thr = uniform_ptr(R.self_thr);
        const int n_items = R.n_self_items;
        for (;;) {
            int g = 0;
            if (lane == 0) g = atomicAdd(&s_self_next, 1);
            g = __builtin_amdgcn_readfirstlane(g);
            if (g >= n_items) break;
            const STORM_CONST_AS int32_t *it = items + 8 * g;
            const int code = it[0], grp = it[1], s_begin = it[2], s_end = it[3], at = it[4], as = it[5];
            const float reach2 = __int_as_float(it[6]);
            const float ax = s_cen[(at * 3 + 0) * kLanes + lane] - s_cen[(as * 3 + 0) * kLanes + lane];
            const float ay = s_cen[(at * 3 + 1) * kLanes + lane] - s_cen[(as * 3 + 1) * kLanes + lane];
            const float az = s_cen[(at * 3 + 2) * kLanes + lane] - s_cen[(as * 3 + 2) * kLanes + lane];
            if (__builtin_amdgcn_ballot_w64(fmaf(ax, ax, fmaf(ay, ay, az * az)) < reach2) == 0) continue;
            const int t_first = code & 255, count = code >> 8;
            float mx[4], my[4], mz[4], nt[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int t = t_first + (k < count ? k : count - 1);
                mx[k] = -2.0f * s_cen[(t * 3 + 0) * kLanes + lane];
                my[k] = -2.0f * s_cen[(t * 3 + 1) * kLanes + lane];
                mz[k] = -2.0f * s_cen[(t * 3 + 2) * kLanes + lane];
                nt[k] = s_cn[t * kLanes + lane];
            }
            const STORM_CONST_AS float *tg = thr + (size_t)grp * S * 8;
            // one round: partners s0 and s1 (s1 == s0 for the last of an odd
            // count), whose records start at tp and tp + dt
            auto round = [&](const int s0, const int s1, const STORM_CONST_AS float *tp, const int dt)
                              __attribute__((always_inline)) {
                const int ps[2] = {s0, s1};
                float cx[2], cy[2], cz[2], ns[2], m[2], d[2][4];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int s = ps[u];
                    cx[u] = s_cen[(s * 3 + 0) * kLanes + lane];
                    cy[u] = s_cen[(s * 3 + 1) * kLanes + lane];
                    cz[u] = s_cen[(s * 3 + 2) * kLanes + lane];
                    ns[u] = s_cn[s * kLanes + lane];
                    const STORM_CONST_AS float *th = tp + u * dt;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        d[u][k] = fmaf(cx[u], mx[k], fmaf(cy[u], my[k], fmaf(cz[u], mz[k], nt[k]))) - th[k];
                    m[u] = fminf(fminf(d[u][0], d[u][1]), fminf(d[u][2], d[u][3])) + ns[u];
                }
                // the contact distances come with the thresholds (one scalar
                // load per round), not in the rare branch
                float rc[2][4];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int k = 0; k < 4; ++k) rc[u][k] = tp[u * dt + 4 + k];
                asm volatile("" : : "s"(rc[0][0]), "s"(rc[0][1]), "s"(rc[0][2]), "s"(rc[0][3]), "s"(rc[1][0]),
                             "s"(rc[1][1]), "s"(rc[1][2]), "s"(rc[1][3]));
                if (__builtin_expect(__builtin_amdgcn_ballot_w64(fminf(m[0], m[1]) < 0.0f) != 0, 0)) {
                    // the partners, then the pairs, that some lane passes
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        if (__builtin_amdgcn_ballot_w64(m[u] < 0.0f) == 0) continue;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (k >= count || __builtin_amdgcn_ballot_w64(d[u][k] + ns[u] < 0.0f) == 0) continue;
                            const float dx = fmaf(0.5f, mx[k], cx[u]), dy = fmaf(0.5f, my[k], cy[u]),
                                        dz = fmaf(0.5f, mz[k], cz[u]);
                            const float pen = rc[u][k] - fast_sqrt(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
                            selfpen = fmaxf(selfpen, pen);
                        }
                    }
                }
            };
            int sp = s_begin;
            const STORM_CONST_AS float *tp = tg + 8 * s_begin;
            for (; sp + 1 < s_end; sp += 2, tp += 16) round(sp, sp + 1, tp, 8);
            if (sp < s_end) round(sp, sp, tp, 0);
        }
    }
    s_penv[wave * kLanes + lane] = env;
    s_pself[wave * kLanes + lane] = selfpen;

    __syncthreads();

    // ---- E: running cost (Eq. 15) and horizon cost (Eq. 2) ------------------
    if (wave == 0) {
        float t[kTerms];
#pragma unroll
        for (int k = 0; k < kTerms; ++k) t[k] = 0.0f;
        if (mask & STORM_COST_POSE) {
            t[0] = s_terms[0 * kLanes + lane];
            t[1] = s_terms[1 * kLanes + lane];
        }
        if (mask & STORM_COST_JOINT) t[2] = s_terms[2 * kLanes + lane];
        if (mask & STORM_COST_VEL) t[3] = s_terms[3 * kLanes + lane];
        if (mask & STORM_COST_STOP) t[4] = s_terms[4 * kLanes + lane];
        if (mask & STORM_COST_MANIP) {
            const float m = s_terms[5 * kLanes + lane];
            t[5] = m < s_par[kParKm] ? 1.0f - m : 0.0f;
        }
        if (mask & STORM_COST_SELF)
            for (int w = 0; w < W; ++w) t[6] = fmaxf(t[6], s_pself[w * kLanes + lane]);
        if (mask & STORM_COST_ENV)
            for (int w = 0; w < W; ++w) t[7] += s_penv[w * kLanes + lane];
        const float *wc = s_par + kParW;  // w_pos, w_rot, a_joint, a_vel, a_stop, a_manip, a_coll
        float c = wc[0] * t[0];
        c = fmaf(wc[1], t[1], c);
        c = fmaf(wc[2], t[2], c);
        c = fmaf(wc[3], t[3], c);
        c = fmaf(wc[4], t[4], c);
        c = fmaf(wc[5], t[5], c);
        c = fmaf(wc[6], t[6] + t[7], c);
        if (kTask && (mask & STORM_COST_BALL)) {
            t[8] = s_terms[8 * kLanes + lane];
            c = fmaf(P.w_ball, t[8], c);
        }
        if (valid) {
            if (out.c) out.c[(size_t)i * H + h] = c;
            if (out.terms)
#pragma unroll
                for (int k = 0; k < kTerms; ++k) out.terms[((size_t)k * N + i) * H + h] = t[k];
        }
        // horizon cost (Eq. 2): segmented inclusive scan of the weighted
        // running costs; the particle's last lane holds its total
        const float C_i = segmented_scan(tab[kTabHw + h] * c, h, H);
        if (valid && h == H - 1) {
            P.C[i] = C_i;
            if (out.C) out.C[i] = C_i;
        }
    }
}

// The fields the first loads of a tile depend on come first, as scalar
// arguments, so that they are preloaded into SGPRs; the rest of the problem
// follows in P.
template <int W, bool kTask>
__global__ __launch_bounds__(W * kLanes) void rollout_kernel(uint32_t *step, float *mean, float *sigma2,
                                                             const float *halton, const float *tables, int32_t N,
                                                             int32_t H, int32_t ppt, int32_t n_halton,
                                                             int32_t n_null, uint32_t cost_mask, ProblemDev P,
                                                             RobotDev R, const float *__restrict__ x0,
                                                             const float *__restrict__ goal,
                                                             const float *__restrict__ noise, StepOut out)
{
    extern __shared__ float smem[];
    ProblemDev Q = P;
    Q.step = step;
    Q.mean = mean;
    Q.sigma2 = sigma2;
    Q.halton = halton;
    Q.tables = tables;
    Q.N = N;
    Q.H = H;
    Q.ppt = ppt;
    Q.n_halton = n_halton;
    Q.n_null = n_null;
    Q.cost_mask = cost_mask;
    rollout_tile<W, kTask>(Q, R, blockIdx.x, x0, goal, noise, out, smem);
}

// Persistent form for many problems: each workgroup takes (problem, tile)
// items from an integer work queue, in the order of `items` (the scheduler
// puts the most expensive tiles first), until the queue is empty.  Every
// workgroup draws exactly one index past the end; the one that draws the
// last of those resets the counter for the next launch.
template <int W>
__global__ __launch_bounds__(W * kLanes) void rollout_batch_kernel(const ProblemDev *__restrict__ probs,
                                                                   const int2 *__restrict__ items, int n_items,
                                                                   uint32_t *next, RobotDev R,
                                                                   const float *__restrict__ x0s,
                                                                   const float *__restrict__ goals)
{
    extern __shared__ float smem[];
    __shared__ int s_item;
    const STORM_CONST_AS int32_t *it = uniform_ptr(reinterpret_cast<const int32_t *>(items));
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= n_items) {
            if (threadIdx.x == 0 && item == n_items + (int)gridDim.x - 1) atomicExch(next, 0u);
            return;
        }
        const int p = it[2 * item], tile = it[2 * item + 1];
        const ProblemDev P = load_uniform(probs + p);
        rollout_tile<W>(P, R, tile, x0s + (size_t)p * 3 * kDof, goals + (size_t)p * 12, nullptr, StepOut{}, smem);
        __syncthreads();
    }
}

size_t rollout_lds_bytes(int S, int W, bool task = false)
{
    (void)W;  // the 2 W collision partials sit over the 96 frame rows
    return (size_t)(96 + kTerms + S + rollout_cen_rows(S) + (task ? 2 * kDof : 0)) * kLanes * sizeof(float);
}

}  // namespace

hipError_t set_rollout_lds_limit()
{
    const int bytes16 = (int)rollout_lds_bytes(STORM_MAX_SPHERES, 16);
    const int bytes8 = (int)rollout_lds_bytes(STORM_MAX_SPHERES, 8);
    const int task16 = (int)rollout_lds_bytes(STORM_MAX_SPHERES, 16, true);
    const int task8 = (int)rollout_lds_bytes(STORM_MAX_SPHERES, 8, true);
    const void *fns[6] = {reinterpret_cast<const void *>(&rollout_kernel<16, false>),
                          reinterpret_cast<const void *>(&rollout_kernel<8, false>),
                          reinterpret_cast<const void *>(&rollout_batch_kernel<16>),
                          reinterpret_cast<const void *>(&rollout_batch_kernel<8>),
                          reinterpret_cast<const void *>(&rollout_kernel<16, true>),
                          reinterpret_cast<const void *>(&rollout_kernel<8, true>)};
    const int bytes[6] = {bytes16, bytes8, bytes16, bytes8, task16, task8};
    for (int k = 0; k < 6; ++k) {
        const hipError_t e = hipFuncSetAttribute(fns[k], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[k]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_rollout_batch(const ProblemDev *probs, const int2 *items, int n_items, uint32_t *next,
                                const RobotDev &R, const float *x0s, const float *goals, int waves, int grid,
                                hipStream_t stream)
{
    const size_t lds = rollout_lds_bytes(R.n_spheres, waves);
    if (waves == 16) {
        hipLaunchKernelGGL(rollout_batch_kernel<16>, dim3((unsigned)grid), dim3(16 * kLanes), lds, stream, probs,
                           items, n_items, next, R, x0s, goals);
    } else if (waves == 8) {
        hipLaunchKernelGGL(rollout_batch_kernel<8>, dim3((unsigned)grid), dim3(8 * kLanes), lds, stream, probs,
                           items, n_items, next, R, x0s, goals);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rollout(const ProblemDev &P, const RobotDev &R, const float *x0, const float *goal,
                          const float *noise, const StepOut &out, int waves, hipStream_t stream)
{
    // the task-space form only where it is asked for: the ball term, or the
    // flange velocity and acceleration outputs
    const bool task = (P.cost_mask & STORM_COST_BALL) || P.selfnet || out.xd != nullptr || out.xdd != nullptr;
    const size_t lds = rollout_lds_bytes(R.n_spheres, waves, task);
    const dim3 grid((unsigned)P.n_tiles);
    if (waves != 16 && waves != 8) return hipErrorInvalidValue;
    auto kernel = waves == 16 ? (task ? rollout_kernel<16, true> : rollout_kernel<16, false>)
                              : (task ? rollout_kernel<8, true> : rollout_kernel<8, false>);
    hipLaunchKernelGGL(kernel, grid, dim3(waves * kLanes), lds, stream, P.step, P.mean, P.sigma2, P.halton, P.tables,
                       P.N, P.H, P.ppt, P.n_halton, P.n_null, P.cost_mask, P, R, x0, goal, noise, out);
    return hipGetLastError();
}

}  // namespace storm
