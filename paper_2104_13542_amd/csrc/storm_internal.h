// Internal definitions of the HIP library: device-side problem descriptors,
// table offsets and the kernel launchers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "storm.h"

namespace storm {

constexpr int kDof = STORM_DOF;
constexpr int kFrames = STORM_NFRAMES;
constexpr int kTerms = STORM_NTERMS;
constexpr int kLanes = 64;  // CDNA wavefront width
// waves at the end of a rollout workgroup that evaluate the pose and
// manipulability terms while the others place the body spheres
constexpr int kPoseWaves = 2;
constexpr int kMaxH = STORM_MAX_HORIZON;
constexpr int kAdjChunks = 512;  // adjoint workgroups (tile chunks) per problem, at most

// Offsets (in floats) inside the per-problem table block built at init.
constexpr int kTabDt = 0;           // dt[H]
constexpr int kTabVstop = 64;       // stop-cost velocity limit per step [H]
constexpr int kTabHw = 128;         // horizon weight gamma^h (terminal scaled) [H]
constexpr int kTabJlo = 192;        // band-shrunk joint position limits [7]
constexpr int kTabJhi = 200;
constexpr int kTabVlo = 208;        // band-shrunk joint velocity limits [7]
constexpr int kTabVhi = 216;
constexpr int kTabComb = 224;        // comb filter response g_k (e'_h = sum_k g_k e_{h-k}) [H]
constexpr int kTabSig0 = 288;        // sigma_init^2 [7], appended by a per-step covariance shift
constexpr int kTabSize = 296;

// Learned self-collision network (Eq. 13): layer widths, the packed FP16
// weight fragments (offsets in halves: per column block, k-step and lane, 4
// halves per lane for layer 1's k-steps of 16, 8 for layers 2 and 3's
// k-steps of 32) and the FP32 block of biases and output weights.
constexpr int kNetIn = 14, kNetH1 = 256, kNetH2 = 128, kNetH3 = 64;
constexpr int kNetFrag1 = 0;                                        // 16 column blocks x 1 k-step x 4
constexpr int kNetFrag2 = kNetFrag1 + (kNetH1 / 16) * 1 * 64 * 4;   // 8 x 8 x 8
constexpr int kNetFrag3 = kNetFrag2 + (kNetH2 / 16) * 8 * 64 * 8;   // 4 x 4 x 8
constexpr int kNetFragHalves = kNetFrag3 + (kNetH3 / 16) * 4 * 64 * 8;
constexpr int kNetBias1 = 0, kNetBias2 = 256, kNetBias3 = 384, kNetW4 = 448, kNetBias4 = 512;
constexpr int kNetBiasSize = 516;
static_assert(kNetH1 * kNetIn + kNetH1 + kNetH2 * kNetH1 + kNetH2 + kNetH3 * kNetH2 + 2 * kNetH3 + 1 ==
                  STORM_SELF_MLP_SIZE,
              "network parameter count");


// Per-problem description read by the kernels.  All pointers are device memory.
struct ProblemDev {
    int32_t N, H, n_halton, n_null;
    int32_t n_sph_obs, n_box_obs, ppt, n_tiles;  // ppt = particles per 64-lane tile
    uint32_t cost_mask, seed_lo, seed_hi, grad_mask;  // grad_mask: terms of the differentiable form
    float beta, alpha_mu, alpha_sigma, sigma2_min;
    float k_m, w_pos, w_rot, a_stop;
    float a_joint, a_vel, a_manip, a_coll;
    float alpha_pos[3], alpha_rot[3];
    uint32_t comb;      // the Gaussian particles' noise is comb-filtered (response in the tables)
    uint32_t cov_step;  // sigma2 is [H][7] (Eq. 5 per step) instead of [7]
    float w_ball, ball_g[3], ball_c[2];  // ball term: weight, gravity (world), tray centre (flange x, y)
    const float *tables;    // [kTabSize]
    const float *halton;    // [7][n_halton][H] smoothed Halton standard noise
    const float4 *sph_obs;  // [n_sph_obs] centre, radius
    const float *box_obs;   // [n_box_obs][16]: M = R^T (9, row-major), t = -R^T c (3), half extents (3), pad
    const float4 *obs_bound;  // [n_sph_obs + n_box_obs] centre, culling radius (bounding sphere + 1e-4 m)
    float *mean;            // [H][7]
    float *sigma2;          // [7], or [H][7] with cov_step
    float *u;               // [7][N][H] controls of the last step
    float *C;               // [N] horizon costs of the last step
    uint32_t *step;         // sampling step counter (Philox counter word 3)
    uint32_t *status;       // asynchronous status flags
    uint32_t *last_step;    // counter value the last rollout sampled with (reused by the adjoint)
    float *grad_part;       // [chunks][7][kMaxH] adjoint partial gradients per tile chunk
    float *cost_part;       // [chunks] adjoint partial horizon-cost sums per tile chunk
    float *grad;            // [H][7] gradient of the expected horizon cost
    float *adam_m, *adam_v; // [H][7] Adam moments of the refinement
    float *ball;            // [8]: ball position, velocity (world frame) at the current state, pad
    float *qbuf;            // [7][N][H] joint positions of the last step (stand-alone network pass)
    uint32_t selfnet;       // the self-collision term comes from the learned network (its own kernel)
    const _Float16 *net_frag;  // packed network weights (pack_selfnet)
    const float *net_bias;
};

// Robot constants, passed by value (kernel-argument segment, wave-uniform).
struct RobotDev {
    float ca[kFrames], sa[kFrames], a[kFrames], d[kFrames];  // DH: cos/sin alpha_{k-1}, a_{k-1}, d_k
    int32_t n_spheres, n_pairs, n_self_items, pad0;
    const float4 *sph_local;  // [S] body-frame centre (x, y, z), radius
    const int32_t *sph_body;  // [S] frame index 0..7 the sphere is attached to
    const float *self_thr;    // [groups][S][8] expanded pair test thresholds (4), contact distances (4)
    const int32_t *self_items;  // [n_self_items][8] self-collision work items (self_segments)
};

// Wave-uniform reads through the constant address space: the backend turns
// them into scalar loads whose results feed VALU instructions as SGPR operands.
#define STORM_CONST_AS __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const STORM_CONST_AS T *uniform_ptr(const T *p)
{
    return (const STORM_CONST_AS T *)(p);
}

// Copy a struct from device memory through wave-uniform scalar loads.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "struct of 32-bit words");
    T v;
    const STORM_CONST_AS uint32_t *src = uniform_ptr(reinterpret_cast<const uint32_t *>(p));
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
    return v;
}

// A 32-bit word read by a vector (buffer) load even where its address is
// wave-uniform: workgroup barriers wait for outstanding scalar and LDS
// traffic only, so a value needed after a barrier, fetched this way early,
// does not hold the barrier up for its memory latency.
__device__ __forceinline__ uint32_t vector_load_u32(const void *p)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 4, 0x00020000);
    return __builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0);
}
__device__ __forceinline__ float vector_load_f32(const float *p) { return __uint_as_float(vector_load_u32(p)); }

// Hardware square root (v_sqrt_f32, 1 ulp) for norms and distances.
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Optional per-step outputs.
struct StepOut {
    float *u, *q, *v, *a, *c, *terms, *C;
    float *xd, *xdd;  // [6][N][H] flange velocity and acceleration (Eq. 8)
};

// Launchers (defined in the .hip translation units).
hipError_t launch_init_tables(const ProblemDev &P, const float *d_dt_raw, const float *d_lim_raw, float acc_stop,
                              float gamma, float w_term, float k_jl, float k_vl, const float *d_sigma_init,
                              const float comb[3], int n_knots, const float *d_obs_raw, int n_obs,
                              float4 *d_sph_obs, float *d_box_obs,
                              float4 *d_obs_bound, const float *d_sph_raw, int n_spheres, float4 *d_sph_local,
                              int32_t *d_sph_body, hipStream_t stream);
hipError_t launch_rollout(const ProblemDev &P, const RobotDev &R, const float *x0, const float *goal,
                          const float *noise, const StepOut &out, int waves, hipStream_t stream);
// Raise the dynamic-LDS limit of the rollout kernels to what the largest
// sphere model needs (idempotent).
hipError_t set_rollout_lds_limit();
// Whether the learned self-collision network's weight matrices (W1, W2, W3
// of storm_robot.self_mlp) hold FP16 values only, as its kernel requires.
bool selfnet_weights_fp16(const float *prm);
hipError_t launch_update(const ProblemDev &P, float *mean_out, float *sigma2_out, float *cmd, int shift,
                         hipStream_t stream);
// Learned self-collision term: after the rollout, adds a_coll max(0, d) to
// every running cost and its horizon sum to C (frag and bias packed by
// pack_selfnet from the parameter layout of storm_robot.self_mlp).
hipError_t launch_selfnet(const ProblemDev &P, const _Float16 *frag, const float *bias, const StepOut &out,
                          hipStream_t stream);
void pack_selfnet(const float *prm, std::vector<_Float16> &frag, std::vector<float> &bias);
// Many problems: persistent rollout over a (problem, tile) work queue, and one
// update workgroup per problem (descriptors in device memory).
hipError_t launch_rollout_batch(const ProblemDev *probs, const int2 *items, int n_items, uint32_t *next,
                                const RobotDev &R, const float *x0s, const float *goals, int waves, int grid,
                                hipStream_t stream);
hipError_t launch_update_batch(const ProblemDev *probs, int n_problems, float *cmd, int shift, hipStream_t stream);
// Differentiable form: adjoint + fixed-order reduction (grad, J) per joint;
// with it > 0 the same launch takes Adam step `it` on the stored mean, and
// with cmd it also writes the command and the shift of the refined mean.
// launch_command writes them for a refinement of zero steps.
hipError_t launch_grad(const ProblemDev &P, const RobotDev &R, const float *x0, const float *goal, const float *mean,
                       const float *noise, float *grad_out, float *J_out, int it, float lr, float *cmd, int shift,
                       hipStream_t stream);
hipError_t launch_command(const ProblemDev &P, float *cmd, int shift, hipStream_t stream);
// Batched refinement: `iterations` Adam steps on the gradient of every
// problem (adjoint over the (problem, chunk) items, then reduce + Adam per
// (problem, joint)), the last also writing the commands cmd [P][7] and the
// shift.
hipError_t launch_refine_batch(const ProblemDev *probs, int n_problems, const int2 *items, int n_items,
                               const RobotDev &R, const float *x0s, const float *goals, int iterations, float lr,
                               float *cmd, int shift, hipStream_t stream);
hipError_t launch_fk(const RobotDev &R, const float *q, int n, float *pose, float *manip, hipStream_t stream);

// Self-collision work items of the robot's sphere pairs, eight integers
// each (the rollout's queue; defined with its layout in the interface unit);
// returns the pair count.
// Self-collision groups: the spheres of one body in runs of up to four,
// (t_first, count), whose partners are the spheres s < s_end on bodies at
// least two earlier in the chain.
struct SelfGroup {
    int t_first, count, s_end;
};
std::vector<SelfGroup> self_groups(const storm_robot *robot);
int self_segments(const storm_robot *robot, std::vector<int> &items);
std::vector<float> self_thresholds(const storm_robot *robot, double reach);

}  // namespace storm

// One plain-form problem (the storm_ctx handle of the C ABI).
struct storm_ctx_s {
    int device = 0;
    int waves = 16;
    int32_t error = STORM_OK;  // sticky device error
    bool pending = false;      // a step waits for its update
    storm_params params{};
    storm::ProblemDev P{};
    storm::RobotDev R{};
    _Float16 *net_frag = nullptr;  // learned self-collision weights (packed), when self_model = 1
    float *net_bias = nullptr;
    float *scratch = nullptr;    // this device's static scratch (storm_rollout_grad_noalloc)
    std::vector<void *> allocs;  // every device allocation of this context
};

// An instantiated graph of one control step (plain or batched).
struct storm_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *error = nullptr;  // sticky error word of the owning context or batch
};
