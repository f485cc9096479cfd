// Batched form of the C ABI: many independent problems per launch, the work
// queue and its scheduler, the launch-shape autotuner, graph capture of a
// batch control step, and the closed-loop plant used by the benchmarks.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "storm_internal.h"

using namespace storm;

struct storm_batch_s {
    int device = 0;
    int32_t error = STORM_OK;
    bool pending = false;
    int n_problems = 0;
    int n_cu = 0;
    std::vector<storm_ctx> ctxs;  // per-problem workspace, tables and policy state
    RobotDev R{};                  // robot constants (problem 0's: every problem shares the robot)
    ProblemDev *d_probs = nullptr; // [P] descriptors
    int2 *d_items_cost = nullptr;  // work queue, most expensive tiles first
    int2 *d_items_plain = nullptr; // work queue in problem order
    int n_items = 0;
    uint32_t *d_next = nullptr;    // queue head (0 between launches)
    int2 *d_adj_items = nullptr;   // (problem, tile chunk) items of the batched adjoint
    int n_adj_items = 0;
    bool differentiable = true;    // every problem's gradient terms are differentiable
    storm_launch_config cfg{8, 0, 1};
    std::vector<void *> allocs;
};

namespace {

template <typename T>
hipError_t balloc(storm_batch b, T **ptr, size_t count)
{
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, count > 0 ? count * sizeof(T) : 16);
    if (e != hipSuccess) return e;
    b->allocs.push_back(p);
    *ptr = static_cast<T *>(p);
    return hipSuccess;
}

void free_batch(storm_batch b)
{
    for (storm_ctx c : b->ctxs) storm_rollout_destroy(c);
    b->ctxs.clear();
    for (void *p : b->allocs) (void)hipFree(p);
    b->allocs.clear();
}

// Estimated VALU work of one tile of problem p (the scheduler's sort key),
// in instructions per wave: the per-point kinematics, the environment broad
// phase (wave ball per sphere, one 64-obstacle chunk per pass) plus the few
// exact tests that survive it (about 2% of the pairs), and the sphere pairs.
double tile_cost(const ProblemDev &P, int n_spheres, int n_pairs)
{
    double per_wave = 1500.0;
    if (P.cost_mask & STORM_COST_ENV) {
        const int chunks = (P.n_sph_obs + P.n_box_obs + 63) / 64;
        per_wave += n_spheres * (40.0 + 12.0 * chunks + 0.02 * (5.0 * P.n_sph_obs + 19.0 * P.n_box_obs));
    }
    if (P.cost_mask & STORM_COST_SELF) per_wave += 7.0 * n_pairs;
    return per_wave;
}

int32_t launch_batch_step(storm_batch b, const float *d_x0, const float *d_goal, hipStream_t s)
{
    const RobotDev &R = b->R;
    const int2 *items = b->cfg.cost_order ? b->d_items_cost : b->d_items_plain;
    const hipError_t e =
        launch_rollout_batch(b->d_probs, items, b->n_items, b->d_next, R, d_x0, d_goal, b->cfg.waves, b->cfg.grid, s);
    return e == hipSuccess ? STORM_OK : STORM_E_DEVICE;
}

// One captured control step of the whole batch: K rounds of step + update
// (shift after the last round unless refinement follows), then
// `refine_iters` batched Adam steps, the commands and the shift.
int32_t batch_graph(storm_batch b, const float *d_x0, const float *d_goal, float *d_cmd, int32_t iterations,
                    int32_t shift, int32_t refine_iters, float lr, void *stream, storm_graph *out)
{
    if (!out) return STORM_E_NULL;
    *out = nullptr;
    if (!b || !d_x0 || !d_goal || !d_cmd) return STORM_E_NULL;
    if (iterations < 1 || refine_iters < 0) return STORM_E_RANGE;
    if (refine_iters > 0 && (!(lr >= 0.0f) || !isfinite(lr))) return STORM_E_PARAM;
    if (refine_iters > 0 && !b->differentiable) return STORM_E_UNSUPPORTED;
    if (b->error != STORM_OK) return b->error;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStream_t own = nullptr;
    if (s == nullptr) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) return STORM_E_DEVICE;
        s = own;
    }
    storm_graph g = new (std::nothrow) storm_graph_s();
    if (!g) {
        if (own) (void)hipStreamDestroy(own);
        return STORM_E_NOMEM;
    }
    g->error = &b->error;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    for (int k = 0; e == hipSuccess && k < iterations; ++k) {
        if (launch_batch_step(b, d_x0, d_goal, s) != STORM_OK) e = hipErrorLaunchFailure;
        const bool last_shift = (k == iterations - 1) && shift != 0 && refine_iters == 0;
        if (e == hipSuccess) e = launch_update_batch(b->d_probs, b->n_problems, d_cmd, last_shift, s);
    }
    if (e == hipSuccess && refine_iters > 0)
        e = launch_refine_batch(b->d_probs, b->n_problems, b->d_adj_items, b->n_adj_items, b->R, d_x0, d_goal,
                                refine_iters, lr, d_cmd, shift != 0, s);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    g->graph = graph;
    if (own) (void)hipStreamDestroy(own);
    if (e != hipSuccess) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return STORM_E_DEVICE;
    }
    *out = g;
    return STORM_OK;
}

__global__ void plant_kernel(float *__restrict__ x, const float *__restrict__ cmd, int n, float dt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kDof) return;
    const int p = t / kDof, j = t - p * kDof;
    float *xp = x + (size_t)p * 3 * kDof;
    const float u = cmd[t];
    const float v = fmaf(dt, u, xp[kDof + j]);
    xp[kDof + j] = v;
    xp[j] = fmaf(dt, v, xp[j]);
    xp[2 * kDof + j] = u;
}

}  // namespace

extern "C" {

int32_t storm_batch_init(storm_batch *out, int32_t n_problems, const storm_params *params, const storm_robot *robot,
                         const storm_scene *scenes, void *stream)
{
    if (!out) return STORM_E_NULL;
    *out = nullptr;
    if (!params || !robot) return STORM_E_NULL;
    if (n_problems < 1) return STORM_E_RANGE;
    // the ball term needs a per-problem ball state and the task-space form
    // of the rollout, which the persistent batched kernel does not carry
    for (int p = 0; p < n_problems; ++p)
        if ((params[p].cost_mask & STORM_COST_BALL) || params[p].self_model != 0) return STORM_E_UNSUPPORTED;
    storm_batch b = new (std::nothrow) storm_batch_s();
    if (!b) return STORM_E_NOMEM;
    b->n_problems = n_problems;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t st = STORM_OK;
    for (int p = 0; p < n_problems && st == STORM_OK; ++p) {
        storm_ctx c = nullptr;
        st = storm_rollout_init(&c, &params[p], robot, scenes ? &scenes[p] : nullptr, stream);
        if (st == STORM_OK) b->ctxs.push_back(c);
    }
    if (st != STORM_OK) {
        free_batch(b);
        delete b;
        return st;
    }
    hipError_t e = hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, b->device);
    if (e == hipSuccess) {
        b->n_cu = prop.multiProcessorCount;
        b->cfg.grid = 2 * b->n_cu;
    }
    if (e == hipSuccess) b->R = b->ctxs[0]->R;

    // descriptors and the work queues
    std::vector<ProblemDev> probs(n_problems);
    std::vector<int2> plain;
    std::vector<double> cost;
    for (int p = 0; p < n_problems; ++p) {
        probs[p] = b->ctxs[p]->P;
        const double tc = tile_cost(probs[p], robot->n_spheres, b->ctxs[p]->R.n_pairs);
        for (int t = 0; t < probs[p].n_tiles; ++t) {
            plain.push_back(make_int2(p, t));
            cost.push_back(tc);
        }
    }
    b->n_items = (int)plain.size();
    std::vector<int2> adj;
    for (int p = 0; p < n_problems; ++p) {
        const int chunks = probs[p].n_tiles < kAdjChunks ? probs[p].n_tiles : kAdjChunks;
        for (int c = 0; c < chunks; ++c) adj.push_back(make_int2(p, c));
        if (probs[p].grad_mask & ~(STORM_COST_POSE | STORM_COST_JOINT | STORM_COST_VEL | STORM_COST_STOP))
            b->differentiable = false;
    }
    b->n_adj_items = (int)adj.size();
    std::vector<int> order(plain.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<int2> sorted(plain.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = plain[order[k]];
    if (e == hipSuccess) e = balloc(b, &b->d_probs, (size_t)n_problems);
    if (e == hipSuccess) e = balloc(b, &b->d_items_cost, plain.size());
    if (e == hipSuccess) e = balloc(b, &b->d_items_plain, plain.size());
    if (e == hipSuccess) e = balloc(b, &b->d_next, (size_t)1);
    if (e == hipSuccess) e = balloc(b, &b->d_adj_items, adj.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->d_adj_items, adj.data(), sizeof(int2) * adj.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_probs, probs.data(), sizeof(ProblemDev) * probs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_items_cost, sorted.data(), sizeof(int2) * sorted.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_items_plain, plain.data(), sizeof(int2) * plain.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_next, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_batch(b);
        delete b;
        return e == hipErrorOutOfMemory ? STORM_E_NOMEM : STORM_E_DEVICE;
    }
    *out = b;
    return STORM_OK;
}

int32_t storm_batch_step(storm_batch b, const float *d_x0, const float *d_goal, void *stream)
{
    if (!b || !d_x0 || !d_goal) return STORM_E_NULL;
    if (b->error != STORM_OK) return b->error;
    const int32_t st = launch_batch_step(b, d_x0, d_goal, static_cast<hipStream_t>(stream));
    if (st != STORM_OK) {
        b->error = st;
        return st;
    }
    b->pending = true;
    return STORM_OK;
}

int32_t storm_batch_update(storm_batch b, float *d_cmd, int32_t shift, void *stream)
{
    if (!b || !d_cmd) return STORM_E_NULL;
    if (b->error != STORM_OK) return b->error;
    if (!b->pending) return STORM_E_STATE;
    if (launch_update_batch(b->d_probs, b->n_problems, d_cmd, shift != 0, static_cast<hipStream_t>(stream)) !=
        hipSuccess) {
        b->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    b->pending = false;
    return STORM_OK;
}

int32_t storm_batch_graph_create(storm_batch b, const float *d_x0, const float *d_goal, float *d_cmd,
                                 int32_t iterations, int32_t shift, void *stream, storm_graph *out)
{
    return batch_graph(b, d_x0, d_goal, d_cmd, iterations, shift, 0, 0.0f, stream, out);
}

int32_t storm_batch_graph_create_refine(storm_batch b, const float *d_x0, const float *d_goal, float *d_cmd,
                                        int32_t iterations, int32_t shift, int32_t refine_iters, float lr,
                                        void *stream, storm_graph *out)
{
    return batch_graph(b, d_x0, d_goal, d_cmd, iterations, shift, refine_iters, lr, stream, out);
}

int32_t storm_batch_refine(storm_batch b, const float *d_x0, const float *d_goal, int32_t iterations, float lr,
                           float *d_cmd, int32_t shift, void *stream)
{
    if (!b || !d_x0 || !d_goal || !d_cmd) return STORM_E_NULL;
    if (iterations < 0) return STORM_E_RANGE;
    if (!(lr >= 0.0f) || !isfinite(lr)) return STORM_E_PARAM;
    if (b->error != STORM_OK) return b->error;
    if (!b->differentiable) return STORM_E_UNSUPPORTED;
    if (launch_refine_batch(b->d_probs, b->n_problems, b->d_adj_items, b->n_adj_items, b->R, d_x0, d_goal,
                            iterations, lr, d_cmd, shift != 0, static_cast<hipStream_t>(stream)) != hipSuccess) {
        b->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_batch_set_config(storm_batch b, const storm_launch_config *cfg)
{
    if (!b || !cfg) return STORM_E_NULL;
    if ((cfg->waves != 8 && cfg->waves != 16) || cfg->grid < 1) return STORM_E_RANGE;
    b->cfg = *cfg;
    b->cfg.cost_order = cfg->cost_order != 0;
    return STORM_OK;
}

int32_t storm_batch_get_config(storm_batch b, storm_launch_config *cfg)
{
    if (!b || !cfg) return STORM_E_NULL;
    *cfg = b->cfg;
    return STORM_OK;
}

int32_t storm_batch_autotune(storm_batch b, const float *d_x0, const float *d_goal, int32_t reps, void *stream,
                             storm_launch_config *best, float *h_times, int32_t *n_candidates)
{
    if (!b || !d_x0 || !d_goal) return STORM_E_NULL;
    if (reps < 1) return STORM_E_RANGE;
    if (b->error != STORM_OK) return b->error;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<storm_launch_config> cand;
    for (int w : {8, 16})
        for (int k = 1; k <= 4; ++k)
            for (int order : {1, 0}) cand.push_back(storm_launch_config{w, k * b->n_cu, order});
    const storm_launch_config saved = b->cfg;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return STORM_E_DEVICE;
    }
    float best_us = INFINITY;
    storm_launch_config best_cfg = saved;
    int32_t st = STORM_OK;
    const int cap = n_candidates ? *n_candidates : 0;
    for (size_t k = 0; k < cand.size() && st == STORM_OK; ++k) {
        b->cfg = cand[k];
        st = launch_batch_step(b, d_x0, d_goal, s);  // warm-up
        if (st != STORM_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) st = STORM_E_DEVICE;
        for (int r = 0; r < reps && st == STORM_OK; ++r) st = launch_batch_step(b, d_x0, d_goal, s);
        float ms = 0.0f;
        if (st == STORM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = STORM_E_DEVICE;
        const float us = 1000.0f * ms / (float)reps;
        if (h_times && (int)k < cap) h_times[k] = us;
        if (st == STORM_OK && us < best_us) {
            best_us = us;
            best_cfg = cand[k];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_candidates) *n_candidates = (int32_t)cand.size();
    if (st != STORM_OK) {
        b->cfg = saved;
        b->error = STORM_E_DEVICE;
        return st;
    }
    b->cfg = best_cfg;
    b->pending = false;
    if (best) *best = best_cfg;
    return STORM_OK;
}

int32_t storm_batch_get_state(storm_batch b, int32_t problem, float *h_mean, float *h_sigma2, uint32_t *h_step,
                              void *stream)
{
    if (!b) return STORM_E_NULL;
    if (problem < 0 || problem >= b->n_problems) return STORM_E_RANGE;
    return storm_rollout_get_state(b->ctxs[problem], h_mean, h_sigma2, h_step, stream);
}

int32_t storm_batch_set_state(storm_batch b, int32_t problem, const float *h_mean, const float *h_sigma2,
                              const uint32_t *h_step, void *stream)
{
    if (!b) return STORM_E_NULL;
    if (problem < 0 || problem >= b->n_problems) return STORM_E_RANGE;
    const int32_t st = storm_rollout_set_state(b->ctxs[problem], h_mean, h_sigma2, h_step, stream);
    if (st == STORM_OK) b->pending = false;
    return st;
}

int32_t storm_batch_costs(storm_batch b, int32_t problem, float *h_C, void *stream)
{
    if (!b || !h_C) return STORM_E_NULL;
    if (problem < 0 || problem >= b->n_problems) return STORM_E_RANGE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const ProblemDev &P = b->ctxs[problem]->P;
    hipError_t e = hipMemcpyAsync(h_C, P.C, sizeof(float) * P.N, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? STORM_OK : STORM_E_DEVICE;
}

int32_t storm_batch_destroy(storm_batch b)
{
    if (!b) return STORM_OK;
    (void)hipDeviceSynchronize();
    free_batch(b);
    delete b;
    return STORM_OK;
}

int32_t storm_plant_step(float *d_x, const float *d_cmd, int32_t n, float dt, void *stream)
{
    if (n < 0) return STORM_E_RANGE;
    if (n > 0 && (!d_x || !d_cmd)) return STORM_E_NULL;
    if (!(dt > 0.0f) || !isfinite(dt)) return STORM_E_PARAM;
    if (n == 0) return STORM_OK;
    const int total = n * kDof;
    hipLaunchKernelGGL(plant_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), d_x, d_cmd, n, dt);
    return hipGetLastError() == hipSuccess ? STORM_OK : STORM_E_DEVICE;
}

}  // extern "C"
