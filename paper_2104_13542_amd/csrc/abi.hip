// C ABI of the STORM MPPI library: validation, device workspace and launch
// order for init / step / update / destroy (Alg. 1), status and state I/O.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "storm_internal.h"

using namespace storm;

// Scratch of storm_rollout_grad_noalloc: the adjoint's partial gradients
// [kAdjChunks][7][kMaxH] and partial horizon-cost sums [kAdjChunks] of any
// context (its chunk count is at most kAdjChunks), 0.9 MB per device, held
// until the process ends.  Host code never uses this name as an address: the
// device address of each device's copy comes from hipGetSymbolAddress, once
// per device, in storm_rollout_init.
namespace {
constexpr size_t kNoallocGradFloats = (size_t)kAdjChunks * STORM_DOF * kMaxH;
constexpr size_t kNoallocFloats = kNoallocGradFloats + (size_t)kAdjChunks;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) float scratch[kNoallocFloats];

namespace {

std::mutex g_scratch_mutex;
float *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call for that device), or nullptr if it cannot be had.
float *scratch_on_current_device(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[device] = static_cast<float *>(ptr);
    }
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

bool finite_f(float x) { return isfinite(x) != 0; }

int32_t validate_robot(const storm_robot *robot)
{
    if (!robot) return STORM_E_NULL;
    if (robot->n_spheres < 0 || robot->n_spheres > STORM_MAX_SPHERES) return STORM_E_RANGE;
    if (robot->n_spheres > 0 && !robot->spheres) return STORM_E_NULL;
    for (int k = 0; k < STORM_NFRAMES; ++k)
        for (int c = 0; c < 3; ++c)
            if (!finite_f(robot->dh[k][c])) return STORM_E_PARAM;
    for (int j = 0; j < STORM_DOF; ++j) {
        if (!finite_f(robot->q_min[j]) || !finite_f(robot->q_max[j]) || !(robot->q_min[j] < robot->q_max[j]))
            return STORM_E_PARAM;
        if (!finite_f(robot->qd_max[j]) || !(robot->qd_max[j] > 0.0f)) return STORM_E_PARAM;
    }
    for (int s = 0; s < robot->n_spheres; ++s) {
        const float *r = robot->spheres + 5 * s;
        const int b = (int)r[0];
        if ((float)b != r[0] || b < 1 || b > STORM_NFRAMES) return STORM_E_PARAM;
        if (s > 0 && r[0] < robot->spheres[5 * (s - 1)]) return STORM_E_PARAM;  // sorted by body
        for (int c = 1; c < 5; ++c)
            if (!finite_f(r[c])) return STORM_E_PARAM;
        if (!(r[4] > 0.0f && r[4] < 1.0f)) return STORM_E_PARAM;  // body spheres: 0 < r < 1 m
    }
    return STORM_OK;
}

int32_t validate_scene(const storm_scene *scene)
{
    if (!scene) return STORM_OK;  // no obstacles
    if (scene->n_obstacles < 0 || scene->n_obstacles > STORM_MAX_OBSTACLES) return STORM_E_RANGE;
    if (scene->n_obstacles > 0 && !scene->obstacles) return STORM_E_NULL;
    for (int o = 0; o < scene->n_obstacles; ++o) {
        const float *r = scene->obstacles + STORM_OBSTACLE_STRIDE * o;
        for (int c = 0; c < STORM_OBSTACLE_STRIDE; ++c)
            if (!finite_f(r[c])) return STORM_E_PARAM;
        if (r[0] == (float)STORM_OBSTACLE_SPHERE) {
            if (!(r[4] > 0.0f)) return STORM_E_PARAM;
        } else if (r[0] == (float)STORM_OBSTACLE_CUBOID) {
            if (!(r[4] > 0.0f && r[5] > 0.0f && r[6] > 0.0f)) return STORM_E_PARAM;
        } else {
            return STORM_E_PARAM;
        }
    }
    return STORM_OK;
}

// Element count of the stored variance: [7], or [H][7] per step.
int n_sigma2(const storm::ProblemDev &P) { return P.cov_step ? P.H * STORM_DOF : STORM_DOF; }

int32_t validate_params(const storm_params *p)
{
    if (!p) return STORM_E_NULL;
    if (p->n_particles < 1 || p->n_particles > STORM_MAX_PARTICLES) return STORM_E_RANGE;
    if (p->horizon < 1 || p->horizon > STORM_MAX_HORIZON) return STORM_E_RANGE;
    if (p->n_null < 0 || p->n_null > p->n_particles) return STORM_E_RANGE;
    if (p->n_halton < 0 || p->n_halton > p->n_particles - p->n_null) return STORM_E_RANGE;
    if (p->n_halton > 0 && (p->n_knots < 4 || p->n_knots > 32)) return STORM_E_RANGE;
    if (p->cost_mask & ~(STORM_COST_ALL | STORM_COST_BALL)) return STORM_E_PARAM;
    if (p->grad_mask & ~(STORM_COST_POSE | STORM_COST_JOINT | STORM_COST_VEL | STORM_COST_STOP)) return STORM_E_PARAM;
    if (p->comb_filter != 0 && p->comb_filter != 1) return STORM_E_PARAM;
    if (p->cov_per_step != 0 && p->cov_per_step != 1) return STORM_E_PARAM;
    if (p->self_model != 0 && p->self_model != 1) return STORM_E_PARAM;
    for (int c = 0; c < 3; ++c)
        if (!finite_f(p->comb[c]) || !finite_f(p->ball_gravity[c])) return STORM_E_PARAM;
    if (!finite_f(p->w_ball) || p->w_ball < 0.0f) return STORM_E_PARAM;
    if (!finite_f(p->ball_center[0]) || !finite_f(p->ball_center[1])) return STORM_E_PARAM;
    if (!p->dt) return STORM_E_NULL;
    for (int h = 0; h < p->horizon; ++h)
        if (!finite_f(p->dt[h]) || !(p->dt[h] > 0.0f)) return STORM_E_PARAM;
    for (int j = 0; j < STORM_DOF; ++j)
        if (!finite_f(p->sigma_init[j]) || !(p->sigma_init[j] > 0.0f)) return STORM_E_PARAM;
    const float scalars[] = {p->beta,  p->gamma, p->alpha_mu, p->alpha_sigma, p->w_term, p->sigma2_min,
                             p->acc_stop, p->k_jl, p->k_vl, p->k_m, p->w_pos, p->w_rot,
                             p->a_stop, p->a_joint, p->a_vel, p->a_manip, p->a_coll};
    for (float s : scalars)
        if (!finite_f(s)) return STORM_E_PARAM;
    for (int c = 0; c < 3; ++c)
        if (!finite_f(p->alpha_pos[c]) || !finite_f(p->alpha_rot[c])) return STORM_E_PARAM;
    if (!(p->beta > 0.0f)) return STORM_E_PARAM;
    if (p->gamma < 0.0f || p->gamma > 1.0f) return STORM_E_PARAM;
    if (p->alpha_mu < 0.0f || p->alpha_mu > 1.0f) return STORM_E_PARAM;
    if (p->alpha_sigma < 0.0f || p->alpha_sigma > 1.0f) return STORM_E_PARAM;
    if (p->w_term < 0.0f || p->sigma2_min < 0.0f || p->acc_stop < 0.0f) return STORM_E_PARAM;
    if (p->k_jl < 0.0f || p->k_jl >= 0.5f || p->k_vl < 0.0f || p->k_vl >= 0.5f) return STORM_E_PARAM;
    return STORM_OK;
}

// Robot constants in device form.  cos/sin of the DH twist are formed in
// double; values within 1e-12 of 0 or +-1 are snapped so that the usual
// twists of +-pi/2 give exact axis permutations.
void fill_robot_consts(const storm_robot *robot, RobotDev &R)
{
    for (int k = 0; k < STORM_NFRAMES; ++k) {
        double c = cos((double)robot->dh[k][2]), s = sin((double)robot->dh[k][2]);
        if (fabs(c) < 1e-12) c = 0.0;
        if (fabs(s) < 1e-12) s = 0.0;
        if (fabs(fabs(c) - 1.0) < 1e-12) c = c > 0 ? 1.0 : -1.0;
        if (fabs(fabs(s) - 1.0) < 1e-12) s = s > 0 ? 1.0 : -1.0;
        R.ca[k] = (float)c;
        R.sa[k] = (float)s;
        R.a[k] = robot->dh[k][0];
        R.d[k] = robot->dh[k][1];
    }
    R.n_spheres = robot->n_spheres;
}

// Upper bound of the distance from the base of any body-sphere centre: the
// frame origins move along a chain whose links have lengths at most
// |a_k| + |d_k|, and a sphere sits |local centre| from its frame origin.
double reach_bound(const storm_robot *robot)
{
    double r = 0.0, loc = 0.0;
    for (int k = 0; k < STORM_NFRAMES; ++k) r += fabs((double)robot->dh[k][0]) + fabs((double)robot->dh[k][1]);
    for (int s = 0; s < robot->n_spheres; ++s) {
        const float *q = robot->spheres + 5 * s;
        loc = fmax(loc, sqrt((double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]));
    }
    return r + loc;
}

}  // namespace

std::vector<storm::SelfGroup> storm::self_groups(const storm_robot *robot)
{
    const int S = robot->n_spheres;
    std::vector<SelfGroup> g;
    for (int t = 0; t < S;) {
        const int body = (int)robot->spheres[5 * t];
        int n = 1;
        while (t + n < S && n < 4 && (int)robot->spheres[5 * (t + n)] == body) ++n;
        int s_end = 0;  // spheres are sorted by body
        while (s_end < S && (int)robot->spheres[5 * s_end] <= body - 2) ++s_end;
        g.push_back(SelfGroup{t, n, s_end});
        t += n;
    }
    return g;
}

// Self-collision work items: one per (group, partner body), partners
// [s_begin, s_end) the spheres of that body, written as eight integers
// (t_first | count << 8, group, s_begin, s_end, a_t, a_s, bits of reach2, 0).
// Broad phase: a_t is the sphere of the group, a_s the sphere of the partner
// body, about whose centres the balls of radius R_t = max |c_t - c_a_t| + r_t
// and R_s (likewise) hold every sphere of each side (each anchor chosen to
// make its radius smallest); reach2 = (R_t + R_s + 1 mm)^2 rounded up.  Where
// the anchors' centres are farther apart than R_t + R_s, no pair of the item
// touches, and the millimetre covers the FP32 rounding of the centres
// (micrometres within the robot's reach).  The rollout workgroup's waves take
// the items from a queue in this order: most rounds (pairs of partners)
// first.  Returns the pair count.
int storm::self_segments(const storm_robot *robot, std::vector<int> &items)
{
    const std::vector<SelfGroup> groups = self_groups(robot);
    const float *sp = robot->spheres;
    auto anchor = [&](int lo, int hi, double &radius) {
        int best = lo;
        radius = INFINITY;
        for (int k = lo; k < hi; ++k) {
            double r = 0.0;
            for (int m = lo; m < hi; ++m) {
                const double dx = (double)sp[5 * m + 1] - sp[5 * k + 1], dy = (double)sp[5 * m + 2] - sp[5 * k + 2],
                             dz = (double)sp[5 * m + 3] - sp[5 * k + 3];
                r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz) + (double)sp[5 * m + 4]);
            }
            if (r < radius) {
                radius = r;
                best = k;
            }
        }
        return best;
    };
    struct Item {
        int v[8];
        int rounds, order;
    };
    std::vector<Item> list;
    long long pairs = 0;
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        const SelfGroup &g = groups[gi];
        pairs += (long long)g.count * g.s_end;
        double rt = 0.0;
        const int at = anchor(g.t_first, g.t_first + g.count, rt);
        for (int lo = 0; lo < g.s_end;) {
            int hi = lo + 1;
            while (hi < g.s_end && (int)sp[5 * hi] == (int)sp[5 * lo]) ++hi;
            double rs = 0.0;
            const int as = anchor(lo, hi, rs);
            const double reach = rt + rs + 1.0e-3;
            const float reach2 = nextafterf((float)(reach * reach), INFINITY);
            Item it{};
            it.v[0] = g.t_first | (g.count << 8);
            it.v[1] = gi;
            it.v[2] = lo;
            it.v[3] = hi;
            it.v[4] = at;
            it.v[5] = as;
            memcpy(&it.v[6], &reach2, sizeof(float));
            it.rounds = (hi - lo + 1) / 2;
            it.order = (int)list.size();
            list.push_back(it);
            lo = hi;
        }
    }
    std::stable_sort(list.begin(), list.end(), [](const Item &x, const Item &y) { return x.rounds > y.rounds; });
    items.clear();
    for (const Item &it : list) items.insert(items.end(), it.v, it.v + 8);
    return (int)pairs;
}

// Records of the expanded pair test, [group][s][8] for partner s of the
// group spheres t = t_first + k: entries k = 0..3 the threshold of
// |c_s|^2 - 2 c_s.c_t + |c_t|^2 < (r_s + r_t)^2 + slack, entries 4 + k the
// contact distance r_s + r_t.  The FP32 evaluation of the test errs by less
// than 2^-24 * 12 (|c_s| + |c_t|)^2, and the slack, 2^-18 (2 reach + r_s +
// r_t)^2, is over five times that with both centres within the robot's
// reach.  Slots past a group's count, and partners s outside its range, hold
// the threshold -1e30 (never a hit) and contact distance 0.
std::vector<float> storm::self_thresholds(const storm_robot *robot, double reach)
{
    const int S = robot->n_spheres;
    const std::vector<SelfGroup> groups = self_groups(robot);
    std::vector<float> thr(groups.size() * (size_t)S * 8, 0.0f);
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (int s = 0; s < S; ++s)
            for (int k = 0; k < 4; ++k) {
                float *rec = &thr[(gi * S + s) * 8];
                rec[k] = -1.0e30f;
                if (s >= groups[gi].s_end || k >= groups[gi].count) continue;
                const int t = groups[gi].t_first + k;
                const double rs = (double)robot->spheres[5 * s + 4] + (double)robot->spheres[5 * t + 4];
                const double span = 2.0 * reach + rs;
                rec[k] = (float)(rs * rs + ldexp(span * span, -18));
                rec[4 + k] = (float)rs;
            }
    return thr;
}

namespace {

template <typename T>
hipError_t dalloc(storm_ctx c, T **ptr, size_t count)
{
    void *p = nullptr;
    const size_t bytes = count > 0 ? count * sizeof(T) : 16;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    c->allocs.push_back(p);
    *ptr = static_cast<T *>(p);
    return hipSuccess;
}

void free_all(storm_ctx c)
{
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

int32_t map_error(hipError_t e) { return e == hipErrorOutOfMemory ? STORM_E_NOMEM : STORM_E_DEVICE; }

}  // namespace

extern "C" {

const char *storm_status_str(int32_t status)
{
    switch (status) {
    case STORM_OK: return "ok";
    case STORM_E_NULL: return "null pointer";
    case STORM_E_RANGE: return "size out of range";
    case STORM_E_PARAM: return "invalid parameter";
    case STORM_E_DEVICE: return "device error";
    case STORM_E_STATE: return "call out of order";
    case STORM_E_NOMEM: return "out of device memory";
    case STORM_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int32_t storm_rollout_init(storm_ctx *out, const storm_params *params, const storm_robot *robot,
                           const storm_scene *scene, void *stream)
{
    if (!out) return STORM_E_NULL;
    *out = nullptr;
    int32_t st = validate_params(params);
    if (st != STORM_OK) return st;
    st = validate_robot(robot);
    if (st != STORM_OK) return st;
    st = validate_scene(scene);
    if (st != STORM_OK) return st;
    if (params->self_model == 1) {
        if (!robot->self_mlp) return STORM_E_NULL;
        for (int k = 0; k < STORM_SELF_MLP_SIZE; ++k)
            if (!finite_f(robot->self_mlp[k])) return STORM_E_PARAM;
        if (!storm::selfnet_weights_fp16(robot->self_mlp)) return STORM_E_PARAM;
    }

    hipStream_t s = static_cast<hipStream_t>(stream);
    storm_ctx c = new (std::nothrow) storm_ctx_s();
    if (!c) return STORM_E_NOMEM;
    c->params = *params;
    c->params.dt = nullptr;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return STORM_E_DEVICE;
    }
    c->scratch = scratch_on_current_device(c->device);
    if (!c->scratch) {
        delete c;
        return STORM_E_DEVICE;
    }
    if (storm::set_rollout_lds_limit() != hipSuccess) {
        delete c;
        return STORM_E_DEVICE;
    }

    const int N = params->n_particles, H = params->horizon;
    const int n_obs = scene ? scene->n_obstacles : 0;
    // obstacle records re-ordered: spheres first, then cuboids
    std::vector<float> obs_sorted;
    obs_sorted.reserve((size_t)STORM_OBSTACLE_STRIDE * n_obs);
    int n_sph_obs = 0, n_box_obs = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int o = 0; o < n_obs; ++o) {
            const float *r = scene->obstacles + STORM_OBSTACLE_STRIDE * o;
            const bool is_sphere = r[0] == (float)STORM_OBSTACLE_SPHERE;
            if (is_sphere != (pass == 0)) continue;
            obs_sorted.insert(obs_sorted.end(), r, r + STORM_OBSTACLE_STRIDE);
            if (is_sphere) ++n_sph_obs; else ++n_box_obs;
        }
    const float comb[3] = {params->comb_filter ? params->comb[0] : 1.0f, params->comb_filter ? params->comb[1] : 0.0f,
                           params->comb_filter ? params->comb[2] : 0.0f};
    std::vector<int> seg;
    const int n_pairs = storm::self_segments(robot, seg);
    std::vector<_Float16> net_frag;
    std::vector<float> net_bias;
    if (params->self_model == 1) storm::pack_selfnet(robot->self_mlp, net_frag, net_bias);
    const std::vector<float> thr = storm::self_thresholds(robot, reach_bound(robot));
    const int n_seg = (int)seg.size() / 8;

    ProblemDev &P = c->P;
    P.N = N;
    P.H = H;
    P.n_halton = params->n_halton;
    P.comb = params->comb_filter ? 1u : 0u;
    P.cov_step = params->cov_per_step ? 1u : 0u;
    P.n_null = params->n_null;
    P.n_sph_obs = n_sph_obs;
    P.n_box_obs = n_box_obs;
    P.ppt = storm::kLanes / H;
    P.n_tiles = (N + P.ppt - 1) / P.ppt;
    P.cost_mask = params->cost_mask;
    P.grad_mask = params->grad_mask != 0 ? params->grad_mask : params->cost_mask;
    // the learned model replaces the sphere pairs: the rollout leaves the
    // self-collision term to the network pass
    P.selfnet = (params->self_model == 1 && (params->cost_mask & STORM_COST_SELF)) ? 1u : 0u;
    if (P.selfnet) P.cost_mask &= ~STORM_COST_SELF;
    P.seed_lo = (uint32_t)params->seed;
    P.seed_hi = (uint32_t)(params->seed >> 32);
    P.beta = params->beta;
    P.alpha_mu = params->alpha_mu;
    P.alpha_sigma = params->alpha_sigma;
    P.sigma2_min = params->sigma2_min;
    P.k_m = params->k_m;
    P.w_pos = params->w_pos;
    P.w_rot = params->w_rot;
    P.a_stop = params->a_stop;
    P.a_joint = params->a_joint;
    P.a_vel = params->a_vel;
    P.a_manip = params->a_manip;
    P.a_coll = params->a_coll;
    for (int k = 0; k < 3; ++k) {
        P.alpha_pos[k] = params->alpha_pos[k];
        P.alpha_rot[k] = params->alpha_rot[k];
        P.ball_g[k] = params->ball_gravity[k];
    }
    P.w_ball = params->w_ball;
    P.ball_c[0] = params->ball_center[0];
    P.ball_c[1] = params->ball_center[1];
    fill_robot_consts(robot, c->R);
    c->R.n_pairs = n_pairs;

    float *tables, *halton, *box_obs, *mean, *sigma2, *u, *C, *dt_raw, *lim_raw, *sig_raw, *obs_raw, *sph_raw_d;
    float *self_thr, *grad_part, *cost_part, *grad, *adam, *ball, *qbuf = nullptr;
    float4 *sph_obs, *obs_bound, *sph_local;
    int32_t *sph_body, *self_seg;
    uint32_t *counters;
    hipError_t e = hipSuccess;
#define STORM_TRY(expr)        \
    do {                       \
        e = (expr);            \
        if (e != hipSuccess) { \
            goto fail;         \
        }                      \
    } while (0)
    STORM_TRY(dalloc(c, &tables, storm::kTabSize));
    STORM_TRY(dalloc(c, &halton, (size_t)STORM_DOF * params->n_halton * H));
    STORM_TRY(dalloc(c, &sph_obs, (size_t)n_sph_obs));
    STORM_TRY(dalloc(c, &box_obs, (size_t)16 * n_box_obs));
    STORM_TRY(dalloc(c, &obs_bound, (size_t)n_obs));
    STORM_TRY(dalloc(c, &mean, (size_t)H * STORM_DOF));
    STORM_TRY(dalloc(c, &sigma2, (size_t)H * STORM_DOF));  // [7] or [H][7] (cov_per_step)
    STORM_TRY(dalloc(c, &u, (size_t)STORM_DOF * N * H));
    STORM_TRY(dalloc(c, &C, (size_t)N));
    STORM_TRY(dalloc(c, &counters, (size_t)4));
    {
        const int chunks = P.n_tiles < storm::kAdjChunks ? P.n_tiles : storm::kAdjChunks;
        STORM_TRY(dalloc(c, &grad_part, (size_t)chunks * STORM_DOF * storm::kMaxH));
        STORM_TRY(dalloc(c, &cost_part, (size_t)chunks));
    }
    STORM_TRY(dalloc(c, &grad, (size_t)H * STORM_DOF));
    STORM_TRY(dalloc(c, &adam, (size_t)2 * H * STORM_DOF));
    STORM_TRY(dalloc(c, &ball, (size_t)8));
    if (P.selfnet) {
        STORM_TRY(dalloc(c, &qbuf, (size_t)STORM_DOF * N * H));
        STORM_TRY(dalloc(c, &c->net_frag, net_frag.size()));
        STORM_TRY(dalloc(c, &c->net_bias, net_bias.size()));
        STORM_TRY(hipMemcpyAsync(c->net_frag, net_frag.data(), sizeof(_Float16) * net_frag.size(),
                                 hipMemcpyHostToDevice, s));
        STORM_TRY(hipMemcpyAsync(c->net_bias, net_bias.data(), sizeof(float) * net_bias.size(),
                                 hipMemcpyHostToDevice, s));
    }
    STORM_TRY(dalloc(c, &sph_local, (size_t)robot->n_spheres));
    STORM_TRY(dalloc(c, &sph_body, (size_t)robot->n_spheres));
    STORM_TRY(dalloc(c, &self_thr, thr.size()));
    STORM_TRY(dalloc(c, &self_seg, (size_t)8 * n_seg));
    // staging copies of the host inputs (freed at destroy with the rest)
    STORM_TRY(dalloc(c, &dt_raw, (size_t)H));
    STORM_TRY(dalloc(c, &lim_raw, (size_t)3 * STORM_DOF));
    STORM_TRY(dalloc(c, &sig_raw, (size_t)STORM_DOF));
    STORM_TRY(dalloc(c, &obs_raw, (size_t)STORM_OBSTACLE_STRIDE * n_obs));
    STORM_TRY(dalloc(c, &sph_raw_d, (size_t)5 * robot->n_spheres));
    {
        float lim[3 * STORM_DOF];
        for (int j = 0; j < STORM_DOF; ++j) {
            lim[j] = robot->q_min[j];
            lim[STORM_DOF + j] = robot->q_max[j];
            lim[2 * STORM_DOF + j] = robot->qd_max[j];
        }
        STORM_TRY(hipMemcpyAsync(dt_raw, params->dt, sizeof(float) * H, hipMemcpyHostToDevice, s));
        STORM_TRY(hipMemcpyAsync(lim_raw, lim, sizeof(lim), hipMemcpyHostToDevice, s));
        STORM_TRY(hipMemcpyAsync(sig_raw, params->sigma_init, sizeof(float) * STORM_DOF, hipMemcpyHostToDevice, s));
        if (n_obs > 0)
            STORM_TRY(hipMemcpyAsync(obs_raw, obs_sorted.data(), sizeof(float) * obs_sorted.size(),
                                     hipMemcpyHostToDevice, s));
        if (robot->n_spheres > 0)
            STORM_TRY(hipMemcpyAsync(sph_raw_d, robot->spheres, sizeof(float) * 5 * robot->n_spheres,
                                     hipMemcpyHostToDevice, s));
        if (n_seg > 0)
            STORM_TRY(hipMemcpyAsync(self_seg, seg.data(), sizeof(int) * seg.size(), hipMemcpyHostToDevice, s));
        if (!thr.empty())
            STORM_TRY(hipMemcpyAsync(self_thr, thr.data(), sizeof(float) * thr.size(), hipMemcpyHostToDevice, s));
        P.tables = tables;
        P.halton = halton;
        P.sph_obs = sph_obs;
        P.box_obs = box_obs;
        P.obs_bound = obs_bound;
        P.mean = mean;
        P.sigma2 = sigma2;
        P.u = u;
        P.C = C;
        P.step = counters;
        P.status = counters + 1;
        P.last_step = counters + 2;
        P.grad_part = grad_part;
        P.cost_part = cost_part;
        P.grad = grad;
        P.ball = ball;
        P.qbuf = qbuf;
        P.net_frag = c->net_frag;
        P.net_bias = c->net_bias;
        P.adam_m = adam;
        P.adam_v = adam + (size_t)H * STORM_DOF;
        c->R.sph_local = sph_local;
        c->R.sph_body = sph_body;
        c->R.self_thr = self_thr;
        c->R.self_items = self_seg;
        c->R.n_self_items = n_seg;
        STORM_TRY(storm::launch_init_tables(P, dt_raw, lim_raw, params->acc_stop, params->gamma, params->w_term,
                                            params->k_jl, params->k_vl, sig_raw, comb, params->n_knots, obs_raw,
                                            n_obs,
                                            sph_obs, box_obs, obs_bound, sph_raw_d, robot->n_spheres, sph_local,
                                            sph_body, s));
        STORM_TRY(hipStreamSynchronize(s));
    }
#undef STORM_TRY
    *out = c;
    return STORM_OK;
fail:
    (void)hipStreamSynchronize(s);
    free_all(c);
    delete c;
    return map_error(e);
}

// The rollout of one step, and with the learned self-collision model its
// network pass after it.
static hipError_t enqueue_rollout(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_noise,
                                  const StepOut &out, hipStream_t s)
{
    hipError_t e = storm::launch_rollout(ctx->P, ctx->R, d_x0, d_goal, d_noise, out, ctx->waves, s);
    if (e == hipSuccess && ctx->P.selfnet)
        e = storm::launch_selfnet(ctx->P, ctx->net_frag, ctx->net_bias, out, s);
    return e;
}

int32_t storm_rollout_step(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_noise,
                           const storm_debug *dbg, float *d_C, void *stream)
{
    if (!ctx || !d_x0 || !d_goal) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    StepOut out{};
    if (dbg) {
        out.u = dbg->u;
        out.q = dbg->q;
        out.v = dbg->v;
        out.a = dbg->a;
        out.c = dbg->c;
        out.terms = dbg->terms;
        out.xd = dbg->xd;
        out.xdd = dbg->xdd;
    }
    out.C = d_C;
    const hipError_t e = enqueue_rollout(ctx, d_x0, d_goal, d_noise, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    ctx->pending = true;
    return STORM_OK;
}

int32_t storm_rollout_update(storm_ctx ctx, float *d_mean, float *d_sigma2, float *d_cmd, int32_t shift,
                             void *stream)
{
    if (!ctx || !d_cmd) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    if (!ctx->pending) return STORM_E_STATE;
    const hipError_t e = storm::launch_update(ctx->P, d_mean, d_sigma2, d_cmd, shift != 0,
                                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    ctx->pending = false;
    return STORM_OK;
}

int32_t storm_rollout_set_ball(storm_ctx ctx, const float *d_ball, void *stream)
{
    if (!ctx || !d_ball) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    const hipError_t e = hipMemcpyAsync(ctx->P.ball, d_ball, sizeof(float) * 6, hipMemcpyDeviceToDevice,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_rollout_destroy(storm_ctx ctx)
{
    if (!ctx) return STORM_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_all(ctx);
    (void)hipSetDevice(prev);
    delete ctx;
    return STORM_OK;
}

int32_t storm_rollout_status(storm_ctx ctx, uint32_t *h_flags, void *stream)
{
    if (!ctx || !h_flags) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, ctx->P.status, sizeof(v), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const uint32_t zero = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->P.status, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    *h_flags = v;
    return STORM_OK;
}

int32_t storm_rollout_get_state(storm_ctx ctx, float *h_mean, float *h_sigma2, uint32_t *h_step, void *stream)
{
    if (!ctx) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (h_mean)
        e = hipMemcpyAsync(h_mean, ctx->P.mean, sizeof(float) * ctx->P.H * STORM_DOF, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && h_sigma2)
        e = hipMemcpyAsync(h_sigma2, ctx->P.sigma2, sizeof(float) * n_sigma2(ctx->P), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && h_step) e = hipMemcpyAsync(h_step, ctx->P.step, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_rollout_set_state(storm_ctx ctx, const float *h_mean, const float *h_sigma2, const uint32_t *h_step,
                                void *stream)
{
    if (!ctx) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    if (h_mean)
        for (int k = 0; k < ctx->P.H * STORM_DOF; ++k)
            if (!finite_f(h_mean[k])) return STORM_E_PARAM;
    if (h_sigma2)
        for (int j = 0; j < n_sigma2(ctx->P); ++j)
            if (!finite_f(h_sigma2[j]) || h_sigma2[j] < 0.0f) return STORM_E_PARAM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (h_mean)
        e = hipMemcpyAsync(ctx->P.mean, h_mean, sizeof(float) * ctx->P.H * STORM_DOF, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && h_sigma2)
        e = hipMemcpyAsync(ctx->P.sigma2, h_sigma2, sizeof(float) * n_sigma2(ctx->P), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && h_step) e = hipMemcpyAsync(ctx->P.step, h_step, sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    ctx->pending = false;
    return STORM_OK;
}

namespace {
constexpr uint32_t kDiffMask = STORM_COST_POSE | STORM_COST_JOINT | STORM_COST_VEL | STORM_COST_STOP;

hipError_t enqueue_refine(storm_ctx ctx, const float *d_x0, const float *d_goal, int iterations, float lr,
                          float *d_cmd, int shift, hipStream_t s)
{
    hipError_t e = hipSuccess;
    // each launch: adjoint, then the reduction with Adam step `it` fused; the
    // last also writes the command and the shift
    for (int it = 1; e == hipSuccess && it <= iterations; ++it)
        e = storm::launch_grad(ctx->P, ctx->R, d_x0, d_goal, ctx->P.mean, nullptr, nullptr, nullptr, it, lr,
                               it == iterations ? d_cmd : nullptr, shift, s);
    if (e == hipSuccess && iterations == 0) e = storm::launch_command(ctx->P, d_cmd, shift, s);
    return e;
}

int32_t create_graph(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd, int32_t iterations,
                     int32_t shift, int32_t refine_iters, float lr, void *stream, storm_graph *out)
{
    if (!out) return STORM_E_NULL;
    *out = nullptr;
    if (!ctx || !d_x0 || !d_goal || !d_cmd) return STORM_E_NULL;
    if (iterations < 1 || refine_iters < 0) return STORM_E_RANGE;
    if (refine_iters > 0 && (!(lr >= 0.0f) || !isfinite(lr))) return STORM_E_PARAM;
    if (refine_iters > 0 && (ctx->P.grad_mask & ~kDiffMask)) return STORM_E_UNSUPPORTED;
    if (ctx->error != STORM_OK) return ctx->error;
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
    g->error = &ctx->error;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    StepOut none{};
    for (int k = 0; e == hipSuccess && k < iterations; ++k) {
        const bool last = k == iterations - 1;
        e = enqueue_rollout(ctx, d_x0, d_goal, nullptr, none, s);
        if (e == hipSuccess)
            e = storm::launch_update(ctx->P, nullptr, nullptr, d_cmd, last && shift != 0 && refine_iters == 0, s);
    }
    if (e == hipSuccess && refine_iters > 0) e = enqueue_refine(ctx, d_x0, d_goal, refine_iters, lr, d_cmd, shift, s);
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
}  // namespace

int32_t storm_rollout_control(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd,
                              int32_t iterations, int32_t shift, void *stream)
{
    if (!ctx || !d_x0 || !d_goal || !d_cmd) return STORM_E_NULL;
    if (iterations < 1) return STORM_E_RANGE;
    if (ctx->error != STORM_OK) return ctx->error;
    hipStream_t s = static_cast<hipStream_t>(stream);
    StepOut none{};
    hipError_t e = hipSuccess;
    for (int k = 0; e == hipSuccess && k < iterations; ++k) {
        e = enqueue_rollout(ctx, d_x0, d_goal, nullptr, none, s);
        if (e == hipSuccess)
            e = storm::launch_update(ctx->P, nullptr, nullptr, d_cmd, k == iterations - 1 && shift != 0, s);
    }
    if (e != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    ctx->pending = false;
    return STORM_OK;
}

int32_t storm_rollout_graph_create(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd,
                                   int32_t iterations, int32_t shift, void *stream, storm_graph *out)
{
    return create_graph(ctx, d_x0, d_goal, d_cmd, iterations, shift, 0, 0.0f, stream, out);
}

int32_t storm_rollout_graph_create_refine(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd,
                                          int32_t iterations, int32_t shift, int32_t refine_iters, float lr,
                                          void *stream, storm_graph *out)
{
    return create_graph(ctx, d_x0, d_goal, d_cmd, iterations, shift, refine_iters, lr, stream, out);
}

int32_t storm_rollout_grad(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_mean,
                           const float *d_noise, float *d_grad, float *d_J, void *stream)
{
    if (!ctx || !d_x0 || !d_goal || !d_mean) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    if (ctx->P.grad_mask & ~kDiffMask) return STORM_E_UNSUPPORTED;
    if (storm::launch_grad(ctx->P, ctx->R, d_x0, d_goal, d_mean, d_noise, d_grad, d_J, 0, 0.0f, nullptr, 0,
                           static_cast<hipStream_t>(stream)) != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_rollout_grad_noalloc(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_mean,
                                   const float *d_noise, float *d_grad, float *d_J, void *stream)
{
    if (!ctx || !d_x0 || !d_goal || !d_mean) return STORM_E_NULL;
    if (ctx->error != STORM_OK) return ctx->error;
    if (ctx->P.grad_mask & ~kDiffMask) return STORM_E_UNSUPPORTED;
    ProblemDev P = ctx->P;
    const size_t chunks = (size_t)(P.n_tiles < kAdjChunks ? P.n_tiles : kAdjChunks);
    if (chunks * STORM_DOF * kMaxH > kNoallocGradFloats || P.H > kMaxH) return STORM_E_RANGE;
    // the partials go to this device's static scratch instead of the
    // context's own buffers; everything else is the context's
    P.grad_part = ctx->scratch;
    P.cost_part = ctx->scratch + kNoallocGradFloats;
    if (storm::launch_grad(P, ctx->R, d_x0, d_goal, d_mean, d_noise, d_grad, d_J, 0, 0.0f, nullptr, 0,
                           static_cast<hipStream_t>(stream)) != hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_rollout_refine(storm_ctx ctx, const float *d_x0, const float *d_goal, int32_t iterations, float lr,
                             float *d_cmd, int32_t shift, void *stream)
{
    if (!ctx || !d_x0 || !d_goal || !d_cmd) return STORM_E_NULL;
    if (iterations < 0) return STORM_E_RANGE;
    if (!(lr >= 0.0f) || !isfinite(lr)) return STORM_E_PARAM;
    if (ctx->error != STORM_OK) return ctx->error;
    if (ctx->P.grad_mask & ~kDiffMask) return STORM_E_UNSUPPORTED;
    if (enqueue_refine(ctx, d_x0, d_goal, iterations, lr, d_cmd, shift != 0, static_cast<hipStream_t>(stream)) !=
        hipSuccess) {
        ctx->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_rollout_graph_launch(storm_graph graph, void *stream)
{
    if (!graph) return STORM_E_NULL;
    if (*graph->error != STORM_OK) return *graph->error;
    if (hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)) != hipSuccess) {
        *graph->error = STORM_E_DEVICE;
        return STORM_E_DEVICE;
    }
    return STORM_OK;
}

int32_t storm_rollout_graph_destroy(storm_graph graph)
{
    if (!graph) return STORM_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return STORM_OK;
}

int32_t storm_fk(const storm_robot *robot, const float *d_q, int32_t n, float *d_pose, float *d_manip, void *stream)
{
    if (!robot) return STORM_E_NULL;
    if (n < 0) return STORM_E_RANGE;
    if (n > 0 && (!d_q || !d_pose)) return STORM_E_NULL;
    for (int k = 0; k < STORM_NFRAMES; ++k)
        for (int c = 0; c < 3; ++c)
            if (!finite_f(robot->dh[k][c])) return STORM_E_PARAM;
    RobotDev R{};
    fill_robot_consts(robot, R);
    R.n_spheres = 0;
    const hipError_t e = storm::launch_fk(R, d_q, n, d_pose, d_manip, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? STORM_OK : STORM_E_DEVICE;
}

}  // extern "C"
