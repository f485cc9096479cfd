// Init-time kernels: per-problem constant tables, the Halton + B-spline noise
// table (Sec. 3.3) and the device form of the robot and scene records.
// These run once per context; they are computed in FP64 and rounded to the
// FP32 the step uses.
#include "storm_internal.h"

namespace storm {
namespace {

// Tables: dt, stop-cost velocity limit (Eq. 10: max acceleration times the
// time left to the end of the horizon, step h included), horizon weights
// (Eq. 2: gamma^h, terminal step scaled by w_term), band-shrunk position and
// velocity limits (Eq. 11), initial mean 0 and variance sigma_init^2.
__global__ void tables_kernel(ProblemDev P, float *tables, const float *dt_raw, const float *lim_raw, float acc_stop,
                              float gamma, float w_term, float k_jl, float k_vl, const float *sigma_init, float c1,
                              float c2, float c3)
{
    const int t = threadIdx.x;
    const int H = P.H;
    if (t < H && P.cov_step)
        for (int j = 0; j < kDof; ++j) P.sigma2[t * kDof + j] = (float)((double)sigma_init[j] * sigma_init[j]);
    if (t < H) {
        double rem = 0.0;
        for (int k = t; k < H; ++k) rem += (double)dt_raw[k];
        tables[kTabDt + t] = dt_raw[t];
        tables[kTabVstop + t] = (float)((double)acc_stop * rem);
        double w = pow((double)gamma, (double)t);
        if (t == H - 1) w *= (double)w_term;
        tables[kTabHw + t] = (float)w;
        for (int j = 0; j < kDof; ++j) P.mean[t * kDof + j] = 0.0f;
    }
    if (t < kDof) {
        const double lo = lim_raw[t], hi = lim_raw[kDof + t], vm = lim_raw[2 * kDof + t];
        tables[kTabJlo + t] = (float)(lo + (double)k_jl * (hi - lo));
        tables[kTabJhi + t] = (float)(hi - (double)k_jl * (hi - lo));
        tables[kTabVlo + t] = (float)(-vm + (double)k_vl * 2.0 * vm);
        tables[kTabVhi + t] = (float)(vm - (double)k_vl * 2.0 * vm);
        const double s = sigma_init[t];
        tables[kTabSig0 + t] = (float)(s * s);
        if (!P.cov_step) P.sigma2[t] = (float)(s * s);
    }
    if (t < 8) P.ball[t] = 0.0f;  // no ball state until storm_rollout_set_ball
    if (t == 0) {
        *P.step = 0u;
        *P.status = 0u;
        *P.last_step = 0u;
        // comb filter (Sec. 3.3) as a convolution: e'_h = sum_{k <= h} g_k e_{h-k}
        // with g_k = c1 r_k, r the impulse response of r_k = c2 r_{k-1} + c3 r_{k-2}
        // (zero past H: the kernels read the response in batches of eight)
        double r1 = 0.0, r2 = 0.0;
        for (int k = 0; k < kMaxH; ++k) {
            const double r = k == 0 ? 1.0 : (double)c2 * r1 + (double)c3 * r2;
            tables[kTabComb + k] = k < H ? (float)((double)c1 * r) : 0.0f;
            r2 = r1;
            r1 = r;
        }
    }
}

// Geometry records in device form, one flat index space over all of them.
//   sphere obstacles: (centre, radius)
//   all obstacles:    the culling ball (centre, bounding radius + margin)
//   cuboids:          the world-to-box map l = M x + t with M = R^T,
//                     t = -R^T c, then the half extents
//   body spheres:     (local centre, radius) and the frame index
__global__ void geometry_kernel(const float *sph_obs_raw, int n_so, const float *box_raw, int n_bo,
                                float4 *sph_obs, float *box_obs, float4 *obs_bound, const float *sph_raw, int S,
                                float4 *sph_local, int32_t *sph_body)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_so) {
        const float *r = sph_obs_raw + t * STORM_OBSTACLE_STRIDE;
        sph_obs[t] = make_float4(r[1], r[2], r[3], r[4]);
    }
    if (t < n_so + n_bo) {
        // culling record: the obstacle lies inside the ball (centre, radius);
        // a cuboid's ball has the radius of its half-extent diagonal.  The
        // 1e-4 m margin dwarfs the FP32 rounding of any distance the cull or
        // the exact tests form, so no contact the exact tests would report is
        // ever culled.
        const bool sphere = t < n_so;
        const float *r = sphere ? sph_obs_raw + t * STORM_OBSTACLE_STRIDE
                                : box_raw + (t - n_so) * STORM_OBSTACLE_STRIDE;
        const double rad = sphere ? (double)r[4]
                                  : sqrt((double)r[4] * r[4] + (double)r[5] * r[5] + (double)r[6] * r[6]);
        obs_bound[t] = make_float4(r[1], r[2], r[3], (float)(rad + 1e-4));
    }
    if (t < n_bo) {
        const float *r = box_raw + t * STORM_OBSTACLE_STRIDE;
        float *b = box_obs + 16 * t;
        const float *Rw = r + 7;
        for (int row = 0; row < 3; ++row) {
            double tt = 0.0;
            for (int c = 0; c < 3; ++c) {
                b[row * 3 + c] = Rw[c * 3 + row];
                tt -= (double)Rw[c * 3 + row] * (double)r[1 + c];
            }
            b[9 + row] = (float)tt;
            b[12 + row] = r[4 + row];
        }
        b[15] = 0.0f;
    }
    if (t < S) {
        const float *q = sph_raw + t * 5;
        sph_local[t] = make_float4(q[1], q[2], q[3], q[4]);
        sph_body[t] = (int32_t)q[0] - 1;
    }
}

// Inverse standard normal CDF by Newton's method in FP64, started at the
// inflection point x = 0 so that it converges monotonically; the residual of
// each tail is formed with erfc so that small tail probabilities keep their
// relative accuracy.
__device__ double inverse_normal_cdf(double p)
{
    const double inv_sqrt_2pi = 0.39894228040143267794;
    const bool upper = p > 0.5;
    const double target = upper ? 1.0 - p : p;
    double x = 0.0;
    for (int it = 0; it < 100; ++it) {
        // tail(x) = P(Z < x) for the lower branch, P(Z > -x) mirrored for the upper one
        const double tail = 0.5 * erfc((upper ? x : -x) * 0.70710678118654752440);
        const double dens = inv_sqrt_2pi * exp(-0.5 * x * x);
        const double f = upper ? (target - tail) : (tail - target);
        const double dx = f / dens;
        x -= dx;
        if (fabs(dx) <= 1e-15 * fmax(1.0, fabs(x))) break;
    }
    return x;
}

// Z[i][k][j] = inverse-CDF of the radical inverse of Halton index 1 + i K + k
// in the base of the j-th prime.
__global__ void halton_points_kernel(int n_halton, int K, double *Z)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = n_halton * K * kDof;
    if (t >= total) return;
    const int j = t % kDof;
    const int k = (t / kDof) % K;
    const int i = t / (kDof * K);
    const unsigned primes[kDof] = {2u, 3u, 5u, 7u, 11u, 13u, 17u};
    const unsigned b = primes[j];
    unsigned long long idx = 1ull + (unsigned long long)i * (unsigned long long)K + (unsigned long long)k;
    double v = 0.0, scale = 1.0 / (double)b;
    while (idx > 0ull) {
        v += scale * (double)(idx % b);
        idx /= b;
        scale /= (double)b;
    }
    Z[t] = inverse_normal_cdf(v);
}

// Knot t_m of the clamped uniform cubic knot vector for K control points.
__device__ double clamped_knot(int K, int m)
{
    if (m <= 3) return 0.0;
    if (m >= K) return 1.0;
    return (double)(m - 3) / (double)(K - 3);
}

// eps[j][i][h] = sum_k B_k(s_h) Z[i][k][j], s_h = h / (H - 1): the K
// Gaussianised Halton values of each joint are the control points of a
// clamped cubic B-spline sampled at the H horizon steps.  The four non-zero
// basis functions of the knot span are evaluated with the triangular
// recurrence of de Boor (Piegl and Tiller, The NURBS Book, Alg. A2.2).
__global__ void halton_smooth_kernel(int n_halton, int K, int H, const double *Z, float *eps)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = kDof * n_halton * H;
    if (t >= total) return;
    const int h = t % H;
    const int i = (t / H) % n_halton;
    const int j = t / (H * n_halton);
    const double s = H > 1 ? (double)h / (double)(H - 1) : 0.0;
    int span = 3 + (int)floor(s * (double)(K - 3));
    if (span > K - 1) span = K - 1;
    double Nb[4], left[4], right[4];
    Nb[0] = 1.0;
    for (int d = 1; d <= 3; ++d) {
        left[d] = s - clamped_knot(K, span + 1 - d);
        right[d] = clamped_knot(K, span + d) - s;
        double saved = 0.0;
        for (int r = 0; r < d; ++r) {
            const double tmp = Nb[r] / (right[r + 1] + left[d - r]);
            Nb[r] = saved + right[r + 1] * tmp;
            saved = left[d - r] * tmp;
        }
        Nb[d] = saved;
    }
    double acc = 0.0;
    for (int r = 0; r < 4; ++r) acc += Nb[r] * Z[((size_t)i * K + (span - 3 + r)) * kDof + j];
    eps[t] = (float)acc;
}

}  // namespace

hipError_t launch_init_tables(const ProblemDev &P, const float *d_dt_raw, const float *d_lim_raw, float acc_stop,
                              float gamma, float w_term, float k_jl, float k_vl, const float *d_sigma_init,
                              const float comb[3], int n_knots, const float *d_obs_raw, int n_obs, float4 *d_sph_obs, float *d_box_obs,
                              float4 *d_obs_bound, const float *d_sph_raw, int n_spheres, float4 *d_sph_local,
                              int32_t *d_sph_body, hipStream_t stream)
{
    (void)n_obs;
    hipLaunchKernelGGL(tables_kernel, dim3(1), dim3(kMaxH), 0, stream, P, const_cast<float *>(P.tables), d_dt_raw,
                       d_lim_raw, acc_stop, gamma, w_term, k_jl, k_vl, d_sigma_init, comb[0], comb[1], comb[2]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // d_obs_raw holds the sphere records first, then the cuboid records
    const int S = n_spheres, n_so = P.n_sph_obs, n_bo = P.n_box_obs;
    int ng = S;
    if (n_so + n_bo > ng) ng = n_so + n_bo;
    const int gthreads = 256;
    const int gblocks = ng > 0 ? (ng + gthreads - 1) / gthreads : 1;
    hipLaunchKernelGGL(geometry_kernel, dim3(gblocks), dim3(gthreads), 0, stream, d_obs_raw, n_so,
                       d_obs_raw + (size_t)STORM_OBSTACLE_STRIDE * n_so, n_bo, d_sph_obs, d_box_obs, d_obs_bound,
                       d_sph_raw, S, d_sph_local, d_sph_body);
    e = hipGetLastError();
    if (e != hipSuccess || P.n_halton == 0) return e;
    double *Z = nullptr;
    const size_t nz = (size_t)P.n_halton * n_knots * kDof;
    e = hipMalloc((void **)&Z, nz * sizeof(double));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(halton_points_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, stream, P.n_halton,
                       n_knots, Z);
    e = hipGetLastError();
    if (e == hipSuccess) {
        const size_t ne = (size_t)kDof * P.n_halton * P.H;
        hipLaunchKernelGGL(halton_smooth_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, stream,
                           P.n_halton, n_knots, P.H, Z, const_cast<float *>(P.halton));
        e = hipGetLastError();
    }
    const hipError_t sync = hipStreamSynchronize(stream);
    const hipError_t f = hipFree(Z);
    if (e != hipSuccess) return e;
    return sync != hipSuccess ? sync : f;
}

}  // namespace storm
