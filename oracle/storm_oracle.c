/*
 * storm_oracle.c - plain, slow FP64 CPU oracle of one STORM MPC iteration
 * (STORM: a tensorised sampling-based MPC for manipulators, arXiv 2104.13542).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
 * leg of the benchmark are the only code allowed to load this library; the
 * product path never does.  It shares no code, header or table with the HIP
 * library: both sides receive the same robot, scene and noise as plain data.
 *
 * Each step is written out as the paper states it, in double precision, with
 * no blocking, fusion or reordering:
 *   sampling        Sec. 3.3 (Halton sequence, cubic B-spline smoothing,
 *                   per-joint covariance, null particles, comb filter) plus
 *                   Gaussian noise
 *   integrator      Sec. 3.1, Eq. 7
 *   kinematics      Sec. 3.1, Eq. 8 (FK and geometric Jacobian)
 *   running cost    Sec. 3.2, Eq. 9-15
 *   horizon cost    Sec. 3, Eq. 2
 *   update          Sec. 3, Eq. 4-6, followed by next command and shift (Alg. 1)
 *   gradient        reverse pass of the expected horizon cost with respect to
 *                   the mean (not in the paper; an added differentiable form)
 *
 * Readings of points the paper leaves open are listed with each function.
 * Parity status: every function here is pinned by a CPU test against closed
 * forms, library routines or brute force, except the composition of the whole
 * step, which the paper gives no worked example for (parity unpinned as a
 * whole; pinned through its parts).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DOF 7
#define NFRAMES 8
#define OBS_STRIDE 16

#define MASK_POSE (1u << 0)
#define MASK_JOINT (1u << 1)
#define MASK_VEL (1u << 2)
#define MASK_STOP (1u << 3)
#define MASK_MANIP (1u << 4)
#define MASK_SELF (1u << 5)
#define MASK_ENV (1u << 6)
#define MASK_BALL (1u << 7)

/* Number of per-step cost terms reported: pos, rot, joint, vel, stop, manip,
 * self, env, ball (all unweighted). */
#define NTERMS 9

typedef struct {
    int32_t n;        /* particles N */
    int32_t h;        /* horizon H */
    int32_t n_halton; /* particles [0, n_halton) use Halton + B-spline noise */
    int32_t n_null;   /* particles [N - n_null, N) are zero-acceleration */
    int32_t n_knots;  /* B-spline control points K */
    int32_t pad0;
    uint64_t seed;
    double beta, gamma, alpha_mu, alpha_sigma, w_term, sigma2_min;
    double acc_stop, k_jl, k_vl, k_m;
    double w_pos, w_rot;
    double alpha_pos[3], alpha_rot[3];
    double a_stop, a_joint, a_vel, a_manip, a_coll;
    uint32_t cost_mask;
    int32_t comb_filter; /* 1: comb-filter the Gaussian particles' noise (Sec. 3.3) */
    double comb[3];      /* c1, c2, c3 */
    int32_t cov_per_step; /* 1: Eq. 5 per step: sigma2 is [H][7], shifted with sigma_init2 appended */
    int32_t pad2;
    double sigma_init2[DOF]; /* the value a per-step shift appends */
    /* ball on the tray (appendix on dynamic object balancing) */
    double w_ball;           /* weight of the ball term */
    double ball_gravity[3];  /* g in the world frame */
    double ball_center[2];   /* tray centre in the flange frame (x, y) */
    double ball[6];          /* ball position and velocity in the world frame at the current state */
    int32_t self_model;      /* 0: sphere pairs; 1: the learned self-collision network (jointNERF form) */
    int32_t pad3;
} oracle_params;

typedef struct {
    double dh[NFRAMES][3]; /* (a_{k-1}, d_k, alpha_{k-1}) for frames 1..8 */
    double q_min[DOF], q_max[DOF], qd_max[DOF];
    int32_t n_spheres, pad0;
    const double *spheres; /* [S][5]: body (1..8), x, y, z, r in the body frame */
    int32_t n_obstacles, pad1;
    const double *obstacles; /* [O][16]: kind, centre, extents, R (row-major) */
    const double *self_mlp;  /* the network's parameters (oracle_self_mlp), or NULL */
} oracle_model;

/* ------------------------------------------------------------------------ */
/* Counter-based Gaussian noise.                                             */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplies, with a Weyl-sequence key schedule. */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Box-Muller (1958) on 24-bit uniforms: u1 = (x0 >> 8 + 1) 2^-24 in (0, 1],
 * u2 = (x1 >> 8) 2^-24 in [0, 1); returns the cosine and sine normals. */
static void box_muller(uint32_t x0, uint32_t x1, double *z_cos, double *z_sin)
{
    double u1 = ((double)(x0 >> 8) + 1.0) * ldexp(1.0, -24);
    double u2 = (double)(x1 >> 8) * ldexp(1.0, -24);
    double r = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    *z_cos = r * cos(ang);
    *z_sin = r * sin(ang);
}

/* Standard normals for particle i, horizon step h, control step `step`.
 * Two Philox calls with counter (i, h, k, step), k = 0, 1, key = the 64-bit
 * seed split into words; each call gives four normals, joints 4k..4k+3
 * (the eighth normal is unused). */
void oracle_gauss7(uint64_t seed, uint32_t step, uint32_t i, uint32_t h, double eps[DOF])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double z[8];
    for (uint32_t k = 0; k < 2; ++k) {
        uint32_t ctr[4] = {i, h, k, step}, x[4];
        oracle_philox4x32_10(ctr, key, x);
        box_muller(x[0], x[1], &z[4 * k + 0], &z[4 * k + 1]);
        box_muller(x[2], x[3], &z[4 * k + 2], &z[4 * k + 3]);
    }
    for (int j = 0; j < DOF; ++j) eps[j] = z[j];
}

/* ------------------------------------------------------------------------ */
/* Halton + B-spline noise (Sec. 3.3).                                       */
/* ------------------------------------------------------------------------ */

/* Radical inverse phi_b(i) = sum_a i_a b^{-a} of the base-b digits of i. */
double oracle_radical_inverse(uint64_t i, uint32_t b)
{
    double r = 0.0, f = 1.0;
    while (i > 0) {
        f /= (double)b;
        r += f * (double)(i % b);
        i /= b;
    }
    return r;
}

/* Standard normal CDF through libm's complementary error function. */
double oracle_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Inverse normal CDF by bisection to double resolution.  Slow and plain on
 * purpose.  Above p = 1/2 the upper tail 1 - Phi(x) = erfc(x / sqrt 2) / 2 is
 * matched against 1 - p (exact in double there), so both tails keep full
 * relative accuracy. */
double oracle_ndtri(double p)
{
    if (!(p > 0.0 && p < 1.0)) return NAN;
    int upper = p > 0.5;
    double target = upper ? 1.0 - p : p;
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 4000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double f = upper ? 0.5 * erfc(mid / sqrt(2.0)) : oracle_normal_cdf(mid);
        int go_right = upper ? (f > target) : (f < target);
        if (go_right)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Clamped uniform knot vector for K control points of a cubic: four zeros,
 * K - 4 interior knots j / (K - 3), four ones. */
static double knot(int K, int idx)
{
    if (idx <= 3) return 0.0;
    if (idx >= K) return 1.0;
    return (double)(idx - 3) / (double)(K - 3);
}

/* Cox-de Boor recursion for B-spline basis N_{i,p}(s) on the clamped uniform
 * knot vector above; the right end of the parameter range belongs to the
 * last non-empty span. */
static double cox_de_boor(int K, int i, int p, double s)
{
    if (p == 0) {
        double t0 = knot(K, i), t1 = knot(K, i + 1);
        if (t0 <= s && s < t1) return 1.0;
        /* s = 1: the last non-degenerate span [t_{K-1}, t_K] is closed. */
        if (s == 1.0 && t1 == 1.0 && t0 < 1.0) return 1.0;
        return 0.0;
    }
    double r = 0.0;
    double d0 = knot(K, i + p) - knot(K, i);
    double d1 = knot(K, i + p + 1) - knot(K, i + 1);
    if (d0 > 0.0) r += (s - knot(K, i)) / d0 * cox_de_boor(K, i, p - 1, s);
    if (d1 > 0.0) r += (knot(K, i + p + 1) - s) / d1 * cox_de_boor(K, i + 1, p - 1, s);
    return r;
}

/* B[h][k]: cubic B-spline basis function k of K control points evaluated at
 * s_h = h / (H - 1) (s_0 = 0 when H = 1).  The paper fits a degree-3 B-spline
 * to the Halton samples and sub-samples it at the horizon resolution; here
 * the K Gaussianised Halton values per joint are the control points. */
int oracle_bspline_basis(int H, int K, double *B)
{
    if (H < 1 || K < 4) return -1;
    for (int h = 0; h < H; ++h) {
        double s = H == 1 ? 0.0 : (double)h / (double)(H - 1);
        for (int k = 0; k < K; ++k) B[h * K + k] = cox_de_boor(K, k, 3, s);
    }
    return 0;
}

static const uint32_t kPrimes[DOF] = {2, 3, 5, 7, 11, 13, 17};

/* Halton noise of particle i, row[h][j]: Halton point index 1 + i K + k in
 * dimension j (prime p_j), mapped to a standard normal by the inverse CDF,
 * then smoothed by the B-spline basis B [H][K] over k.  Index 0 (the origin)
 * is skipped.  Z is scratch of K x 7. */
static void halton_row(int i, int H, int K, const double *B, double *Z, double *row)
{
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < DOF; ++j)
            Z[k * DOF + j] = oracle_ndtri(oracle_radical_inverse((uint64_t)1 + (uint64_t)i * K + k, kPrimes[j]));
    for (int h = 0; h < H; ++h)
        for (int j = 0; j < DOF; ++j) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += B[h * K + k] * Z[k * DOF + j];
            row[(size_t)h * DOF + j] = acc;
        }
}

/* Halton noise table eps[i][h][j], i < n_halton (halton_row of every
 * particle).  Drawn once; the same table is used at every step. */
int oracle_halton_noise(int n_halton, int H, int K, double *eps)
{
    double *B = (double *)malloc(sizeof(double) * (size_t)H * (size_t)K);
    double *Z = (double *)malloc(sizeof(double) * (size_t)K * DOF);
    if (!B || !Z || oracle_bspline_basis(H, K, B) != 0) {
        free(B);
        free(Z);
        return -1;
    }
    for (int i = 0; i < n_halton; ++i) halton_row(i, H, K, B, Z, eps + (size_t)i * H * DOF);
    free(B);
    free(Z);
    return 0;
}

/* Comb filter (Sec. 3.3) of one joint's noise sequence x_0 .. x_{H-1}
 * (stride DOF), applied in step order and in place, so that the earlier
 * terms are already filtered: x'_h = c1 x_h + c2 x'_{h-1} + c3 x'_{h-2} with
 * x'_{-1} = x'_{-2} = 0.  The paper prints the third term with the index of
 * the second; it is read as the step before that. */
static void comb_filter(int H, const double c[3], double *x)
{
    double p1 = 0.0, p2 = 0.0;
    for (int h = 0; h < H; ++h) {
        const double y = c[0] * x[(size_t)h * DOF] + c[1] * p1 + c[2] * p2;
        x[(size_t)h * DOF] = y;
        p2 = p1;
        p1 = y;
    }
}

/* Full standard-noise tensor eps[N][H][7] for control step `step`: Halton
 * particles first, then Gaussian particles (comb-filtered when enabled),
 * then null particles (zero). */
int oracle_noise(const oracle_params *p, uint32_t step, double *eps)
{
    int N = p->n, H = p->h;
    if (p->n_halton > 0) {
        if (oracle_halton_noise(p->n_halton, H, p->n_knots, eps) != 0) return -1;
    }
    for (int i = p->n_halton; i < N; ++i)
        for (int h = 0; h < H; ++h) {
            double *e = eps + ((size_t)i * H + h) * DOF;
            if (i >= N - p->n_null)
                for (int j = 0; j < DOF; ++j) e[j] = 0.0;
            else
                oracle_gauss7(p->seed, step, (uint32_t)i, (uint32_t)h, e);
        }
    if (p->comb_filter)
        for (int i = p->n_halton; i < N - p->n_null; ++i)
            for (int j = 0; j < DOF; ++j) comb_filter(H, p->comb, eps + (size_t)i * H * DOF + j);
    return 0;
}

/* The rows of oracle_noise for the particles idx[0 .. n_idx) only (any order,
 * each in 0 .. N-1): eps[m][H][7] is particle idx[m]'s noise, so that a few
 * particles of a large problem can be checked without the whole tensor. */
int oracle_noise_particles(const oracle_params *p, uint32_t step, const int32_t *idx, int n_idx, double *eps)
{
    int N = p->n, H = p->h, K = p->n_knots;
    double *B = NULL, *Z = NULL;
    if (p->n_halton > 0) {
        B = (double *)malloc(sizeof(double) * (size_t)H * (size_t)K);
        Z = (double *)malloc(sizeof(double) * (size_t)K * DOF);
        if (!B || !Z || oracle_bspline_basis(H, K, B) != 0) {
            free(B);
            free(Z);
            return -1;
        }
    }
    int rc = 0;
    for (int m = 0; m < n_idx && rc == 0; ++m) {
        const int i = idx[m];
        double *row = eps + (size_t)m * H * DOF;
        if (i < 0 || i >= N) {
            rc = -1;
        } else if (i < p->n_halton) {
            halton_row(i, H, K, B, Z, row);
        } else if (i >= N - p->n_null) {
            for (int k = 0; k < H * DOF; ++k) row[k] = 0.0;
        } else {
            for (int h = 0; h < H; ++h) oracle_gauss7(p->seed, step, (uint32_t)i, (uint32_t)h, row + (size_t)h * DOF);
            if (p->comb_filter)
                for (int j = 0; j < DOF; ++j) comb_filter(H, p->comb, row + j);
        }
    }
    free(B);
    free(Z);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Integrator (Sec. 3.1, Eq. 7).                                             */
/* ------------------------------------------------------------------------ */

/* Acceleration = control; velocity = v0 + S_l(1) diag(dt) acceleration;
 * position = q0 + S_l(1) diag(dt) velocity.  S_l(1) is lower triangular with
 * ones on and below the diagonal, so step h already includes its own dt_h.
 * The prefix sums are written as the sums they are. */
void oracle_integrate(int H, const double *dt, const double q0[DOF], const double v0[DOF], const double *u,
                      double *q, double *v, double *a)
{
    for (int h = 0; h < H; ++h)
        for (int j = 0; j < DOF; ++j) {
            double sv = 0.0;
            for (int k = 0; k <= h; ++k) sv += dt[k] * u[k * DOF + j];
            v[h * DOF + j] = v0[j] + sv;
            a[h * DOF + j] = u[h * DOF + j];
        }
    for (int h = 0; h < H; ++h)
        for (int j = 0; j < DOF; ++j) {
            double sq = 0.0;
            for (int k = 0; k <= h; ++k) sq += dt[k] * v[k * DOF + j];
            q[h * DOF + j] = q0[j] + sq;
        }
}

/* ------------------------------------------------------------------------ */
/* Kinematics (Sec. 3.1, Eq. 8).                                             */
/* ------------------------------------------------------------------------ */

static void mat4_mul(const double A[16], const double B[16], double C[16])
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[r * 4 + k] * B[k * 4 + c];
            C[r * 4 + c] = s;
        }
}

static void mat4_identity(double A[16])
{
    memset(A, 0, sizeof(double) * 16);
    A[0] = A[5] = A[10] = A[15] = 1.0;
}

/* Frames T_1..T_8 (row-major 4x4, base frame = world):
 * T_k = T_{k-1} RotX(alpha_{k-1}) TransX(a_{k-1}) RotZ(theta_k) TransZ(d_k),
 * theta_k = q_k for the seven joints and 0 for the flange frame 8. */
void oracle_fk(const double dh[NFRAMES][3], const double q[DOF], double T[NFRAMES][16])
{
    double prev[16], A[16], B[16], M[16];
    mat4_identity(prev);
    for (int k = 0; k < NFRAMES; ++k) {
        double a = dh[k][0], d = dh[k][1], al = dh[k][2];
        double th = k < DOF ? q[k] : 0.0;
        double rx[16], tx[16], rz[16], tz[16];
        mat4_identity(rx);
        rx[5] = cos(al);
        rx[6] = -sin(al);
        rx[9] = sin(al);
        rx[10] = cos(al);
        mat4_identity(tx);
        tx[3] = a;
        mat4_identity(rz);
        rz[0] = cos(th);
        rz[1] = -sin(th);
        rz[4] = sin(th);
        rz[5] = cos(th);
        mat4_identity(tz);
        tz[11] = d;
        mat4_mul(rx, tx, A);
        mat4_mul(A, rz, B);
        mat4_mul(B, tz, M);
        mat4_mul(prev, M, T[k]);
        memcpy(prev, T[k], sizeof(prev));
    }
}

/* Geometric Jacobian of the flange origin, 6 x 7 (rows: linear x, y, z, then
 * angular x, y, z).  Joint k turns about the z axis of frame k through that
 * frame's origin: column k = [z_k x (p_ee - o_k); z_k]. */
void oracle_jacobian(const double T[NFRAMES][16], double J[6][DOF])
{
    const double *E = T[NFRAMES - 1];
    double pe[3] = {E[3], E[7], E[11]};
    for (int k = 0; k < DOF; ++k) {
        const double *F = T[k];
        double z[3] = {F[2], F[6], F[10]};
        double o[3] = {F[3], F[7], F[11]};
        double r[3] = {pe[0] - o[0], pe[1] - o[1], pe[2] - o[2]};
        J[0][k] = z[1] * r[2] - z[2] * r[1];
        J[1][k] = z[2] * r[0] - z[0] * r[2];
        J[2][k] = z[0] * r[1] - z[1] * r[0];
        J[3][k] = z[0];
        J[4][k] = z[1];
        J[5][k] = z[2];
    }
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Task-space velocity and acceleration of the flange (Eq. 8): xd = J qd and
 * xdd = Jdot qd + J qdd, rows linear x, y, z then angular x, y, z.  Jdot is
 * formed from its definition, Jdot = sum_m (dJ/dq_m) qd_m, with the partial
 * derivatives of a revolute chain: for m < k, dz_k/dq_m = z_m x z_k and
 * do_k/dq_m = z_m x (o_k - o_m) (joint m does not move frames before it, and
 * joint k turns frame k about its own z through its own origin), and
 * dp/dq_m = z_m x (p - o_m) for the flange origin p. */
void oracle_task_space(const double dh[NFRAMES][3], const double q[DOF], const double qd[DOF],
                       const double qdd[DOF], double xd[6], double xdd[6])
{
    double T[NFRAMES][16], J[6][DOF], Jd[6][DOF];
    oracle_fk(dh, q, T);
    oracle_jacobian(T, J);
    const double *E = T[NFRAMES - 1];
    double pe[3] = {E[3], E[7], E[11]};
    double z[DOF][3], o[DOF][3];
    for (int k = 0; k < DOF; ++k)
        for (int c = 0; c < 3; ++c) {
            z[k][c] = T[k][c * 4 + 2];
            o[k][c] = T[k][c * 4 + 3];
        }
    for (int r = 0; r < 6; ++r)
        for (int k = 0; k < DOF; ++k) Jd[r][k] = 0.0;
    for (int k = 0; k < DOF; ++k) {
        double rk[3] = {pe[0] - o[k][0], pe[1] - o[k][1], pe[2] - o[k][2]};
        for (int m = 0; m < DOF; ++m) {
            double dz[3] = {0.0, 0.0, 0.0}, dok[3] = {0.0, 0.0, 0.0}, dp[3];
            double rm[3] = {pe[0] - o[m][0], pe[1] - o[m][1], pe[2] - o[m][2]};
            cross3(z[m], rm, dp);
            if (m < k) {
                double okm[3] = {o[k][0] - o[m][0], o[k][1] - o[m][1], o[k][2] - o[m][2]};
                cross3(z[m], z[k], dz);
                cross3(z[m], okm, dok);
            }
            /* d/dq_m of column k: linear z_k x (p - o_k), angular z_k */
            double t1[3], t2[3], dr[3] = {dp[0] - dok[0], dp[1] - dok[1], dp[2] - dok[2]};
            cross3(dz, rk, t1);
            cross3(z[k], dr, t2);
            for (int c = 0; c < 3; ++c) {
                Jd[c][k] += (t1[c] + t2[c]) * qd[m];
                Jd[3 + c][k] += dz[c] * qd[m];
            }
        }
    }
    for (int r = 0; r < 6; ++r) {
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < DOF; ++k) {
            s1 += J[r][k] * qd[k];
            s2 += Jd[r][k] * qd[k] + J[r][k] * qdd[k];
        }
        xd[r] = s1;
        xdd[r] = s2;
    }
}

/* Ball on the tray (appendix on dynamic object balancing).  The ball's state
 * at the current arm state q0 is moved into the flange frame, x = R0^T
 * (x_w - p0) and v = R0^T v_w with its z velocity set to 0.  At step h the
 * flange rotation R_h of the rolled-out state gives the ball's acceleration
 * in the tray plane, [g_x, g_y, 0] of g_ee = R_h^T g_w, and the ball is
 * integrated with the scheme of Eq. 7: v_h = v + sum_{k<=h} dt_k a_k,
 * x_h = x + sum_{k<=h} dt_k v_k.  Writes xb[H][3]. */
void oracle_ball_traj(const oracle_params *p, const oracle_model *mdl, const double *dt, const double q0[DOF],
                      const double *q, double *xb)
{
    double T[NFRAMES][16];
    oracle_fk(mdl->dh, q0, T);
    const double *E = T[NFRAMES - 1];
    double x[3], v[3];
    for (int c = 0; c < 3; ++c) {
        x[c] = 0.0;
        v[c] = 0.0;
        for (int r = 0; r < 3; ++r) {
            x[c] += E[r * 4 + c] * (p->ball[r] - E[r * 4 + 3]);
            v[c] += E[r * 4 + c] * p->ball[3 + r];
        }
    }
    v[2] = 0.0;
    int H = p->h;
    double *a = (double *)malloc(sizeof(double) * (size_t)H * 2);
    double *vh = (double *)malloc(sizeof(double) * (size_t)H * 2);
    if (!a || !vh) {
        free(a);
        free(vh);
        for (int k = 0; k < 3 * H; ++k) xb[k] = NAN;
        return;
    }
    for (int h = 0; h < H; ++h) {
        oracle_fk(mdl->dh, q + h * DOF, T);
        E = T[NFRAMES - 1];
        for (int c = 0; c < 2; ++c) {
            a[h * 2 + c] = 0.0;
            for (int r = 0; r < 3; ++r) a[h * 2 + c] += E[r * 4 + c] * p->ball_gravity[r];
        }
    }
    for (int h = 0; h < H; ++h)
        for (int c = 0; c < 2; ++c) {
            double sv = 0.0;
            for (int k = 0; k <= h; ++k) sv += dt[k] * a[k * 2 + c];
            vh[h * 2 + c] = v[c] + sv;
        }
    for (int h = 0; h < H; ++h) {
        for (int c = 0; c < 2; ++c) {
            double sx = 0.0;
            for (int k = 0; k <= h; ++k) sx += dt[k] * vh[k * 2 + c];
            xb[h * 3 + c] = x[c] + sx;
        }
        xb[h * 3 + 2] = x[2];
    }
    free(a);
    free(vh);
}

/* The ball term: distance of the ball from the tray centre in the tray plane. */
double oracle_cost_ball(const oracle_params *p, const double xb[3])
{
    double dx = xb[0] - p->ball_center[0], dy = xb[1] - p->ball_center[1];
    return sqrt(dx * dx + dy * dy);
}

/* Determinant by Gaussian elimination with partial pivoting (A is overwritten). */
double oracle_det(int n, double *A)
{
    double det = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return 0.0;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            det = -det;
        }
        det *= A[c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
        }
    }
    return det;
}

/* Manipulability sqrt(det(J J^T)) (Sec. 3.2, Eq. 12). */
double oracle_manipulability(const double J[6][DOF])
{
    double A[36];
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double s = 0.0;
            for (int k = 0; k < DOF; ++k) s += J[r][k] * J[c][k];
            A[r * 6 + c] = s;
        }
    double d = oracle_det(6, A);
    return d > 0.0 ? sqrt(d) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Running cost terms (Sec. 3.2).                                            */
/* ------------------------------------------------------------------------ */

/* Pose cost, Eq. 9.  goal = [R_g row-major (9), p_g (3)].  Rotation term:
 * Frobenius norm of diag(alpha_rot)(I - R_g^T R_ee); position term: Euclidean
 * norm of diag(alpha_pos) R_g^T (p_ee - p_g). */
void oracle_cost_pose(const oracle_params *p, const double Tee[16], const double goal[12], double *pos,
                      double *rot)
{
    const double *Rg = goal;
    const double *pg = goal + 9;
    double s = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double m = 0.0; /* (R_g^T R_ee)[r][c] */
            for (int k = 0; k < 3; ++k) m += Rg[k * 3 + r] * Tee[k * 4 + c];
            double e = p->alpha_rot[r] * ((r == c ? 1.0 : 0.0) - m);
            s += e * e;
        }
    *rot = sqrt(s);
    double d[3] = {Tee[3] - pg[0], Tee[7] - pg[1], Tee[11] - pg[2]};
    s = 0.0;
    for (int r = 0; r < 3; ++r) {
        double e = 0.0;
        for (int k = 0; k < 3; ++k) e += Rg[k * 3 + r] * d[k];
        e *= p->alpha_pos[r];
        s += e * e;
    }
    *pos = sqrt(s);
}

/* Band-shrunk box limit (Sec. 3.2, Eq. 11): the safe interval is the full
 * interval shrunk by ratio k of its width at both ends; the cost is the
 * Euclidean norm of the per-joint violation of the safe interval. */
double oracle_cost_box(const double *x, const double *lo, const double *hi, double k)
{
    double s = 0.0;
    for (int j = 0; j < DOF; ++j) {
        double w = hi[j] - lo[j];
        double l = lo[j] + k * w, u = hi[j] - k * w;
        double e = 0.0;
        if (x[j] < l) e = l - x[j];
        if (x[j] > u) e = x[j] - u;
        s += e * e;
    }
    return sqrt(s);
}

/* Stop cost (Sec. 3.2, Eq. 10): velocity limit at step h is the maximum
 * acceleration times the time left to the end of the horizon, including
 * step h (upper-triangular S_u(1) with a unit diagonal).  Joints whose |v|
 * exceed it are penalised by the Euclidean norm of the excess. */
double oracle_stop_limit(int H, const double *dt, double acc, int h)
{
    double s = 0.0;
    for (int k = h; k < H; ++k) s += dt[k];
    return acc * s;
}

double oracle_cost_stop(const double v[DOF], double vmax)
{
    double s = 0.0;
    for (int j = 0; j < DOF; ++j) {
        double e = fabs(v[j]) - vmax;
        if (e > 0.0) s += e * e;
    }
    return sqrt(s);
}

/* Manipulability cost, Eq. 12: 1 - m when m < k_m, else 0. */
double oracle_cost_manip(double m, double k_m) { return m < k_m ? 1.0 - m : 0.0; }

/* World centre of sphere s. */
static void sphere_centre(const oracle_model *mdl, const double T[NFRAMES][16], int s, double c[3])
{
    const double *sp = mdl->spheres + (size_t)s * 5;
    int b = (int)sp[0];
    const double *F = T[b - 1];
    for (int r = 0; r < 3; ++r) c[r] = F[r * 4 + 0] * sp[1] + F[r * 4 + 1] * sp[2] + F[r * 4 + 2] * sp[3] + F[r * 4 + 3];
}

/* Self-collision (replaces the learned distance of Eq. 13 with its
 * analytic definition): largest penetration r_s + r_t - |c_s - c_t| over
 * sphere pairs on bodies at least two apart, clipped at zero. */
double oracle_cost_self(const oracle_model *mdl, const double T[NFRAMES][16])
{
    double best = 0.0;
    for (int s = 0; s < mdl->n_spheres; ++s)
        for (int t = s + 1; t < mdl->n_spheres; ++t) {
            int bs = (int)mdl->spheres[s * 5], bt = (int)mdl->spheres[t * 5];
            if (abs(bs - bt) < 2) continue;
            double cs[3], ct[3];
            sphere_centre(mdl, T, s, cs);
            sphere_centre(mdl, T, t, ct);
            double d = sqrt((cs[0] - ct[0]) * (cs[0] - ct[0]) + (cs[1] - ct[1]) * (cs[1] - ct[1]) +
                            (cs[2] - ct[2]) * (cs[2] - ct[2]));
            double pen = mdl->spheres[s * 5 + 4] + mdl->spheres[t * 5 + 4] - d;
            if (pen > best) best = pen;
        }
    return best;
}

/* Signed distance from point x to obstacle o (negative inside).
 * Sphere: |x - c| - r.  Cuboid with box-to-world rotation R and half extents
 * e: with y = |R^T (x - c)| - e, sdf = |max(y, 0)| + min(max_k y_k, 0). */
double oracle_sdf(const double *o, const double x[3])
{
    double d[3] = {x[0] - o[1], x[1] - o[2], x[2] - o[3]};
    if ((int)o[0] == 0) return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - o[4];
    const double *R = o + 7;
    double y[3], out = 0.0, inmax = -INFINITY;
    for (int k = 0; k < 3; ++k) {
        double l = R[0 * 3 + k] * d[0] + R[1 * 3 + k] * d[1] + R[2 * 3 + k] * d[2];
        y[k] = fabs(l) - o[4 + k];
        if (y[k] > 0.0) out += y[k] * y[k];
        if (y[k] > inmax) inmax = y[k];
    }
    return sqrt(out) + (inmax < 0.0 ? inmax : 0.0);
}

/* Environment collision (a continuous signed-distance form of Eq. 14): sum
 * over body spheres of the penetration r_s - min_o sdf_o(c_s), clipped at 0. */
double oracle_cost_env(const oracle_model *mdl, const double T[NFRAMES][16])
{
    double total = 0.0;
    for (int s = 0; s < mdl->n_spheres; ++s) {
        double c[3];
        sphere_centre(mdl, T, s, c);
        double dmin = INFINITY;
        for (int o = 0; o < mdl->n_obstacles; ++o) {
            double d = oracle_sdf(mdl->obstacles + (size_t)o * OBS_STRIDE, c);
            if (d < dmin) dmin = d;
        }
        double pen = mdl->spheres[s * 5 + 4] - dmin;
        if (pen > 0.0) total += pen;
    }
    return total;
}

/* Learned self-collision distance (Sec. 3.2, Eq. 13, the jointNERF form):
 * input [sin q, cos q] (14), three hidden layers of 256, 128 and 64 units
 * with ReLU, then one linear output, the predicted closest distance
 * between the links (positive when they penetrate).  prm holds, in order,
 * W1 [256][14], b1 [256], W2 [128][256], b2 [128], W3 [64][128], b3 [64],
 * w4 [64], b4 (each weight matrix [out][in]). */
#define MLP_H1 256
#define MLP_H2 128
#define MLP_H3 64
#define MLP_IN 14
double oracle_self_mlp(const double *prm, const double q[DOF])
{
    double x[MLP_IN], a1[MLP_H1], a2[MLP_H2], a3[MLP_H3];
    for (int j = 0; j < DOF; ++j) {
        x[j] = sin(q[j]);
        x[DOF + j] = cos(q[j]);
    }
    const double *W1 = prm, *b1 = W1 + MLP_H1 * MLP_IN;
    const double *W2 = b1 + MLP_H1, *b2 = W2 + MLP_H2 * MLP_H1;
    const double *W3 = b2 + MLP_H2, *b3 = W3 + MLP_H3 * MLP_H2;
    const double *w4 = b3 + MLP_H3, *b4 = w4 + MLP_H3;
    for (int o = 0; o < MLP_H1; ++o) {
        double s = b1[o];
        for (int k = 0; k < MLP_IN; ++k) s += W1[o * MLP_IN + k] * x[k];
        a1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < MLP_H2; ++o) {
        double s = b2[o];
        for (int k = 0; k < MLP_H1; ++k) s += W2[o * MLP_H1 + k] * a1[k];
        a2[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < MLP_H3; ++o) {
        double s = b3[o];
        for (int k = 0; k < MLP_H2; ++k) s += W3[o * MLP_H2 + k] * a2[k];
        a3[o] = s > 0.0 ? s : 0.0;
    }
    double d = b4[0];
    for (int k = 0; k < MLP_H3; ++k) d += w4[k] * a3[k];
    return d;
}

/* The sphere model's signed closest distance between links: the largest
 * r_a + r_b - |c_a - c_b| over the checked pairs (positive = penetration),
 * the quantity the network is trained to predict. */
double oracle_self_distance(const oracle_model *mdl, const double T[NFRAMES][16])
{
    double best = -INFINITY;
    for (int a = 0; a < mdl->n_spheres; ++a)
        for (int b = a + 1; b < mdl->n_spheres; ++b) {
            int ba = (int)mdl->spheres[a * 5], bb = (int)mdl->spheres[b * 5];
            if (bb - ba < 2 && ba - bb < 2) continue;
            double ca[3], cb[3];
            sphere_centre(mdl, T, a, ca);
            sphere_centre(mdl, T, b, cb);
            double dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
            double v = mdl->spheres[a * 5 + 4] + mdl->spheres[b * 5 + 4] - sqrt(dx * dx + dy * dy + dz * dz);
            if (v > best) best = v;
        }
    return best;
}

/* All terms at one state; terms = [pos, rot, joint, vel, stop, manip, self,
 * env, ball] (unweighted; the ball term depends on the whole trajectory and
 * is added by the rollout, 0 here); returns the weighted running cost of
 * Eq. 15. */
double oracle_running_cost(const oracle_params *p, const oracle_model *mdl, const double *dt, int h,
                           const double q[DOF], const double v[DOF], const double goal[12], double terms[NTERMS])
{
    double T[NFRAMES][16];
    for (int k = 0; k < NTERMS; ++k) terms[k] = 0.0;
    oracle_fk(mdl->dh, q, T);
    unsigned m = p->cost_mask;
    if (m & MASK_POSE) oracle_cost_pose(p, T[NFRAMES - 1], goal, &terms[0], &terms[1]);
    if (m & MASK_JOINT) terms[2] = oracle_cost_box(q, mdl->q_min, mdl->q_max, p->k_jl);
    if (m & MASK_VEL) {
        double lo[DOF];
        for (int j = 0; j < DOF; ++j) lo[j] = -mdl->qd_max[j];
        terms[3] = oracle_cost_box(v, lo, mdl->qd_max, p->k_vl);
    }
    if (m & MASK_STOP) terms[4] = oracle_cost_stop(v, oracle_stop_limit(p->h, dt, p->acc_stop, h));
    if (m & MASK_MANIP) {
        double J[6][DOF];
        oracle_jacobian(T, J);
        terms[5] = oracle_cost_manip(oracle_manipulability(J), p->k_m);
    }
    if (m & MASK_SELF) {
        if (p->self_model == 1) {
            double d = oracle_self_mlp(mdl->self_mlp, q);
            terms[6] = d > 0.0 ? d : 0.0; /* Eq. 13 */
        } else {
            terms[6] = oracle_cost_self(mdl, T);
        }
    }
    if (m & MASK_ENV) terms[7] = oracle_cost_env(mdl, T);
    return p->w_pos * terms[0] + p->w_rot * terms[1] + p->a_joint * terms[2] + p->a_vel * terms[3] +
           p->a_stop * terms[4] + p->a_manip * terms[5] + p->a_coll * (terms[6] + terms[7]);
}

/* Horizon weight of step h (Eq. 2): gamma^h for h <= H - 2, and
 * gamma^{H-1} w_term for the terminal step, whose cost is the running cost. */
static double horizon_weight(const oracle_params *p, int h)
{
    double w = pow(p->gamma, (double)h);
    if (h == p->h - 1) w *= p->w_term;
    return w;
}

/* ------------------------------------------------------------------------ */
/* Rollout: sample -> integrate -> costs -> horizon cost.                    */
/* ------------------------------------------------------------------------ */

/* x0 = [q0 (7), v0 (7), a0 (7)]; goal = [R_g (9), p_g (3)]; mean[H][7];
 * sigma[H][7] = standard deviation per step and joint (a per-joint sigma is
 * passed repeated over the steps); eps[N][H][7] standard noise.
 * Controls u = mean + sigma * eps (u = 0 for null particles).  Outputs
 * (nullable except C): u, q, v, a [N][H][7], c[N][H], terms[N][H][9], C[N].  With the
 * ball term on, p->ball holds the ball's state at x0 (world frame). */
int oracle_rollout(const oracle_params *p, const oracle_model *mdl, const double *dt, const double x0[3 * DOF],
                   const double goal[12], const double *mean, const double *sigma, const double *eps, double *u_out,
                   double *q_out, double *v_out, double *a_out, double *c_out, double *terms_out, double *C)
{
    int N = p->n, H = p->h;
    double *u = (double *)malloc(sizeof(double) * (size_t)H * DOF * 4);
    if (!u) return -1;
    double *q = u + (size_t)H * DOF, *v = q + (size_t)H * DOF, *a = v + (size_t)H * DOF;
    double *xb = NULL;
    if (p->cost_mask & MASK_BALL) {
        xb = (double *)malloc(sizeof(double) * (size_t)H * 3);
        if (!xb) {
            free(u);
            return -1;
        }
    }
    for (int i = 0; i < N; ++i) {
        int is_null = i >= N - p->n_null;
        for (int h = 0; h < H; ++h)
            for (int j = 0; j < DOF; ++j) {
                size_t idx = ((size_t)i * H + h) * DOF + j;
                u[h * DOF + j] = is_null ? 0.0 : mean[h * DOF + j] + sigma[h * DOF + j] * eps[idx];
            }
        oracle_integrate(H, dt, x0, x0 + DOF, u, q, v, a);
        if (xb) oracle_ball_traj(p, mdl, dt, x0, q, xb);
        double total = 0.0;
        for (int h = 0; h < H; ++h) {
            double terms[NTERMS];
            double c = oracle_running_cost(p, mdl, dt, h, q + h * DOF, v + h * DOF, goal, terms);
            if (xb) {
                terms[8] = oracle_cost_ball(p, xb + h * 3);
                c += p->w_ball * terms[8];
            }
            total += horizon_weight(p, h) * c;
            if (c_out) c_out[(size_t)i * H + h] = c;
            if (terms_out) memcpy(terms_out + ((size_t)i * H + h) * NTERMS, terms, sizeof(terms));
        }
        C[i] = total;
        size_t base = (size_t)i * H * DOF;
        if (u_out) memcpy(u_out + base, u, sizeof(double) * H * DOF);
        if (q_out) memcpy(q_out + base, q, sizeof(double) * H * DOF);
        if (v_out) memcpy(v_out + base, v, sizeof(double) * H * DOF);
        if (a_out) memcpy(a_out + base, a, sizeof(double) * H * DOF);
    }
    free(xb);
    free(u);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Distribution update (Sec. 3, Eq. 4-6), next command and shift (Alg. 1).   */
/* ------------------------------------------------------------------------ */

/* Weights w_i = exp(-C_i / beta) / sum_k exp(-C_k / beta) (Eq. 6,
 * normalised as in Eq. 4-5); min C is subtracted before exponentiating,
 * which leaves the normalised weights unchanged.  Mean (Eq. 4):
 * mu' = (1 - alpha_mu) mu + alpha_mu sum_i w_i u_i.  Covariance (Eq. 5),
 * diagonal per joint and shared over the horizon: sigma2'_j =
 * (1 - alpha_sigma) sigma2_j + alpha_sigma mean_h sum_i w_i (u_ihj - mu'_hj)^2,
 * then floored at sigma2_min.  Next command = mu'_0; the shifted mean drops
 * step 0 and appends a zero mean.  Returns 1 (and leaves mu, sigma2 as they
 * were) when any C is non-finite or the weight sum is not positive. */
int oracle_update(const oracle_params *p, const double *C, const double *u, const double *mean,
                  const double *sigma2, double *w_out, double *mean_new, double *sigma2_new, double *cmd,
                  double *mean_shift, double *sigma2_shift)
{
    int N = p->n, H = p->h;
    const int nsig = p->cov_per_step ? H * DOF : DOF;
    double cmin = INFINITY;
    int bad = 0;
    for (int i = 0; i < N; ++i) {
        if (!isfinite(C[i])) bad = 1;
        if (C[i] < cmin) cmin = C[i];
    }
    double *w = (double *)malloc(sizeof(double) * (size_t)N);
    if (!w) return -1;
    double sw = 0.0;
    for (int i = 0; i < N && !bad; ++i) {
        w[i] = exp(-(C[i] - cmin) / p->beta);
        sw += w[i];
    }
    if (bad || !(sw > 0.0) || !isfinite(sw)) {
        for (int k = 0; k < H * DOF; ++k) mean_new[k] = mean[k];
        for (int k = 0; k < nsig; ++k) sigma2_new[k] = sigma2[k];
        bad = 1;
    } else {
        for (int i = 0; i < N; ++i) w[i] /= sw;
        for (int h = 0; h < H; ++h)
            for (int j = 0; j < DOF; ++j) {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s += w[i] * u[((size_t)i * H + h) * DOF + j];
                mean_new[h * DOF + j] = (1.0 - p->alpha_mu) * mean[h * DOF + j] + p->alpha_mu * s;
            }
        if (p->cov_per_step) {
            /* Eq. 5 as printed, per step h: the weighted variance of joint j
             * about the updated mean at that step */
            for (int h = 0; h < H; ++h)
                for (int j = 0; j < DOF; ++j) {
                    double acc = 0.0;
                    for (int i = 0; i < N; ++i) {
                        double d = u[((size_t)i * H + h) * DOF + j] - mean_new[h * DOF + j];
                        acc += w[i] * d * d;
                    }
                    double s2 = (1.0 - p->alpha_sigma) * sigma2[h * DOF + j] + p->alpha_sigma * acc;
                    sigma2_new[h * DOF + j] = s2 > p->sigma2_min ? s2 : p->sigma2_min;
                }
        } else {
            for (int j = 0; j < DOF; ++j) {
                double acc = 0.0;
                for (int h = 0; h < H; ++h)
                    for (int i = 0; i < N; ++i) {
                        double d = u[((size_t)i * H + h) * DOF + j] - mean_new[h * DOF + j];
                        acc += w[i] * d * d;
                    }
                double s2 = (1.0 - p->alpha_sigma) * sigma2[j] + p->alpha_sigma * acc / (double)H;
                sigma2_new[j] = s2 > p->sigma2_min ? s2 : p->sigma2_min;
            }
        }
    }
    if (w_out)
        for (int i = 0; i < N; ++i) w_out[i] = bad ? 0.0 : w[i];
    for (int j = 0; j < DOF; ++j) cmd[j] = mean_new[j];
    if (mean_shift) {
        for (int h = 0; h + 1 < H; ++h)
            for (int j = 0; j < DOF; ++j) mean_shift[h * DOF + j] = mean_new[(h + 1) * DOF + j];
        for (int j = 0; j < DOF; ++j) mean_shift[(H - 1) * DOF + j] = 0.0;
    }
    /* the covariance shift (Alg. 1): a per-step covariance moves forward with
     * sigma_init^2 appended; a per-joint one, shared over the steps, stays */
    if (sigma2_shift) {
        if (p->cov_per_step) {
            for (int h = 0; h + 1 < H; ++h)
                for (int j = 0; j < DOF; ++j) sigma2_shift[h * DOF + j] = sigma2_new[(h + 1) * DOF + j];
            for (int j = 0; j < DOF; ++j) sigma2_shift[(H - 1) * DOF + j] = p->sigma_init2[j];
        } else {
            for (int j = 0; j < DOF; ++j) sigma2_shift[j] = sigma2_new[j];
        }
    }
    free(w);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Gradient of the expected horizon cost with respect to the mean.           */
/* ------------------------------------------------------------------------ */

/* d(cost at one state)/dq and d/dv for the differentiable terms (pose,
 * joint, velocity, stop), with hinge and norm kinks given subgradient 0.
 * Returns the running cost at that state. */
static double state_cost_grad(const oracle_params *p, const oracle_model *mdl, const double *dt, int h,
                              const double q[DOF], const double v[DOF], const double goal[12], double gq[DOF],
                              double gv[DOF])
{
    double T[NFRAMES][16], terms[NTERMS];
    double c = oracle_running_cost(p, mdl, dt, h, q, v, goal, terms);
    oracle_fk(mdl->dh, q, T);
    for (int j = 0; j < DOF; ++j) gq[j] = gv[j] = 0.0;
    unsigned m = p->cost_mask;
    if (m & MASK_POSE) {
        const double *E = T[NFRAMES - 1];
        const double *Rg = goal, *pg = goal + 9;
        double R[9] = {E[0], E[1], E[2], E[4], E[5], E[6], E[8], E[9], E[10]};
        double pe[3] = {E[3], E[7], E[11]};
        /* d pos / d p_ee = R_g diag(alpha_pos) e / |e|, e = diag(alpha_pos) R_g^T (p - p_g) */
        double gp[3] = {0, 0, 0};
        if (terms[0] > 0.0) {
            double e[3];
            for (int r = 0; r < 3; ++r) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += Rg[k * 3 + r] * (pe[k] - pg[k]);
                e[r] = p->alpha_pos[r] * s;
            }
            for (int k = 0; k < 3; ++k) {
                double s = 0.0;
                for (int r = 0; r < 3; ++r) s += Rg[k * 3 + r] * p->alpha_pos[r] * e[r];
                gp[k] = p->w_pos * s / terms[0];
            }
        }
        /* d rot / d R_ee = -R_g diag(alpha_rot) M / |M|_F, M = diag(alpha_rot)(I - R_g^T R_ee) */
        double GR[9] = {0};
        if (terms[1] > 0.0) {
            double M[9];
            for (int r = 0; r < 3; ++r)
                for (int c2 = 0; c2 < 3; ++c2) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k) s += Rg[k * 3 + r] * R[k * 3 + c2];
                    M[r * 3 + c2] = p->alpha_rot[r] * ((r == c2 ? 1.0 : 0.0) - s);
                }
            for (int r = 0; r < 3; ++r)
                for (int c2 = 0; c2 < 3; ++c2) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k) s += Rg[r * 3 + k] * p->alpha_rot[k] * M[k * 3 + c2];
                    GR[r * 3 + c2] = -p->w_rot * s / terms[1];
                }
        }
        /* Joint k turns everything beyond it about axis z_k through o_k:
         * dp/dq_k = z_k x (p - o_k), dR/dq_k = [z_k]x R. */
        for (int k = 0; k < DOF; ++k) {
            const double *F = T[k];
            double z[3] = {F[2], F[6], F[10]};
            double o[3] = {F[3], F[7], F[11]};
            double r[3] = {pe[0] - o[0], pe[1] - o[1], pe[2] - o[2]};
            double dp[3] = {z[1] * r[2] - z[2] * r[1], z[2] * r[0] - z[0] * r[2], z[0] * r[1] - z[1] * r[0]};
            double Z[9] = {0, -z[2], z[1], z[2], 0, -z[0], -z[1], z[0], 0};
            double g = gp[0] * dp[0] + gp[1] * dp[1] + gp[2] * dp[2];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double dR = 0.0;
                    for (int t = 0; t < 3; ++t) dR += Z[a * 3 + t] * R[t * 3 + b];
                    g += GR[a * 3 + b] * dR;
                }
            gq[k] += g;
        }
    }
    if ((m & MASK_JOINT) && terms[2] > 0.0) {
        for (int j = 0; j < DOF; ++j) {
            double w = mdl->q_max[j] - mdl->q_min[j];
            double l = mdl->q_min[j] + p->k_jl * w, u = mdl->q_max[j] - p->k_jl * w;
            if (q[j] < l) gq[j] += p->a_joint * (q[j] - l) / terms[2];
            if (q[j] > u) gq[j] += p->a_joint * (q[j] - u) / terms[2];
        }
    }
    if ((m & MASK_VEL) && terms[3] > 0.0) {
        for (int j = 0; j < DOF; ++j) {
            double w = 2.0 * mdl->qd_max[j];
            double l = -mdl->qd_max[j] + p->k_vl * w, u = mdl->qd_max[j] - p->k_vl * w;
            if (v[j] < l) gv[j] += p->a_vel * (v[j] - l) / terms[3];
            if (v[j] > u) gv[j] += p->a_vel * (v[j] - u) / terms[3];
        }
    }
    if ((m & MASK_STOP) && terms[4] > 0.0) {
        double vmax = oracle_stop_limit(p->h, dt, p->acc_stop, h);
        for (int j = 0; j < DOF; ++j) {
            double e = fabs(v[j]) - vmax;
            if (e > 0.0) gv[j] += p->a_stop * e * (v[j] > 0.0 ? 1.0 : -1.0) / terms[4];
        }
    }
    return c;
}

/* g[H][7] = d/d mean of J = (1/N) sum_i C_i(mean + sigma * eps_i), eps held
 * fixed (null particles do not depend on the mean).  Only pose, joint,
 * velocity and stop terms are differentiated; returns -2 if the mask holds
 * other terms.  J is written to *J_out.  The reverse pass runs the chain
 * rule back through the integrator: dC/dv_k collects the direct velocity
 * gradient plus dt_k times the position gradients of all later steps, and
 * dC/du_m = dt_m times the velocity gradients of steps m and later. */
int oracle_grad(const oracle_params *p, const oracle_model *mdl, const double *dt, const double x0[3 * DOF],
                const double goal[12], const double *mean, const double *sigma, const double *eps, double *g,
                double *J_out)
{
    int N = p->n, H = p->h;
    if (p->cost_mask & ~(MASK_POSE | MASK_JOINT | MASK_VEL | MASK_STOP)) return -2;
    double *buf = (double *)malloc(sizeof(double) * (size_t)H * DOF * 7);
    if (!buf) return -1;
    double *u = buf, *q = u + H * DOF, *v = q + H * DOF, *a = v + H * DOF, *gq = a + H * DOF, *gv = gq + H * DOF,
           *gu = gv + H * DOF;
    for (int k = 0; k < H * DOF; ++k) g[k] = 0.0;
    double Jsum = 0.0;
    for (int i = 0; i < N; ++i) {
        int is_null = i >= N - p->n_null;
        for (int h = 0; h < H; ++h)
            for (int j = 0; j < DOF; ++j)
                u[h * DOF + j] = is_null ? 0.0 : mean[h * DOF + j] + sigma[h * DOF + j] * eps[((size_t)i * H + h) * DOF + j];
        oracle_integrate(H, dt, x0, x0 + DOF, u, q, v, a);
        double Ci = 0.0;
        for (int h = 0; h < H; ++h) {
            double w = horizon_weight(p, h);
            Ci += w * state_cost_grad(p, mdl, dt, h, q + h * DOF, v + h * DOF, goal, gq + h * DOF, gv + h * DOF);
            for (int j = 0; j < DOF; ++j) {
                gq[h * DOF + j] *= w;
                gv[h * DOF + j] *= w;
            }
        }
        Jsum += Ci;
        if (is_null) continue;
        for (int j = 0; j < DOF; ++j) {
            /* total velocity gradient Gv_k = gv_k + dt_k sum_{h >= k} gq_h */
            for (int k = 0; k < H; ++k) {
                double s = 0.0;
                for (int h = k; h < H; ++h) s += gq[h * DOF + j];
                gv[k * DOF + j] += dt[k] * s;
            }
            for (int m = 0; m < H; ++m) {
                double s = 0.0;
                for (int k = m; k < H; ++k) s += gv[k * DOF + j];
                gu[m * DOF + j] = dt[m] * s;
            }
            for (int m = 0; m < H; ++m) g[m * DOF + j] += gu[m * DOF + j];
        }
    }
    for (int k = 0; k < H * DOF; ++k) g[k] /= (double)N;
    if (J_out) *J_out = Jsum / (double)N;
    free(buf);
    return 0;
}

/* Expected horizon cost J(mean) alone (for finite differences). */
int oracle_expected_cost(const oracle_params *p, const oracle_model *mdl, const double *dt, const double x0[3 * DOF],
                         const double goal[12], const double *mean, const double *sigma, const double *eps,
                         double *J_out)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)p->n);
    if (!C) return -1;
    int rc = oracle_rollout(p, mdl, dt, x0, goal, mean, sigma, eps, NULL, NULL, NULL, NULL, NULL, NULL, C);
    double s = 0.0;
    for (int i = 0; i < p->n; ++i) s += C[i];
    *J_out = s / (double)p->n;
    free(C);
    return rc;
}
