// Device kinematics shared by the rollout and FK kernels: one modified-DH
// link transform (Sec. 3.1, Eq. 8) and the manipulability measure of Eq. 12.
#pragma once

#include "storm_internal.h"

namespace storm {

// F <- F RotX(alpha) TransX(a) RotZ(theta) TransZ(d) for a frame held as a
// row-major rotation r[9] and origin p[3].  RotX mixes rotation columns 1 and
// 2, RotZ mixes columns 0 and 1, the translations move the origin along the
// current x and z axes.
// One row of dh_step: row i of R and component i of p depend only on row i
// of the previous frame, so the rows can be carried separately.
__device__ __forceinline__ void dh_step_row(float r[3], float &p, float ca, float sa, float a, float d, float ct,
                                            float st)
{
    const float y = r[1], z = r[2];
    r[1] = fmaf(ca, y, sa * z);
    r[2] = fmaf(-sa, y, ca * z);
    p = fmaf(a, r[0], p);
    const float x = r[0], y2 = r[1];
    r[0] = fmaf(ct, x, st * y2);
    r[1] = fmaf(-st, x, ct * y2);
    p = fmaf(d, r[2], p);
}

__device__ __forceinline__ void dh_step(float r[9], float p[3], float ca, float sa, float a, float d, float ct,
                                        float st)
{
#pragma unroll
    for (int row = 0; row < 3; ++row) dh_step_row(r + 3 * row, p[row], ca, sa, a, d, ct, st);
}

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float c[3])
{
    c[0] = fmaf(a[1], b[2], -a[2] * b[1]);
    c[1] = fmaf(a[2], b[0], -a[0] * b[2]);
    c[2] = fmaf(a[0], b[1], -a[1] * b[0]);
}

// Flange velocity and acceleration (Eq. 8), xd = J qd and xdd = Jdot qd +
// J qdd, by outward passes over the joints instead of forming Jdot: w is the
// angular velocity of the link that carries joint k's axis, so that
// zdot_k = w x z_k, and the origin o_k, fixed in that link, moves with
// od_k = od_{k-1} + w x (o_k - o_{k-1}).  Column k of Jdot is then
// [zdot_k x (p - o_k) + z_k x (pd - od_k); zdot_k].  The first pass gives
// the flange velocity pd; the second repeats the recursion and sums the
// acceleration.  The frames are read from LDS as each pass needs them
// (F = this lane's first frame entry, `stride` floats between entries: R
// row-major then the origin, 12 entries per frame) in loops that are not
// unrolled, which keeps the register footprint small.  Rows: linear, angular.
__device__ __forceinline__ void task_space(const float *F, const int stride, const float qd[kDof],
                                           const float qdd[kDof], float xd[6], float xdd[6])
{
    auto axis = [&](int k, float zk[3]) {
        zk[0] = F[(k * 12 + 2) * stride];
        zk[1] = F[(k * 12 + 5) * stride];
        zk[2] = F[(k * 12 + 8) * stride];
    };
    auto origin = [&](int k, float ok[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ok[c] = F[(k * 12 + 9 + c) * stride];
    };
    float pe[3];
    origin(kFrames - 1, pe);
    float w[3] = {0.0f, 0.0f, 0.0f}, od[3] = {0.0f, 0.0f, 0.0f}, prev[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int k = 0; k < kDof; ++k) {
        float zk[3], ok[3];
        axis(k, zk);
        origin(k, ok);
        if (k > 0) {
            const float d[3] = {ok[0] - prev[0], ok[1] - prev[1], ok[2] - prev[2]};
            float t[3];
            cross3(w, d, t);
#pragma unroll
            for (int c = 0; c < 3; ++c) od[c] += t[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w[c] = fmaf(zk[c], qd[k], w[c]);
            prev[c] = ok[c];
        }
    }
    float pd[3];
    {
        const float d[3] = {pe[0] - prev[0], pe[1] - prev[1], pe[2] - prev[2]};
        cross3(w, d, pd);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pd[c] += od[c];
            xd[c] = pd[c];
            xd[3 + c] = w[c];
        }
    }
    float lin[3] = {0.0f, 0.0f, 0.0f}, ang[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        w[c] = 0.0f;
        od[c] = 0.0f;
    }
#pragma unroll 1
    for (int k = 0; k < kDof; ++k) {
        float zk[3], ok[3];
        axis(k, zk);
        origin(k, ok);
        if (k > 0) {
            const float d[3] = {ok[0] - prev[0], ok[1] - prev[1], ok[2] - prev[2]};
            float t[3];
            cross3(w, d, t);
#pragma unroll
            for (int c = 0; c < 3; ++c) od[c] += t[c];
        }
        float zd[3];
        cross3(w, zk, zd);
        const float r[3] = {pe[0] - ok[0], pe[1] - ok[1], pe[2] - ok[2]};
        const float dv[3] = {pd[0] - od[0], pd[1] - od[1], pd[2] - od[2]};
        float t1[3], t2[3], jc[3];
        cross3(zd, r, t1);
        cross3(zk, dv, t2);
        cross3(zk, r, jc);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lin[c] = fmaf(t1[c] + t2[c], qd[k], fmaf(jc[c], qdd[k], lin[c]));
            ang[c] = fmaf(zd[c], qd[k], fmaf(zk[c], qdd[k], ang[c]));
            w[c] = fmaf(zk[c], qd[k], w[c]);
            prev[c] = ok[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xdd[c] = lin[c];
        xdd[3 + c] = ang[c];
    }
}

// sqrt(det(J J^T)) for the geometric Jacobian whose column k is
// [z_k x (p_e - o_k); z_k].  J J^T (6x6, symmetric positive semi-definite) is
// accumulated over the seven columns and factorised as L D L^T; the
// determinant is the product of the pivots.  A non-positive pivot means a
// singular configuration (m = 0).
__device__ __forceinline__ float manipulability(const float z[kDof][3], const float o[kDof][3], const float pe[3])
{
    float M[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) M[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < kDof; ++k) {
        const float rx = pe[0] - o[k][0], ry = pe[1] - o[k][1], rz = pe[2] - o[k][2];
        float col[6];
        col[0] = z[k][1] * rz - z[k][2] * ry;
        col[1] = z[k][2] * rx - z[k][0] * rz;
        col[2] = z[k][0] * ry - z[k][1] * rx;
        col[3] = z[k][0];
        col[4] = z[k][1];
        col[5] = z[k][2];
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                const int idx = i * (i + 1) / 2 + j;
                M[idx] = fmaf(col[i], col[j], M[idx]);
            }
    }
    // L D L^T in place on the packed lower triangle: after step i, M(i,i)
    // holds D_i and M(j,i) (j > i) holds L_ji.
    float det = 1.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const int ii = i * (i + 1) / 2 + i;
        float di = M[ii];
#pragma unroll
        for (int k = 0; k < i; ++k) {
            const float lik = M[i * (i + 1) / 2 + k];
            di = fmaf(-lik * lik, M[k * (k + 1) / 2 + k], di);
        }
        M[ii] = di;
        det *= di;
        const float inv = di > 0.0f ? 1.0f / di : 0.0f;
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            float s = M[j * (j + 1) / 2 + i];
#pragma unroll
            for (int k = 0; k < i; ++k)
                s = fmaf(-M[j * (j + 1) / 2 + k] * M[i * (i + 1) / 2 + k], M[k * (k + 1) / 2 + k], s);
            M[j * (j + 1) / 2 + i] = s * inv;
        }
        if (!(di > 0.0f)) det = 0.0f;
    }
    return det > 0.0f ? fast_sqrt(det) : 0.0f;
}

}  // namespace storm
