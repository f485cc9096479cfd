// Batched forward kinematics and manipulability (Sec. 3.1, Eq. 8; Eq. 12):
// one lane per joint configuration.
#include "kinematics.h"

namespace storm {
namespace {

__global__ __launch_bounds__(256) void fk_kernel(RobotDev R, const float *__restrict__ q, int n,
                                                 float *__restrict__ pose, float *__restrict__ manip)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float r[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
    float p[3] = {0.0f, 0.0f, 0.0f};
    float z[kDof][3], o[kDof][3];
#pragma unroll
    for (int f = 0; f < kFrames; ++f) {
        float st = 0.0f, ct = 1.0f;
        if (f < kDof) sincosf(q[(size_t)f * n + t], &st, &ct);
        dh_step(r, p, R.ca[f], R.sa[f], R.a[f], R.d[f], ct, st);
        if (f < kDof) {
            z[f][0] = r[2];
            z[f][1] = r[5];
            z[f][2] = r[8];
            o[f][0] = p[0];
            o[f][1] = p[1];
            o[f][2] = p[2];
        }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) pose[(size_t)c * n + t] = r[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) pose[(size_t)(9 + c) * n + t] = p[c];
    if (manip) manip[t] = manipulability(z, o, p);
}

}  // namespace

hipError_t launch_fk(const RobotDev &R, const float *q, int n, float *pose, float *manip, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fk_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, R, q, n, pose, manip);
    return hipGetLastError();
}

}  // namespace storm
