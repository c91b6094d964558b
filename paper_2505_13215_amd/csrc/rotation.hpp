// Rotations of the Gaussians as the kernels build them (FP64): the left and
// right isoclinic matrices of Eq. 4, whose product R_l R_r rotates (x, y, z, t),
// the unit-quaternion rotation of Eq. 2, and a quaternion column loaded and
// normalised.
#pragma once

#include <hip/hip_runtime.h>

namespace h4d {

__device__ inline void rot_left(const double q[4], double M[4][4]) {
    const double a = q[0], b = q[1], c = q[2], d = q[3];
    M[0][0] = a; M[0][1] = -b; M[0][2] = -c; M[0][3] = -d;
    M[1][0] = b; M[1][1] = a;  M[1][2] = -d; M[1][3] = c;
    M[2][0] = c; M[2][1] = d;  M[2][2] = a;  M[2][3] = -b;
    M[3][0] = d; M[3][1] = -c; M[3][2] = b;  M[3][3] = a;
}
__device__ inline void rot_right(const double q[4], double M[4][4]) {
    const double p = q[0], qq = q[1], r = q[2], s = q[3];
    M[0][0] = p;  M[0][1] = -qq; M[0][2] = -r;  M[0][3] = -s;
    M[1][0] = qq; M[1][1] = p;   M[1][2] = s;   M[1][3] = -r;
    M[2][0] = r;  M[2][1] = -s;  M[2][2] = p;   M[2][3] = qq;
    M[3][0] = s;  M[3][1] = r;   M[3][2] = -qq; M[3][3] = p;
}

__device__ inline double load_unit4(const float* q, int n, int i, double out[4]) {
    double a[4];
    for (int k = 0; k < 4; ++k) a[k] = (double)q[(size_t)k * n + i];
    const double nrm = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
    const double inv = 1.0 / nrm;
    for (int k = 0; k < 4; ++k) out[k] = a[k] * inv;
    return nrm;
}

__device__ inline void quat_rot3(const double q[4], double R[3][3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z); R[0][1] = 2.0 * (x * y - w * z); R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z); R[1][1] = 1.0 - 2.0 * (x * x + z * z); R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y); R[2][1] = 2.0 * (y * z + w * x); R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

}  // namespace h4d
