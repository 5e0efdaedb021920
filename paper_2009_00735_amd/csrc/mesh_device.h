// Mesh helpers shared by the rotated-reference and look-up-table kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ar {

// Rotation matrix (row-major) of the quaternion (w, x, y, z) / |q|, FP64.
__device__ __forceinline__ void quat_matrix64(const double *q, double M[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    const double nq = sqrt(w * w + x * x + y * y + z * z);
    w /= nq; x /= nq; y /= nq; z /= nq;
    M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
    M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
    M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

// Index of the mesh node closest to the unit vector r (largest dot product):
// an FP32 scan finds the maximum, then every node within 1e-5 of it is
// re-ranked in FP64, ties to the lower index.  The FP32 dot products are
// within ~1e-7 of the exact ones, so the FP64 winner is always re-ranked.
// The node reads are the same for every lane of a wave.
__device__ __forceinline__ int nearest_node(double rx, double ry, double rz, const float *__restrict__ dirs,
                                            int n_dir)
{
    const float fx = (float)rx, fy = (float)ry, fz = (float)rz;
    float best = -INFINITY;
    for (int u = 0; u < n_dir; ++u) {
        const float d = fmaf(fz, dirs[3 * u + 2], fmaf(fy, dirs[3 * u + 1], fx * dirs[3 * u]));
        best = fmaxf(best, d);
    }
    double bd = -INFINITY;
    int arg = 0;
    const float thr = best - 1e-5f;
    for (int u = 0; u < n_dir; ++u) {
        const float d = fmaf(fz, dirs[3 * u + 2], fmaf(fy, dirs[3 * u + 1], fx * dirs[3 * u]));
        if (d >= thr) {
            const double dd = rx * (double)dirs[3 * u] + ry * (double)dirs[3 * u + 1] + rz * (double)dirs[3 * u + 2];
            if (dd > bd) {
                bd = dd;
                arg = u;
            }
        }
    }
    return arg;
}

}  // namespace ar
