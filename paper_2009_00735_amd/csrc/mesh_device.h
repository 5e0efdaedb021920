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

// Cube-map cells over the unit sphere for the nearest-node search: the
// face is the axis a of the largest |r_a| (first of x, y, z on ties) and its
// sign, (u, v) = the other two coordinates (in axis order) over |r_a|, and
// each face is cut into G x G equal squares of (u, v).  Cell c holds the
// sorted list of every node that can be the nearest node, or fall inside
// the FP64 re-rank window, for any direction in the cell (built by
// build_mesh_cells); count -1 marks a cell whose list would exceed the cap,
// which is then searched over all nodes.
struct MeshCells {
    int G = 0, cap = 0;
    const int32_t *count = nullptr;   // [6 G^2]
    const int32_t *list = nullptr;    // [6 G^2][cap]
};

__device__ __forceinline__ int mesh_cell(double x, double y, double z, int G)
{
    const double ax = fabs(x), ay = fabs(y), az = fabs(z);
    int a;
    double m, u, v, ra;
    if (ax >= ay && ax >= az) {
        a = 0; ra = x; m = ax; u = y; v = z;
    } else if (ay >= az) {
        a = 1; ra = y; m = ay; u = x; v = z;
    } else {
        a = 2; ra = z; m = az; u = x; v = y;
    }
    const int face = 2 * a + (ra < 0.0 ? 1 : 0);
    int iu = (int)floor((u / m + 1.0) * 0.5 * G), iv = (int)floor((v / m + 1.0) * 0.5 * G);
    iu = min(max(iu, 0), G - 1);
    iv = min(max(iv, 0), G - 1);
    return (face * G + iu) * G + iv;
}

// Index of the mesh node closest to the unit vector r (largest dot product):
// an FP32 scan of the candidate nodes finds the maximum, then every candidate
// within 1e-5 of it is re-ranked in FP64, ties to the lower index.  The
// FP32 dot products are within ~1e-7 of the exact ones, so the FP64 winner
// is always re-ranked.  The candidates are the node list of r's cell (in
// index order), which holds every node the same scan over all nodes would
// rank or re-rank, so the result equals that of a scan over all nodes.
__device__ __forceinline__ int nearest_node(double rx, double ry, double rz, const float *__restrict__ dirs,
                                            int n_dir, const MeshCells &mc)
{
    const float fx = (float)rx, fy = (float)ry, fz = (float)rz;
    const int cell = mesh_cell(rx, ry, rz, mc.G);
    const int cnt = mc.count[cell];
    const bool all = cnt < 0;
    const int n = all ? n_dir : cnt;
    const int32_t *lst = mc.list + (size_t)cell * mc.cap;
    float best = -INFINITY;
    for (int k = 0; k < n; ++k) {
        const int u = all ? k : lst[k];
        const float d = fmaf(fz, dirs[3 * u + 2], fmaf(fy, dirs[3 * u + 1], fx * dirs[3 * u]));
        best = fmaxf(best, d);
    }
    double bd = -INFINITY;
    int arg = 0;
    const float thr = best - 1e-5f;
    for (int k = 0; k < n; ++k) {
        const int u = all ? k : lst[k];
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
