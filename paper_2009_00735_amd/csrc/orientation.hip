// Orientation helpers: FP64 cubic disorientation (supplement, "Creation of
// test orientations") and rotated reference images by nearest mesh node
// (supplement, "Indexing algorithm").
#include <math.h>

#include "ar_internal.h"
#include "mesh_device.h"

namespace ar {
namespace {

struct Q64 {
    double w, x, y, z;
};

__device__ __forceinline__ Q64 qmul(const Q64 &a, const Q64 &b)
{
    return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// Largest |w| of m * S over the 24 proper rotations S of the cube:
// identity, 180 deg about <100>, +-90 deg about <100>, 180 deg about <110>,
// +-120 deg about <111>.
__device__ __forceinline__ double best_cos_half(const Q64 &m)
{
    const double h = 0.70710678118654752440;
    double best = 0.0;
    // identity, 180 about x, y, z
    const Q64 G[24] = {
        {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1},
        {h, h, 0, 0}, {h, -h, 0, 0}, {h, 0, h, 0}, {h, 0, -h, 0}, {h, 0, 0, h}, {h, 0, 0, -h},
        {0, h, h, 0}, {0, h, -h, 0}, {0, 0, h, h}, {0, 0, h, -h}, {0, h, 0, h}, {0, -h, 0, h},
        {0.5, 0.5, 0.5, 0.5}, {0.5, 0.5, 0.5, -0.5}, {0.5, 0.5, -0.5, 0.5}, {0.5, 0.5, -0.5, -0.5},
        {0.5, -0.5, 0.5, 0.5}, {0.5, -0.5, 0.5, -0.5}, {0.5, -0.5, -0.5, 0.5}, {0.5, -0.5, -0.5, -0.5}};
#pragma unroll
    for (int s = 0; s < 24; ++s) {
        const Q64 t = qmul(m, G[s]);
        best = fmax(best, fabs(t.w));
    }
    return best;
}

__global__ __launch_bounds__(256) void k_disorientation(const double *__restrict__ qa, const double *__restrict__ qb,
                                                        int64_t n, double *__restrict__ deg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Q64 a = {qa[4 * i], qa[4 * i + 1], qa[4 * i + 2], qa[4 * i + 3]};
    Q64 b = {qb[4 * i], qb[4 * i + 1], qb[4 * i + 2], qb[4 * i + 3]};
    const double na = sqrt(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
    const double nb = sqrt(b.w * b.w + b.x * b.x + b.y * b.y + b.z * b.z);
    const Q64 ai = {a.w / na, -a.x / na, -a.y / na, -a.z / na};
    const Q64 bn = {b.w / nb, b.x / nb, b.y / nb, b.z / nb};
    const double c = fmin(1.0, best_cos_half(qmul(ai, bn)));
    deg[i] = 2.0 * acos(c) * (180.0 / 3.14159265358979323846);
}

// One thread per (entry, node): rotate n_v by R(q)^T and take the reference
// value at the closest node (nearest_node over the cell's candidate list:
// FP32 scan, FP64 re-rank, ties to the lower index).
__global__ __launch_bounds__(256) void k_rotate_reference(const float *__restrict__ ref, int n_win,
                                                          const float *__restrict__ dirs, int n_dir,
                                                          const double *__restrict__ quats,
                                                          const int32_t *__restrict__ phase, int n_phase,
                                                          int64_t n_lib, MeshCells mc, float *__restrict__ out)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t l = gid / n_dir;
    const int v = (int)(gid - l * n_dir);
    const bool valid = l < n_lib;
    double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (valid) quat_matrix64(quats + 4 * l, M);
    const double nx = valid ? dirs[3 * v] : 0.0, ny = valid ? dirs[3 * v + 1] : 0.0, nz = valid ? dirs[3 * v + 2] : 0.0;
    const double rx = M[0] * nx + M[3] * ny + M[6] * nz;
    const double ry = M[1] * nx + M[4] * ny + M[7] * nz;
    const double rz = M[2] * nx + M[5] * ny + M[8] * nz;
    const int arg = nearest_node(rx, ry, rz, dirs, n_dir, mc);
    if (!valid) return;
    const int p = min(max(phase[l], 0), n_phase - 1);   // out-of-range phases are clamped
    for (int w = 0; w < n_win; ++w)
        out[((size_t)l * n_win + w) * n_dir + v] = ref[((size_t)p * n_win + w) * n_dir + arg];
}

}  // namespace
}  // namespace ar

extern "C" {

ar_status ar_disorientation_cubic(const double *qa, const double *qb, int64_t n, double *deg, void *stream)
{
    AR_CHECK(n >= 0, "n must be >= 0");
    if (n == 0) return AR_OK;
    AR_CHECK(qa && qb && deg, "qa/qb/deg must not be NULL");
    ar::k_disorientation<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(qa, qb, n, deg);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

ar_status ar_rotate_reference(ar_context *ctx, const float *reference, int32_t n_phase, int32_t n_win,
                              const float *directions, int32_t n_dir, const double *quats, const int32_t *phase,
                              int64_t n_lib, float *out, void *stream)
{
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(reference && directions && quats && phase && out, "NULL argument");
    AR_CHECK(n_phase >= 1 && n_win >= 1 && n_dir >= 1 && n_lib >= 0, "bad sizes");
    if (n_lib == 0) return AR_OK;
    AR_HIP(hipSetDevice(ctx->device));
    const int64_t n = n_lib * n_dir;
    AR_CHECK((n + 255) / 256 < (int64_t)INT32_MAX, "too many items");
    ar::MeshCells mc;
    AR_TRY(ar::build_mesh_cells(ctx, directions, n_dir, (hipStream_t)stream, mc));
    ar::k_rotate_reference<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        reference, n_win, directions, n_dir, quats, phase, n_phase, n_lib, mc, out);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // extern "C"
