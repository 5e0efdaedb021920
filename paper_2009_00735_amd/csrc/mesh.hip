// Cube-map candidate lists for the nearest-node search (rotated references
// and the sparse look-up table; supplement, "Indexing algorithm": a rotated
// node is replaced by its closest neighbouring mesh node).
//
// For cell C (centre c, angular radius r_c to its farthest corner) let a_c
// be the angle from c to its nearest node.  Every direction p in C then has
// a node within D = r_c + a_c, so the exact best dot product is at least
// cos D (less 1e-7 for FP32-rounded unit nodes), and every node the FP32
// scan keeps for the FP64 re-rank (within 1e-5 of the FP32 best, FP32 dot
// products within 5e-7 of exact) has an exact dot product of at least
// cmin = cos D - 2e-5.  Such a node is within rho = acos(cmin - 1e-7) of p,
// hence within r_c + rho of c: the list of C is every node n with
// n . c >= cos(r_c + rho) - 1e-6 (FP64), in index order.  The scan of that
// list ranks and re-ranks exactly the nodes a scan of the whole mesh would,
// so the chosen node is the same.
//
// One wave per cell; the lists have a fixed capacity, and a cell whose list
// would exceed it is marked (count -1) and searched over the whole mesh, as
// is every cell of a mesh whose nodes are not unit vectors.
#include "ar_internal.h"
#include "mesh_device.h"

namespace ar {
namespace mesh {

constexpr int kCap = 256;

__device__ __forceinline__ void gnomonic(int a, double sgn, double u, double v, double d[3])
{
    double e[3];
    e[a] = sgn;
    e[a == 0 ? 1 : 0] = u;
    e[a == 2 ? 1 : 2] = v;
    const double n = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    d[0] = e[0] / n;
    d[1] = e[1] / n;
    d[2] = e[2] / n;
}

// one wave per cell, four cells per 256-thread workgroup
__global__ __launch_bounds__(256) void k_mesh_cells(const float *__restrict__ dirs, int n_dir, int G,
                                                    int32_t *__restrict__ count, int32_t *__restrict__ list)
{
    const int lane = threadIdx.x & 63;
    const int cell = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int n_cells = 6 * G * G;
    if (cell >= n_cells) return;
    const int face = cell / (G * G), rem = cell - face * G * G;
    const int iu = rem / G, iv = rem - iu * G;
    const int a = face >> 1;
    const double sgn = (face & 1) ? -1.0 : 1.0;
    const double u0 = -1.0 + 2.0 * iu / G, u1 = -1.0 + 2.0 * (iu + 1) / G;
    const double v0 = -1.0 + 2.0 * iv / G, v1 = -1.0 + 2.0 * (iv + 1) / G;
    double c[3];
    gnomonic(a, sgn, 0.5 * (u0 + u1), 0.5 * (v0 + v1), c);
    double rc = 0.0;
    for (int k = 0; k < 4; ++k) {
        double q[3];
        gnomonic(a, sgn, (k & 1) ? u1 : u0, (k & 2) ? v1 : v0, q);
        rc = fmax(rc, acos(fmin(1.0, c[0] * q[0] + c[1] * q[1] + c[2] * q[2])));
    }
    rc += 1e-9;   // rounding of the cell assignment
    // nearest node to the centre (dot over the node's length); the bounds
    // assume unit nodes (FP32-rounded), so a mesh with any node off the unit
    // sphere by more than 1e-5 in |n|^2 is searched in full
    double best = -2.0;
    bool off_unit = false;
    for (int u = lane; u < n_dir; u += 64) {
        const double x = dirs[3 * u], y = dirs[3 * u + 1], z = dirs[3 * u + 2];
        const double n2 = x * x + y * y + z * z;
        off_unit |= !(fabs(n2 - 1.0) <= 1e-5);
        best = fmax(best, (c[0] * x + c[1] * y + c[2] * z) / sqrt(n2));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if (__ballot(off_unit) != 0ull) {
        if (lane == 0) count[cell] = -1;
        return;
    }
    const double ac = acos(fmax(-1.0, fmin(1.0, best)));
    const double cmin = cos(fmin(M_PI, rc + ac)) - 2e-5;
    const double rho = acos(fmax(-1.0, cmin - 1e-7));
    const double lim = cos(fmin(M_PI, rc + rho)) - 1e-6;
    // ordered compaction of the nodes with n . c >= lim
    int n = 0;
    for (int u0n = 0; u0n < n_dir; u0n += 64) {
        const int u = u0n + lane;
        bool in = false;
        if (u < n_dir) in = c[0] * dirs[3 * u] + c[1] * dirs[3 * u + 1] + c[2] * dirs[3 * u + 2] >= lim;
        const uint64_t m = __ballot(in);
        const int pos = n + __popcll(m & ((1ull << lane) - 1ull));
        if (in && pos < kCap) list[(size_t)cell * kCap + pos] = u;
        n += __popcll(m);
    }
    if (lane == 0) count[cell] = n <= kCap ? n : -1;
}

}  // namespace mesh

int mesh_grid(int n_dir)
{
    int G = (int)floor(sqrt((double)n_dir / 12.0));
    return G < 1 ? 1 : G;
}

ar_status build_mesh_cells(ar_context *ctx, const float *dirs, int n_dir, hipStream_t s, MeshCells &mc)
{
    const int G = mesh_grid(n_dir);
    const int n_cells = 6 * G * G;
    AR_TRY(ctx->m_cells.reserve(sizeof(int32_t) * (size_t)n_cells * (mesh::kCap + 1)));
    int32_t *count = ctx->m_cells.as<int32_t>(), *list = count + n_cells;
    mesh::k_mesh_cells<<<(unsigned)((n_cells + 3) / 4), 256, 0, s>>>(dirs, n_dir, G, count, list);
    AR_HIP(hipGetLastError());
    mc.G = G;
    mc.cap = mesh::kCap;
    mc.count = count;
    mc.list = list;
    return AR_OK;
}

}  // namespace ar
