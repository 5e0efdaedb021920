// ROI query: atoms within radius R of each ROI centre, as a CSR of relative
// coordinates (Sec. 2.1: spherical ROIs scan the dataset; supplement, cost
// model: one neighbour query per ROI before the projections).
//
// GPU design: a uniform cell grid (cell edge R/2) over the box spanned by the
// ROI centres +- R; atoms are bucketed by cell with a counting sort (per-cell
// counts by atomics, an exclusive scan for the cell starts, an atomic
// scatter, then each cell's atoms put back in input order, so the result is
// the stable sort by cell id), each ROI is served by one wavefront that walks
// the rows of cells overlapping its ball (+-1 cell of slack against FP32
// rounding of the cell index).  Rows of cells are contiguous in the sorted
// array, so each row is one coalesced range.
// Membership is decided exactly as the paper's single-precision test:
// fmaf(dz,dz,fmaf(dy,dy,dx*dx)) <= (float)(R*R).
#include <math.h>

#include <algorithm>

#include "ar_internal.h"
#include "scan_device.h"

namespace ar {
namespace {

struct Grid {
    float ox, oy, oz, inv_h;
    int nx, ny, nz;
};

__global__ __launch_bounds__(1024) void k_centre_bbox(const float *__restrict__ c, int64_t n,
                                                      float *__restrict__ out)
{
    __shared__ float red[6][1024];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        for (int a = 0; a < 3; ++a) {
            float v = c[3 * i + a];
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = lo[a];
        red[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ int cell_coord(float p, float o, float inv_h) { return (int)floorf((p - o) * inv_h); }

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *__restrict__ a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

// Cell id of every atom (ncells for atoms outside the grid) and the count of
// every cell.
__global__ __launch_bounds__(256) void k_cell_keys(const float *__restrict__ pos, int64_t n, Grid g,
                                                   uint32_t *__restrict__ keys, int32_t *__restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t ncells = (uint32_t)g.nx * g.ny * g.nz;
    int cx = cell_coord(pos[3 * i + 0], g.ox, g.inv_h);
    int cy = cell_coord(pos[3 * i + 1], g.oy, g.inv_h);
    int cz = cell_coord(pos[3 * i + 2], g.oz, g.inv_h);
    bool in = cx >= 0 && cx < g.nx && cy >= 0 && cy < g.ny && cz >= 0 && cz < g.nz;
    const uint32_t key = in ? (uint32_t)(cx + g.nx * (cy + g.ny * cz)) : ncells;
    keys[i] = key;
    if (in) atomicAdd(&counts[key], 1);
}

// Each atom inside the grid to a slot of its cell (slots in arrival order,
// fixed afterwards by k_cell_order); cursor starts at zero.
__global__ __launch_bounds__(256) void k_cell_scatter(const uint32_t *__restrict__ keys, int64_t n, uint32_t ncells,
                                                      const int32_t *__restrict__ cell_start,
                                                      int32_t *__restrict__ cursor, int32_t *__restrict__ idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    if (key >= ncells) return;
    idx[cell_start[key] + atomicAdd(&cursor[key], 1)] = (int32_t)i;
}

// One thread per cell: its atoms back into input order (insertion sort of
// the atom indices; cells hold tens of atoms at the R/2 cell edge).
__global__ __launch_bounds__(256) void k_cell_order(const int32_t *__restrict__ cell_start, uint32_t ncells,
                                                    int32_t *__restrict__ idx)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)ncells) return;
    const int a0 = cell_start[c], a1 = cell_start[c + 1];
    for (int a = a0 + 1; a < a1; ++a) {
        const int32_t v = idx[a];
        int b = a - 1;
        while (b >= a0 && idx[b] > v) {
            idx[b + 1] = idx[b];
            --b;
        }
        idx[b + 1] = v;
    }
}

// Sorted positions; the 4th component carries the atom type's bits (0 when
// the call has no types).
__global__ __launch_bounds__(256) void k_sorted_pos(const float *__restrict__ pos, const int32_t *__restrict__ types,
                                                    const int32_t *__restrict__ idx,
                                                    const int32_t *__restrict__ cell_start, uint32_t ncells,
                                                    float4 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cell_start[ncells]) return;
    const int64_t a = idx[i];
    out[i] = make_float4(pos[3 * a], pos[3 * a + 1], pos[3 * a + 2], __int_as_float(types ? types[a] : 0));
}

// Atom type t is accepted iff 0 <= t < 64 and bit t of the mask is set.
__device__ __forceinline__ bool type_accepted(float w, uint64_t mask)
{
    const uint32_t t = (uint32_t)__float_as_int(w);
    return t < 64u && ((mask >> t) & 1ull);
}

// One wavefront per ROI.  FILL == false: count; FILL == true: write rows.
template <bool FILL>
__global__ __launch_bounds__(256) void k_roi_query(const float4 *__restrict__ spos, const int32_t *__restrict__ cell_start,
                                                   Grid g, const float *__restrict__ centres, int64_t n_roi,
                                                   float radius, float R2, uint64_t type_mask,
                                                   int64_t *__restrict__ counts_or_offsets,
                                                   int64_t *__restrict__ offsets0, float4 *__restrict__ rel)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (!FILL && blockIdx.x == 0 && threadIdx.x == 0) offsets0[0] = 0;
    if (r >= n_roi) return;
    const float cx = centres[3 * r], cy = centres[3 * r + 1], cz = centres[3 * r + 2];
    const int x0 = max(cell_coord(cx - radius, g.ox, g.inv_h) - 1, 0);
    const int x1 = min(cell_coord(cx + radius, g.ox, g.inv_h) + 1, g.nx - 1);
    const int y0 = max(cell_coord(cy - radius, g.oy, g.inv_h) - 1, 0);
    const int y1 = min(cell_coord(cy + radius, g.oy, g.inv_h) + 1, g.ny - 1);
    const int z0 = max(cell_coord(cz - radius, g.oz, g.inv_h) - 1, 0);
    const int z1 = min(cell_coord(cz + radius, g.oz, g.inv_h) + 1, g.nz - 1);
    int64_t count = 0;
    const int64_t base = FILL ? counts_or_offsets[r] : 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y) {
            const int row = g.nx * (y + g.ny * z);
            const int a0 = cell_start[row + x0], a1 = cell_start[row + x1 + 1];
            for (int i0 = a0; i0 < a1; i0 += 64) {
                const int i = i0 + lane;
                bool in = false;
                float dx = 0.f, dy = 0.f, dz = 0.f;
                if (i < a1) {
                    const float4 p = spos[i];
                    dx = p.x - cx;
                    dy = p.y - cy;
                    dz = p.z - cz;
                    in = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= R2 && type_accepted(p.w, type_mask);
                }
                const uint64_t m = __ballot(in);
                if (FILL && in) rel[base + count + __popcll(m & lt_mask)] = make_float4(dx, dy, dz, 0.f);
                count += __popcll(m);
            }
        }
    if (!FILL && lane == 0) counts_or_offsets[r] = count;
}

}  // namespace

ar_status gather_csr(ar_context *ctx, const float *positions, const int32_t *types, int64_t n_atoms,
                     const float *centres, int64_t n_roi, float radius, uint64_t type_mask, int64_t *offsets, float *rel,
                     int64_t cap, int64_t *total, hipStream_t stream)
{
    AR_CHECK(ctx != nullptr, "context is NULL");
    AR_CHECK(n_atoms >= 0 && n_atoms < (int64_t)INT32_MAX, "n_atoms must be in [0, 2^31-1)");
    AR_CHECK(n_roi >= 1, "n_roi must be >= 1");
    AR_CHECK(radius > 0.f && isfinite(radius), "radius must be finite and > 0");
    AR_CHECK(centres && offsets && total, "centres/offsets/total must not be NULL");
    AR_CHECK(n_atoms == 0 || positions, "positions is NULL");
    AR_HIP(hipSetDevice(ctx->device));

    // bounding box of the centres
    AR_TRY(ctx->g_bbox.reserve(6 * sizeof(float)));
    k_centre_bbox<<<1, 1024, 0, stream>>>(centres, n_roi, ctx->g_bbox.as<float>());
    AR_HIP(hipGetLastError());
    float bb[6];
    AR_HIP(hipMemcpyAsync(bb, ctx->g_bbox.ptr, sizeof(bb), hipMemcpyDeviceToHost, stream));
    AR_HIP(hipStreamSynchronize(stream));
    for (int a = 0; a < 6; ++a) AR_CHECK(isfinite(bb[a]), "ROI centres must be finite");

    // grid: cell edge R/2, grown if the box would need too many cells
    double h = 0.5 * (double)radius;
    const double pad = (double)radius + h;
    double ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = (double)bb[3 + a] - (double)bb[a] + 2.0 * pad;
    for (;;) {
        double cells = 1.0;
        for (int a = 0; a < 3; ++a) cells *= floor(ext[a] / h) + 1.0;
        if (cells <= 6.4e7) break;
        h *= 1.5;
    }
    Grid g;
    g.ox = (float)((double)bb[0] - pad);
    g.oy = (float)((double)bb[1] - pad);
    g.oz = (float)((double)bb[2] - pad);
    g.inv_h = (float)(1.0 / h);
    g.nx = (int)(floor(ext[0] / h) + 1.0);
    g.ny = (int)(floor(ext[1] / h) + 1.0);
    g.nz = (int)(floor(ext[2] / h) + 1.0);
    const uint32_t ncells = (uint32_t)g.nx * g.ny * g.nz;

    // counting sort of the atoms by cell: counts, cell starts (exclusive
    // scan), scatter, per-cell input order
    const int64_t n = n_atoms;
    AR_TRY(ctx->g_keys.reserve(sizeof(uint32_t) * (n + 1)));
    AR_TRY(ctx->g_vals.reserve(sizeof(int32_t) * (n + 1)));
    AR_TRY(ctx->g_counts32.reserve(sizeof(int32_t) * ((size_t)ncells + 1)));
    AR_TRY(ctx->g_cell_start.reserve(sizeof(int32_t) * ((size_t)ncells + 1)));
    AR_TRY(ctx->g_sorted.reserve(sizeof(float4) * (n + 1)));
    AR_TRY(ctx->g_temp.reserve(std::max(sizeof(int32_t) * scan::tiles(ncells), sizeof(int64_t) * scan::tiles(n_roi)) +
                               16));
    int32_t *counts = ctx->g_counts32.as<int32_t>();
    int32_t *cell_start = ctx->g_cell_start.as<int32_t>();
    const unsigned fill_blocks = (unsigned)std::min<int64_t>(((int64_t)ncells + 255) / 256, 4096);
    k_fill_i32<<<fill_blocks, 256, 0, stream>>>(counts, ncells);
    AR_HIP(hipGetLastError());
    if (n > 0) {
        k_cell_keys<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(positions, n, g, ctx->g_keys.as<uint32_t>(),
                                                                    counts);
        AR_HIP(hipGetLastError());
    }
    AR_TRY((scan::exclusive_scan<int32_t, int32_t>(counts, ncells, cell_start, ctx->g_temp.as<int32_t>(), stream)));
    if (n > 0) {
        k_fill_i32<<<fill_blocks, 256, 0, stream>>>(counts, ncells);
        AR_HIP(hipGetLastError());
        k_cell_scatter<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(ctx->g_keys.as<uint32_t>(), n, ncells,
                                                                       cell_start, counts, ctx->g_vals.as<int32_t>());
        AR_HIP(hipGetLastError());
        k_cell_order<<<(unsigned)(((int64_t)ncells + 255) / 256), 256, 0, stream>>>(cell_start, ncells,
                                                                                     ctx->g_vals.as<int32_t>());
        AR_HIP(hipGetLastError());
        k_sorted_pos<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(positions, types, ctx->g_vals.as<int32_t>(),
                                                                     cell_start, ncells, ctx->g_sorted.as<float4>());
        AR_HIP(hipGetLastError());
    }
    const float R2 = (float)((double)radius * (double)radius);
    const unsigned qblocks = (unsigned)((n_roi + 3) / 4);
    AR_TRY(ctx->g_counts.reserve(sizeof(int64_t) * n_roi));
    k_roi_query<false><<<qblocks, 256, 0, stream>>>(ctx->g_sorted.as<float4>(), ctx->g_cell_start.as<int32_t>(), g,
                                                   centres, n_roi, radius, R2, type_mask, ctx->g_counts.as<int64_t>(),
                                                   offsets, nullptr);
    AR_HIP(hipGetLastError());
    AR_TRY((scan::exclusive_scan<int64_t, int64_t>(ctx->g_counts.as<int64_t>(), n_roi, offsets,
                                                   ctx->g_temp.as<int64_t>(), stream)));
    int64_t tot = 0;
    AR_HIP(hipMemcpyAsync(&tot, offsets + n_roi, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    AR_HIP(hipStreamSynchronize(stream));
    *total = tot;
    if (!rel) return AR_OK;
    AR_CHECK(cap >= tot, "rel capacity %lld is smaller than the %lld gathered rows", (long long)cap, (long long)tot);
    k_roi_query<true><<<qblocks, 256, 0, stream>>>(ctx->g_sorted.as<float4>(), ctx->g_cell_start.as<int32_t>(), g,
                                                  centres, n_roi, radius, R2, type_mask, offsets, nullptr,
                                                  (float4 *)rel);
    AR_HIP(hipGetLastError());
    return AR_OK;
}

}  // namespace ar

extern "C" ar_status ar_roi_gather(ar_context *ctx, const float *positions, int64_t n_atoms, const float *centres,
                                   int64_t n_roi, float radius, int64_t *offsets, float *rel, int64_t cap,
                                   int64_t *total, void *stream)
{
    return ar::gather_csr(ctx, positions, nullptr, n_atoms, centres, n_roi, radius, ~0ull, offsets, rel, cap, total,
                          (hipStream_t)stream);
}

extern "C" ar_status ar_roi_gather_typed(ar_context *ctx, const float *positions, const int32_t *types,
                                         int64_t n_atoms, const float *centres, int64_t n_roi, float radius,
                                         uint64_t type_mask, int64_t *offsets, float *rel, int64_t cap,
                                         int64_t *total, void *stream)
{
    AR_CHECK(n_atoms == 0 || types != nullptr, "types is NULL");
    return ar::gather_csr(ctx, positions, types, n_atoms, centres, n_roi, radius, type_mask, offsets, rel, cap, total,
                          (hipStream_t)stream);
}
