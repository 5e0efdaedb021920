// Internal declarations shared by the HIP translation units of libaraullo.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "araullo.h"

namespace ar {

// Record a thread-local error message and return `s`.
ar_status fail(ar_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define AR_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::ar::fail(AR_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define AR_TRY(expr)                                                                   \
    do {                                                                               \
        ar_status s_ = (expr);                                                         \
        if (s_ != AR_OK) return s_;                                                    \
    } while (0)

#define AR_CHECK(cond, ...)                                                            \
    do {                                                                               \
        if (!(cond)) return ::ar::fail(AR_EINVAL, __VA_ARGS__);                        \
    } while (0)

// Grow-only device buffer.  Growing frees the old allocation (hipFree waits
// for outstanding work on the device).
struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
    ~DeviceBuffer();
    ar_status reserve(size_t n);
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Eq. (1) constants, computed once in FP64 and rounded to FP32.
struct BinConsts {
    float shift;   // (float)(R + dR)
    float scale;   // (float)(nbins / (2R + 2dR))
};
BinConsts bin_consts(float radius, int nbins);

constexpr int kMaxWindows = 16;
struct WindowSet {
    int n;
    int kmin, kmax;          // union of all windows
    int rows;                // 1: n <= 4, kmax - kmin < 64 and every window at most 16 bins wide;
                             // 2: the same within 32 bins (two lanes per bin in the last FFT stage)
    int lo[kMaxWindows];
    int hi[kMaxWindows];
};
ar_status make_windows(const int32_t *windows, int32_t n_win, int32_t nbins, WindowSet *ws);

bool valid_nbins(int32_t nbins);
int log2i(int32_t x);

}  // namespace ar

struct ar_context {
    int device = 0;
    int cu_count = 0;
    int lds_per_block = 0;
    // gather workspace
    ar::DeviceBuffer g_keys, g_vals, g_counts32, g_cell_start, g_sorted, g_counts, g_temp, g_bbox, g_offsets;
    // gathered CSR used by the position-taking signature entry points
    ar::DeviceBuffer s_rel;
    // one channel's images in the typed-signature entry point
    ar::DeviceBuffer s_typed;
    // correlation tile: per-wave 32x32 MFMA tiles (wtm x wtn) and K step; used
    // when set by ar_index_set_tile, else chosen per candidate count
    int corr_waves = 8, corr_wtm = 4, corr_wtn = 2, corr_bk = 32;
    bool corr_tile_set = false;
    // indexing workspace
    ar::DeviceBuffer i_bf16, i_inv, i_cand_idx, i_cand_score, i_merge_idx;
    // sparse indexing workspace
    ar::DeviceBuffer sp_half, sp_inv, sp_cand_s, sp_cand_i, sp_merge;
    // refinement workspace
    ar::DeviceBuffer r_partials, r_state, r_dirs;
    // nearest-node candidate lists of the last mesh (count [6 G^2], lists [6 G^2][cap])
    ar::DeviceBuffer m_cells;
    // twiddle tables exp(-2 pi i j / nbins), j < nbins, per nbins
    std::map<int, std::unique_ptr<ar::DeviceBuffer>> twiddles;
    ar_status twiddle_table(int nbins, const float2 **out);
};

struct ar_library {
    ar_context *ctx = nullptr;
    const float *ref = nullptr;   // caller-owned FP32 raw images [n_lib][K]
    int64_t n_lib = 0;
    int32_t n_win = 0, n_dir = 0;
    int64_t K = 0;                // n_win * n_dir
    int64_t Kp = 0;               // padded to a multiple of the GEMM K tile
    int64_t n_pad = 0;            // n_lib padded to a multiple of the GEMM N tile
    ar::DeviceBuffer bf16;        // [n_pad][Kp] bf16, normalised
    ar::DeviceBuffer norm2;       // [n_pad] float, |bf16 row|^2 (pad rows: +inf)
    ar::DeviceBuffer inv_max;     // [n_lib][n_win] float, 1/max (0 for a zero image)
    ar::DeviceBuffer quats;       // [n_lib][4] double (w, x, y, z), if prepared with orientations
    ar::DeviceBuffer phase;       // [n_lib] int32, if prepared with orientations
    bool has_orientations = false;
};

namespace ar {
// internal entry points used across translation units
ar_status gather_csr(ar_context *ctx, const float *positions, const int32_t *types, int64_t n_atoms,
                     const float *centres, int64_t n_roi, float radius, uint64_t type_mask, int64_t *offsets,
                     float *rel, int64_t cap, int64_t *total, hipStream_t stream);
struct MeshCells;
// cube-map nearest-node candidate lists of `dirs` in ctx->m_cells (mesh.hip)
ar_status build_mesh_cells(ar_context *ctx, const float *dirs, int n_dir, hipStream_t stream, MeshCells &mc);
// looks up, once per device, the device address of the fixed workspace of
// ar_sf_score_grad_noalloc (refine.hip); `device` must be current
ar_status scratch_setup(int device);
}
