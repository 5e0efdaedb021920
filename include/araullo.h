/*
 * araullo.h - C ABI of the MI355X (gfx950) implementation of the real-space
 * signature and orientation-indexing method of Kuehbach, Kasemer, Gault and
 * Breen, "On Open and Strong-Scaling Tools for Atom Probe Crystallography:
 * High-Throughput Methods for Indexing Crystal Structure and Orientation"
 * (arXiv 2009.00735).
 *
 * Conventions for every entry point:
 *  - Lengths are in nm.  Arrays are C-contiguous, row-major.
 *  - "device" pointers are HIP device allocations on the context's device,
 *    owned by the caller; the library reads/writes them in stream order and
 *    never frees or retains them after the stream has passed the call.
 *    "host" pointers are ordinary host memory, read or written before the
 *    function returns.
 *  - All arguments are validated before any work is queued, so a call that
 *    returns an error has written nothing.  Errors: AR_EINVAL (bad argument),
 *    AR_ENOMEM (a workspace allocation failed), AR_EDEVICE (a HIP runtime
 *    error, including an earlier asynchronous fault), AR_EUNSUPPORTED.
 *    ar_last_error(ctx) returns a thread-local message for the last failure.
 *  - No exceptions cross this boundary.
 *  - Work is queued on `stream` (a hipStream_t passed as void*; NULL is the
 *    null stream).  Calls that must know a data-dependent size on the host
 *    (marked "synchronises") wait for the stream.
 *  - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef ARAULLO_H
#define ARAULLO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AR_OK = 0,
    AR_EINVAL = -1,
    AR_ENOMEM = -2,
    AR_EDEVICE = -3,
    AR_EUNSUPPORTED = -4
} ar_status;

typedef struct ar_context ar_context;
typedef struct ar_library ar_library;
typedef struct ar_plan ar_plan;
typedef struct ar_sparse_lut ar_sparse_lut;

/* Message of the last failed call on this thread ("" if none).  The
 * message is kept per thread, not per context: ctx may be NULL, and any
 * context (or none) gives the same message. */
const char *ar_last_error(const ar_context *ctx);

/* Version string of the library build. */
const char *ar_version(void);

/* Create a context on HIP device `device`: it owns reusable device
 * workspace and the tables the kernels read.  Destroy frees them.  Calls
 * that share a context share its workspace: issue them on one stream, or
 * synchronise before switching streams. */
ar_status ar_context_create(int device, ar_context **out);
ar_status ar_context_destroy(ar_context *ctx);

/*
 * Window of DFT indices for a lattice-spacing interval [d_min, d_max]
 * (supplement, reconstruction parameters: an image value is the window
 * maximum of the amplitude spectrum over the bins of a spacing range;
 * Fig. 2 caption: spacing d sits at index L/d with L = 2R + 2dR the
 * histogram span and dR = R / (nbins/2 - 1) the bin width of Eq. (1)).
 * Result: k_lo = ceil(L/d_max), k_hi = floor(L/d_min), evaluated in FP64.
 * Host call.  AR_EINVAL unless nbins is a power of two in [256, 4096],
 * radius > 0, 0 < d_min <= d_max and 1 <= k_lo <= k_hi <= nbins/2.
 */
ar_status ar_window_bins(double radius, int32_t nbins, double d_min, double d_max,
                         int32_t *k_lo, int32_t *k_hi);

/*
 * ROI query (Sec. 2.1: every spherical ROI of radius R collects the atoms
 * around its centre; supplement, cost model: the query precedes the
 * projections).  An atom belongs to ROI r iff, in FP32,
 * fmaf(dz,dz,fmaf(dy,dy,dx*dx)) <= (float)(R*R) with d = p - c_r.
 *   positions  device float [n_atoms][3]
 *   centres    device float [n_roi][3]
 *   offsets    device int64 [n_roi+1], out: CSR row starts (offsets[0] = 0)
 *   rel        device float [cap][4] or NULL, out: relative coordinates
 *              d = p - c (FP32 subtraction), 4th component 0; rows of ROI r
 *              are rel[offsets[r] .. offsets[r+1]); within a ROI atoms come
 *              in a fixed (deterministic) order
 *   total      host int64, out: offsets[n_roi]
 * With rel == NULL only offsets and total are produced.  AR_EINVAL if
 * rel != NULL and cap < total (offsets and total are still written).
 * Synchronises.
 */
ar_status ar_roi_gather(ar_context *ctx, const float *positions, int64_t n_atoms,
                        const float *centres, int64_t n_roi, float radius,
                        int64_t *offsets, float *rel, int64_t cap, int64_t *total,
                        void *stream);

/*
 * ROI query restricted to atom types (Sec. 3.1: the L1_2 Al3Sc case needs
 * one amplitude spectrum per sub-lattice; supplement, Al-Li-Mg specimens:
 * references for the aluminium and the lithium sub-lattices of Al3Li).  As
 * ar_roi_gather, and an atom is gathered only if its type t = types[i]
 * satisfies 0 <= t < 64 and bit t of type_mask is set.
 *   types      device int32 [n_atoms]
 * ar_roi_gather equals this call with every type accepted.  Synchronises.
 */
ar_status ar_roi_gather_typed(ar_context *ctx, const float *positions, const int32_t *types,
                              int64_t n_atoms, const float *centres, int64_t n_roi, float radius,
                              uint64_t type_mask, int64_t *offsets, float *rel, int64_t cap,
                              int64_t *total, void *stream);

/*
 * Real-space signatures (Sec. 2.2, RSP paragraph and Eq. (1); supplement,
 * "Controlled windowing of the SDMs" and reconstruction parameters).  For
 * every ROI r and direction v: the ROI's atoms are projected on v and binned
 * by Eq. (1) into nbins bins spanning [-(R+dR), R+dR], dR = R/(nbins/2-1),
 *   s = fmaf(vz,dz,fmaf(vy,dy,vx*dx)),  t = (s + (float)(R+dR)) *
 *   (float)(nbins/(2R+2dR)),  b = clamp(floor(t), 0, nbins-1)   (FP32),
 * the histogram is Fourier transformed, and
 *   images[r][w][v] = max_{k_lo(w) <= k <= k_hi(w)} |X_k|,
 *   X_k = sum_n h_n exp(-2 pi i k n / nbins)                     (FP32).
 *   positions  device float [n_atoms][3]
 *   centres    device float [n_roi][3]
 *   directions device float [n_dir][3], unit vectors
 *   nbins      2^m, m in [8, 12]
 *   windows    host int32 [n_win][2] inclusive (k_lo, k_hi), 1 <= k_lo <=
 *              k_hi <= nbins/2, n_win in [1, 16]
 *   images     device float [n_roi][n_win][n_dir], out
 *   roi_counts device int32 [n_roi] or NULL, out: atoms per ROI
 * ROIs with no atoms get zero images.  Any atom count is accepted (a ROI
 * larger than the LDS atom stage is streamed through it in chunks).
 * Synchronises (ROI query).
 */
ar_status araullo_signatures(ar_context *ctx, const float *positions, int64_t n_atoms,
                             const float *centres, int64_t n_roi, float radius,
                             const float *directions, int32_t n_dir, int32_t nbins,
                             const int32_t *windows, int32_t n_win,
                             float *images, int32_t *roi_counts, void *stream);

/*
 * Sub-lattice signatures (Sec. 3.1, the Al3Sc discussion: one signature per
 * atom type set; supplement, Al-Li-Mg specimens): for every channel c the
 * signatures of araullo_signatures computed from the atoms whose type is in
 * type_masks[c] (as ar_roi_gather_typed), stacked per ROI:
 *   images[r][c][w][v]     device float [n_roi][n_ch][n_win][n_dir], out
 *   roi_counts[r][c]       device int32 [n_roi][n_ch] or NULL, out
 *   types                  device int32 [n_atoms]
 *   type_masks             host uint64 [n_ch], 1 <= n_ch <= 64
 * The (channel, window) pairs form the window axis the indexing calls read
 * (n_ch * n_win windows), so the stacked images index directly against
 * stacked references.  Channel images are bit-identical to araullo_signatures
 * on the filtered atoms.  Synchronises.
 */
ar_status araullo_signatures_typed(ar_context *ctx, const float *positions, const int32_t *types,
                                   int64_t n_atoms, const float *centres, int64_t n_roi, float radius,
                                   const uint64_t *type_masks, int32_t n_ch, const float *directions,
                                   int32_t n_dir, int32_t nbins, const int32_t *windows, int32_t n_win,
                                   float *images, int32_t *roi_counts, void *stream);

/*
 * Same Eq. (1) histograms and spectra as araullo_signatures, written out in
 * full for inspection and parity checks.
 *   hist  device int32 [n_roi][n_dir][nbins] or NULL, out
 *   amp   device float [n_roi][n_dir][nbins/2+1] or NULL, out: |X_k|
 * Synchronises.
 */
ar_status araullo_sdm(ar_context *ctx, const float *positions, int64_t n_atoms,
                      const float *centres, int64_t n_roi, float radius,
                      const float *directions, int32_t n_dir, int32_t nbins,
                      int32_t *hist, float *amp, void *stream);

/*
 * Signatures from an already gathered CSR (output of ar_roi_gather) with the
 * plain per-launch kernel: one workgroup per (ROI, direction tile).
 *   rel      device float [total][4], offsets device int64 [n_roi+1]
 * Other arguments as araullo_signatures.  Does not synchronise.
 */
ar_status araullo_signatures_csr(ar_context *ctx, const float *rel, const int64_t *offsets,
                                 int64_t n_roi, float radius, const float *directions,
                                 int32_t n_dir, int32_t nbins, const int32_t *windows,
                                 int32_t n_win, float *images, void *stream);

/*
 * Batched signatures for ROIs of uneven atom counts (e.g. clipped at the
 * specimen surface): one persistent launch whose workgroups pull
 * (ROI, direction-chunk) items, largest ROIs first, from a device queue
 * (the paper's scaling limits came from load imbalance, supplement,
 * "Scalability limits").  A plan fixes the shapes, holds its workspace,
 * tunes its tile shape on first use (ar_signature_plan_tune) and replays the
 * whole batch as one captured HIP graph.
 *   max_roi, max_total  capacity of the plan (ROIs, gathered atoms)
 * The run call takes a gathered CSR (ar_roi_gather) and writes the same
 * images as araullo_signatures_csr, bit for bit.
 */
ar_status ar_signature_plan_create(ar_context *ctx, int64_t max_roi, int64_t max_total,
                                   int32_t n_dir, int32_t nbins, int32_t n_win, ar_plan **out);
ar_status ar_signature_plan_destroy(ar_plan *plan);
/* Time the candidate tile shapes on the given batch and keep the fastest.
 * Writes images as a side effect. Synchronises. */
ar_status ar_signature_plan_tune(ar_plan *plan, const float *rel, const int64_t *offsets,
                                 int64_t n_roi, float radius, const float *directions,
                                 const int32_t *windows, float *images, void *stream);
/* Chosen configuration (any out pointer may be NULL): directions per work
 * item, atoms per LDS stage, workgroups launched per compute unit, and the
 * register form (1: as allocated, 4: at most 128 VGPRs per lane so four
 * wavefronts share a SIMD). */
ar_status ar_signature_plan_config(const ar_plan *plan, int32_t *dirs_per_item,
                                   int32_t *atoms_per_stage, int32_t *blocks_per_cu,
                                   int32_t *min_waves);
/* Pin a configuration instead of tuning: directions per work item
 * (1..n_dir), atoms per LDS stage (a multiple of 256 in [256, 4096]; larger
 * ROIs are streamed through it), workgroups per compute unit (1..16) and
 * min_waves 1, or 4 for nbins <= 1024. */
ar_status ar_signature_plan_set_config(ar_plan *plan, int32_t dirs_per_item, int32_t atoms_per_stage,
                                       int32_t blocks_per_cu, int32_t min_waves);
/* Run the batch. The host reads roi sizes once per new `offsets` pointer or
 * n_roi to order the queue (synchronises then); with use_graph != 0 the
 * launch sequence is captured once per argument set and replayed. */
ar_status ar_signature_plan_run(ar_plan *plan, const float *rel, const int64_t *offsets,
                                int64_t n_roi, float radius, const float *directions,
                                const int32_t *windows, float *images, int32_t use_graph,
                                void *stream);

/*
 * Indexing library (Sec. 2.4; supplement, "Indexing algorithm"): rotated
 * reference images, normalised individually by their maximum over the
 * directions of each window (an all-zero image stays zero), kept as a BF16
 * copy for the correlation plus per-entry squared norms of that copy and
 * per-(entry, window) reciprocal maxima for the FP32 rescoring.
 *   ref_images device float [n_lib][n_win][n_dir]; must stay valid and
 *              unchanged while the library exists (FP32 rescoring reads it)
 *   n_win * n_dir at most 4194240 (a 256-row panel of BF16 rows stays
 *              below 2 GiB); larger gives AR_EINVAL
 * The library owns its BF16 copy; destroy frees it.
 */
ar_status ar_library_create(ar_context *ctx, const float *ref_images, int64_t n_lib,
                            int32_t n_win, int32_t n_dir, void *stream, ar_library **out);
/*
 * As ar_library_create, and the library also keeps the orientation and the
 * phase of every entry (Sec. 2.4 and the supplement's indexing paragraph:
 * each reference image is the phase's reference rotated into one test
 * orientation), so that indexing results can be reported as orientations:
 *   quats      device double [n_lib][4] (w, x, y, z), copied
 *   phase      device int32 [n_lib], copied
 * Entry l of ref_images must be the reference of phase[l] rotated by
 * quats[l] (e.g. from ar_rotate_reference with the same arrays).
 */
ar_status ar_library_prepare(ar_context *ctx, const float *ref_images, int64_t n_lib, int32_t n_win,
                             int32_t n_dir, const double *quats, const int32_t *phase, void *stream,
                             ar_library **out);
/*
 * Orientation and phase of library entries, e.g. of the top_idx of an
 * indexing call: quats[i] = quaternion of entry idx[i], phase[i] = its
 * phase; an index of -1 (no candidate) or out of range gives a NaN
 * quaternion and phase -1.
 *   idx    device int32 [n];  quats device double [n][4] or NULL, out;
 *   phase  device int32 [n] or NULL, out
 * AR_EINVAL for a library made by ar_library_create.  Does not synchronise.
 */
ar_status ar_library_lookup(const ar_library *lib, const int32_t *idx, int64_t n, double *quats,
                            int32_t *phase, void *stream);
ar_status ar_library_destroy(ar_library *lib);

/*
 * Orientation indexing: the k library entries with the smallest sum of
 * squared differences of the normalised images (supplement, Eq. S1, taken
 * over all nodes of all windows),
 *   Delta(r,l) = sum_{w,v} (S_r[w][v]/max_v S_r[w] - L_l[w][v]/max_v L_l[w])^2.
 * Candidates come from a BF16-input / FP32-accumulate MFMA correlation
 * (score = |L_l|^2 - 2 <S_r, L_l>) keeping the best `cand` (16 for
 * k <= 16, 32 for k <= 32, else 64) per ROI, which are then rescored in
 * FP32 from the FP32 images; the output is sorted ascending by (FP32 Delta,
 * library index).  The paper keeps many near-best solutions per ROI (Sec.
 * 3.2); k up to 64 returns that many.  Entries past the library's size
 * (k > n_lib) hold index -1 and Delta +inf.
 *   images    device float [n_roi][n_win][n_dir] (raw signatures)
 *   k         1 .. 64 outputs per ROI
 *   top_idx   device int32 [n_roi][k], out
 *   top_score device float [n_roi][k], out: FP32 Delta
 * Does not synchronise.
 */
ar_status index_orientations(ar_context *ctx, const float *images, int64_t n_roi,
                             const ar_library *lib, int32_t k, int32_t *top_idx, float *top_score,
                             void *stream);

/* As index_orientations with an explicit candidate count `cand` (16, 32 or
 * 64, k <= cand; index_orientations uses the smallest that holds k),
 * optionally returning the BF16-stage candidates before rescoring.
 *   cand_idx  device int32 [n_roi][cand] or NULL, out */
ar_status index_orientations_ex(ar_context *ctx, const float *images, int64_t n_roi,
                                const ar_library *lib, int32_t k, int32_t cand, int32_t *top_idx,
                                float *top_score, int32_t *cand_idx, void *stream);

/* Correlation tile of this context's index calls: a workgroup of `waves`
 * wavefronts (4 as a 2x2 grid, 8 as 2x4), each owning wtm x wtn MFMA tiles of
 * 32x32 (workgroup tile 64 wtm x 32 wtn (waves/2)); K advances bk = 32 per
 * step.  Supported (waves, wtm, wtn, bk): (4,2,2,32) (4,2,4,32) (4,4,2,32)
 * (4,4,4,32) (8,2,2,32) (8,4,2,32).  (0,0,0,0) returns to the default choice: (8,4,2,32),
 * a 256 x 256 tile, for 16 candidates and (8,2,2,32), 128 x 256, for 32 and
 * 64 (whose candidate lists would spill beside the larger tile's
 * accumulators).  Results do not depend on the tile: every score accumulates
 * K in the same order.
 * Returns AR_EINVAL for an unsupported tile. */
ar_status ar_index_set_tile(ar_context *ctx, int32_t waves, int32_t wtm, int32_t wtn, int32_t bk);

/*
 * Sparse indexing (supplement, "Indexing algorithm", Eq. S1 over the n_hat
 * strongest reference entries, look-up costs O_lu and O_idx of the
 * complexity paragraph).  The look-up table, per phase c:
 *   - the reference image of c is normalised per window, key = x / max in
 *     FP64 (an all-zero window gives 0); its n_hat entries (w, v) with the
 *     largest key, equal keys by the lower flat index w * n_dir + v, form the
 *     strong list (decreasing key), with values R_i = (float)key;
 *   - for every orientation g of phase c and strong entry i the node
 *     p(g, i) = argmax_u n_u . (R(q_g) n_{v_i}) (FP32 ranking, re-ranked in
 *     FP64 within 1e-5 of the best, ties to the lower index).
 *   reference   device float [n_phase][n_win][n_dir], finite, read during the call only
 *   directions  device float [n_dir][3] unit mesh normals, n_dir <= 65535
 *   quats       device double [n_lib][4] (w, x, y, z); the entries of phase c
 *               are the consecutive rows after those of phases 0 .. c-1
 *   phase_count host int64 [n_phase]: entries per phase (sum = n_lib >= 1)
 *   n_hat       1 .. min(n_win * n_dir, 65535)
 * The table owns copies of everything it needs (2 * n_lib * n_hat bytes of
 * node ids in each of two layouts); destroy frees them.
 */
ar_status ar_sparse_lut_create(ar_context *ctx, const float *reference, int32_t n_phase, int32_t n_win,
                               const float *directions, int32_t n_dir, const double *quats,
                               const int64_t *phase_count, int32_t n_hat, void *stream,
                               ar_sparse_lut **out);
ar_status ar_sparse_lut_destroy(ar_sparse_lut *lut);
/* Copy out the strong lists and the table (any pointer may be NULL):
 *   strong_idx device int32 [n_phase][n_hat]: w * n_dir + v, decreasing key
 *   strong_val device float [n_phase][n_hat]: R_i
 *   nodes      device int32 [n_lib][n_hat]: p(g, i) */
ar_status ar_sparse_lut_export(const ar_sparse_lut *lut, int32_t *strong_idx, float *strong_val,
                               int32_t *nodes, void *stream);
/* The screen the table's mesh gets, as ROIs per LDS read (host int32, out):
 * 8 (8-bit codes, when the 8-ROI window slab and the phase's reference codes
 * fit the LDS of one workgroup), else 2 or 1 (FP16). */
ar_status ar_sparse_lut_screen(const ar_sparse_lut *lut, int32_t *rois_per_read);

/*
 * The k library entries with the smallest sparse Eq. S1
 *   Delta(r, g) = sum_i (S_r[w_i][p(g, i)] / max_v S_r[w_i] - R_i)^2
 * (w_i the window of strong entry i of g's phase).  A screen keeps 16
 * (k <= 16) or 32 candidates per ROI and chunk of orientations: in 8-bit
 * codes round(255 x) of the normalised image and of R_i with exact integer
 * sums, or (meshes too large for that) in FP16 values with FP32
 * accumulation.  The merged candidates are rescored in FP32 from the FP32
 * image; the output is sorted ascending by (FP32 Delta, library index).
 *   images    device float [n_roi][n_win][n_dir] (raw signatures), n_roi >= 1
 *   k         1 .. 32
 *   top_idx   device int32 [n_roi][k], out;  top_score device float [n_roi][k], out
 * Does not synchronise.
 */
ar_status index_orientations_sparse(ar_context *ctx, const float *images, int64_t n_roi,
                                    const ar_sparse_lut *lut, int32_t k, int32_t *top_idx,
                                    float *top_score, void *stream);

/*
 * Reciprocal-space signatures on a cubic grid (Sec. 2.2, FSP paragraph,
 * Eq. (2); supplement, reciprocal-space cost O(N_roi N_w L^3)):
 *   amp[r][a][b][c] = |sum_w exp(-2 pi i k . d_w)|,
 *   k = ((a - L/2), (b - L/2), (c - L/2)) * dk,  dk = 2 k_max / L,
 * over the gathered relative coordinates d_w of ROI r (k in cycles per
 * length unit of the coordinates; the origin a = b = c = L/2 holds N_w).
 * Evaluated as one complex GEMM per ROI on FP32 matrix cores.
 *   rel, offsets  gathered CSR (ar_roi_gather)
 *   L             multiple of 32 in [32, 512]
 *   k_max         > 0 (the grid covers [-k_max, k_max - dk] per axis)
 *   amp           device float [n_roi][L][L][L], out
 * AR_EINVAL if n_roi * L^3 / 4096 workgroups exceed 2^31 - 1.  Does not
 * synchronise.
 */
ar_status ar_fsp_amplitudes(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                            int32_t L, float k_max, float *amp, void *stream);

/*
 * Adaptive ROI-grid refinement (Sec. 3.5, aluminium bicrystal: a coarse
 * cubic ROI grid, then a local octree-like refinement where the signal is
 * strong; supplement, local grid refinement).  Coarse ROI r has atom count
 * counts[r] = N_r and images img[r][w][v]; its intensity in window w is
 * I = max_v img[r][w][v] / N_r (0 if N_r = 0).  ROI r is kept iff for some
 * window w with bit w of window_mask set, I[r][w] >= kappa * max_r' I[r'][w]
 * (FP32).  Every kept ROI's grid cell (edge h, centred on the ROI) is split
 * into split^3 cells whose centres are written, ordered by kept ROI, then x,
 * y, z sub-cell: c + h (2i + 1 - split) / (2 split) per axis (the offset
 * evaluated in FP64 and rounded to FP32, the sum in FP32).
 *   centres      device float [n_roi][3];  images device float [n_roi][n_win][n_dir]
 *   counts       device int32 [n_roi]
 *   n_win        1 .. 32;  split 1 .. 16
 *   out_centres  device float [cap][3], out;  out_parent device int32 [cap] or NULL, out
 *   n_out        host int64, out: refined ROIs (kept * split^3)
 * AR_EINVAL if cap < n_out (n_out is still written).  Synchronises.
 */
ar_status ar_refine_roi_grid(ar_context *ctx, const float *centres, const float *images,
                             const int32_t *counts, int64_t n_roi, int32_t n_win, int32_t n_dir,
                             uint32_t window_mask, float kappa, float h, int32_t split,
                             float *out_centres, int32_t *out_parent, int64_t cap, int64_t *n_out,
                             void *stream);

/*
 * Disorientation angle in degrees under cubic symmetry (supplement,
 * "Creation of test orientations": the misorientation with the smallest
 * rotation angle among the symmetrically equivalent ones), FP64:
 *   deg[i] = 2 acos(min(1, max_S |(qa_i^-1 * qb_i * S).w|)) * 180/pi
 * over the 24 proper rotations S of m-3m.  Quaternions (w, x, y, z),
 * need not be normalised.
 *   qa, qb device double [n][4];  deg device double [n], out
 */
ar_status ar_disorientation_cubic(const double *qa, const double *qb, int64_t n, double *deg,
                                  void *stream);

/*
 * Rotated reference images (supplement, "Indexing algorithm": rotated nodes
 * are replaced by their closest neighbouring mesh node):
 *   out[l][w][v] = reference[phase[l]][w][u*],
 *   u* = argmax_u n_u . (R(q_l)^T n_v)   (ties to the lower index).
 * Candidates are ranked in FP32 and those within 1e-5 of the best re-ranked
 * in FP64.
 *   reference  device float [n_phase][n_win][n_dir]
 *   directions device float [n_dir][3]
 *   quats      device double [n_lib][4] (w, x, y, z), phase device int32 [n_lib]
 *              (values in [0, n_phase); a value outside is clamped)
 *   out        device float [n_lib][n_win][n_dir]
 */
ar_status ar_rotate_reference(ar_context *ctx, const float *reference, int32_t n_phase, int32_t n_win,
                              const float *directions, int32_t n_dir, const double *quats,
                              const int32_t *phase, int64_t n_lib, float *out, void *stream);

/*
 * Structure-factor matching score and its gradient with respect to the ROI
 * orientation quaternion, built on the direct Fourier transform of Eq. (2)
 * (Sec. 2.2, FSP paragraph) evaluated on spherical shells |k| = f_w along
 * the rotated mesh directions u_v = R(q/|q|) n_v:
 *   F_{w,v} = sum_j exp(-2 pi i f_w u_v . x_j),  A = |F| / N_w,
 *   J(q) = sum_{w,v} (A_{w,v} - T_{p,w,v})^2,   p = phase of the ROI,
 *   grad = dJ/dq (4-vector, orthogonal to q).
 * Terms with |F| < 1e-12 N_w add nothing to the gradient.
 *   rel, offsets  gathered CSR (ar_roi_gather)
 *   quats         device float [n_roi][4]
 *   phase         device int32 [n_roi], values in [0, n_phase) (a value
 *                 outside is clamped to that range; nothing is read out of
 *                 bounds)
 *   freqs         device float [n_phase][n_freq]
 *   targets       device float [n_phase][n_freq][n_dir]
 *   score         device float [n_roi], out
 *   grad          device float [n_roi][4] or NULL, out (NULL: forward only)
 * n_freq in [1, 8].  Domain: the phase f_w (u_v . x_j), in turns, goes to
 * the hardware sine and cosine without range reduction, which are specified
 * for |phase| <= 256 turns; their argument carries a rounding error of about
 * |phase| 2^-24 turns, so max|f| max|x| must stay at or below 256 (the
 * Python binding checks it; at f = 10 nm^-1 and R = 2 nm it is 20).  The
 * same holds for ar_sf_amplitudes and ar_refine_orientations; the FP64
 * forward reduces its phases exactly.  Does not synchronise.
 */
ar_status ar_sf_score_grad(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                           const float *quats, const int32_t *phase, const float *directions,
                           int32_t n_dir, const float *freqs, const float *targets, int32_t n_phase,
                           int32_t n_freq, float *score, float *grad, void *stream);

/*
 * ar_sf_score_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or refinement loops, harnesses that
 * forbid allocation): the same kernels, results bit-identical to
 * ar_sf_score_grad, but the workspace (the direction evaluation list and
 * the per-tile partial sums) lives in one fixed 32 MiB device array per GPU
 * that the library holds until the process ends.  The call makes no device
 * allocation or free.  Arguments, layouts and domain as ar_sf_score_grad;
 * the caller owns every buffer passed.
 * Limit: 4 (3 n_dir + 1) rounded up to 256, plus 40 n_roi ceil(n_dir / 256),
 * bytes must fit 32 MiB (about 19800 ROIs at 10242 directions); a larger
 * call returns AR_EINVAL and writes nothing.  The array's device address is
 * looked up by ar_context_create for its device.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (nothing in it needs clearing: each call writes what it reads), so
 * calls that overlap on one GPU (different streams, or other threads,
 * without ordering between them) race: order them on one stream.
 */
ar_status ar_sf_score_grad_noalloc(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                                   const float *quats, const int32_t *phase, const float *directions,
                                   int32_t n_dir, const float *freqs, const float *targets, int32_t n_phase,
                                   int32_t n_freq, float *score, float *grad, void *stream);

/* FP64 forward of the same score (for finite-difference checks):
 *   quats device double [n_roi][4]; score device double [n_roi], out. */
ar_status ar_sf_score_f64(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                          const double *quats, const int32_t *phase, const float *directions,
                          int32_t n_dir, const double *freqs, const double *targets, int32_t n_phase,
                          int32_t n_freq, double *score, void *stream);

/* Structure-factor amplitudes A[r][w][v] (FP32) for given orientations,
 * e.g. to build targets from reference crystals.
 *   amp device float [n_roi][n_freq][n_dir], out; freqs per ROI's phase. */
ar_status ar_sf_amplitudes(ar_context *ctx, const float *rel, const int64_t *offsets, int64_t n_roi,
                           const float *quats, const int32_t *phase, const float *directions,
                           int32_t n_dir, const float *freqs, int32_t n_phase, int32_t n_freq,
                           float *amp, void *stream);

/*
 * Orientation refinement below the library grid: `steps` iterations of
 * projected gradient descent on J (ar_sf_score_grad) with a per-ROI
 * backtracking step along the normalised gradient: a trial
 * q' = normalise(q - a g/|g|) is accepted iff J(q') <= J(q) - 1e-4 a |g|,
 * then a grows by 1.5; otherwise a halves and q stays.  steps + 1
 * evaluations at the trial points of all ROIs (the first at the start):
 * J and its gradient, except the last, which only decides acceptance and
 * takes J alone.
 *   quats  device float [n_roi][4], in: start, out: refined
 *   a0     starting step (quaternion arc length, e.g. 0.01)
 *   score  device float [n_roi] or NULL, out: final J
 * Does not synchronise.
 */
ar_status ar_refine_orientations(ar_context *ctx, const float *rel, const int64_t *offsets,
                                 int64_t n_roi, float *quats, const int32_t *phase,
                                 const float *directions, int32_t n_dir, const float *freqs,
                                 const float *targets, int32_t n_phase, int32_t n_freq,
                                 int32_t steps, float a0, float *score, void *stream);

/*
 * Measured peak rates of the units the kernels are bound by, the
 * denominators of their roofline fractions (not part of the method).  Each
 * probe is a fixed loop on eight workgroups per compute unit, timed on the
 * null stream after one warm-up launch:
 *   out[AR_PEAK_HBM_BYTES]        device copy, bytes read + written per second (1 GiB each way)
 *   out[AR_PEAK_LDS_BYTES]        16-byte LDS reads without bank conflicts, bytes per second
 *   out[AR_PEAK_LDS_ATOMICS]      LDS integer atomics without return, one bank per lane, per second
 *   out[AR_PEAK_FP32_FMA_FLOPS]   non-packed FP32 FMA, flop per second (FMA = 2)
 *   out[AR_PEAK_SIN]              v_sin_f32 per second
 *   out[AR_PEAK_SIN_OVERLAP]      time of 16 FMA chains / time of the same with 4 sin chains beside
 *                                 them (1 = the transcendental unit runs beside the FMA pipeline)
 *   out[AR_PEAK_BF16_MFMA_FLOPS]  v_mfma_f32_32x32x16_bf16, flop per second
 *   out[AR_PEAK_FP32_MFMA_FLOPS]  v_mfma_f32_32x32x2_f32, flop per second
 *   out[AR_PEAK_LDS_GATHER8]      8-byte LDS reads at pseudo-random addresses of a 64 KB table
 *                                 (the look-up gather pattern, bank conflicts included), lane reads per second
 *   out    host double [n_out], n_out >= AR_PEAK_COUNT
 * Allocates 2 GiB of device memory for the copy and frees it.  Synchronises.
 */
enum {
    AR_PEAK_HBM_BYTES = 0,
    AR_PEAK_LDS_BYTES = 1,
    AR_PEAK_LDS_ATOMICS = 2,
    AR_PEAK_FP32_FMA_FLOPS = 3,
    AR_PEAK_SIN = 4,
    AR_PEAK_SIN_OVERLAP = 5,
    AR_PEAK_BF16_MFMA_FLOPS = 6,
    AR_PEAK_LDS_GATHER8 = 7,
    AR_PEAK_FP32_MFMA_FLOPS = 8,
    AR_PEAK_COUNT = 9
};
ar_status ar_measure_peaks(ar_context *ctx, double *out, int32_t n_out);

#ifdef __cplusplus
}
#endif

#endif /* ARAULLO_H */
