/*
 * Reference oracle for the real-space (Araullo-Peters style) signature and
 * indexing method of Kuehbach, Kasemer, Gault, Breen, "On Open and
 * Strong-Scaling Tools for Atom Probe Crystallography" (arXiv 2009.00735).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded-per-item C that
 * writes each definition out directly so that it can be checked against the
 * paper by eye.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library; the product path never does.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Floating point: FP64 wherever the paper leaves the precision open, FP32 only
 * where the paper's single precision decides an integer (ROI membership and
 * the Eq. (1) bin index), with an explicit fmaf order and no contraction
 * (compile with -ffp-contract=off, no fast-math).
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  R1  Eq. (1): Delta R is the bin width, so 2^m bins span
 *      [-(R + dR), R + dR] and dR = R / (2^(m-1) - 1)  (Sec. 2.2, Eq. (1);
 *      Fig. 2 caption; supplement "Controlled windowing of the SDMs", one
 *      zero-count pad bin on each side).
 *  R2  FP32 evaluation order of Eq. (1): s = fmaf(vz,dz,fmaf(vy,dy,vx*dx)),
 *      t = (s + shift) * scale with shift = (float)(R + dR) and
 *      scale = (float)(2^m / (2R + 2dR)) rounded once from FP64,
 *      b = floor(t) clamped to [0, 2^m - 1].  The paper names single
 *      precision (supplement, "Sequential implementation tricks") but no
 *      evaluation order.
 *  R3  ROI membership |p - c| <= R in FP32: d = p - c,
 *      fmaf(dz,dz,fmaf(dy,dy,dx*dx)) <= (float)(R*R).
 *  R4  amplitude spectrum = |unnormalised DFT| of the histogram, one-sided
 *      k = 0 .. 2^m/2, so that A_0 equals the atom count (Sec. 3.1: the peak
 *      at the origin accounts for all atoms of the ROI).
 *  R5  window of a spacing interval [d_min, d_max]: DFT indices k with
 *      ceil(L/d_max) <= k <= floor(L/d_min), L = 2R + 2dR (Fig. 2 caption:
 *      bin b = floor(f L) for a reciprocal spacing f; supplement,
 *      reconstruction parameters: the 1.823-2.230 A interval).
 *  R6  image value = maximum amplitude inside the window (supplement,
 *      reconstruction parameters: the strongest amplitude among the window's
 *      bins is kept).
 *  R7  normalisation = division by the image maximum over the directions,
 *      all-zero images stay zero (Sec. 2.4 and supplement "Indexing
 *      algorithm": images normalised individually).
 *  R8  dense reading of Eq. S1: the sum of squared differences runs over all
 *      nodes of all windows instead of the 1000 strongest reference nodes.
 *  R9  disorientation: smallest rotation angle among the 24 proper cubic
 *      symmetry variants of the misorientation (supplement, "Creation of test
 *      orientations": cubic symmetry, fundamental zone, smallest angle).
 *  R10 rotated reference: the value at lab node v is the reference value at
 *      the mesh node closest to R(q)^T n_v (supplement, "Indexing algorithm":
 *      rotated nodes mapped to their closest neighbouring node).
 *  R11 structure-factor score: Eq. (2) evaluated on spherical shells
 *      |k| = f_w along rotated mesh directions; A = |F| / N_w and
 *      J(q) = sum (A - T)^2.  This refinement score is not in the paper; it is
 *      built on Eq. (2) (Sec. 2.2, FSP paragraph).
 *  R12 sparse form of Eq. S1 (supplement, "Indexing algorithm"; cost O_idx
 *      in the complexity paragraph): per phase, the reference image is
 *      normalised per window (R7) and its n_hat entries (window w, node v)
 *      with the largest normalised value are kept, in decreasing order (the
 *      value is the FP64 quotient x / max of the FP32 inputs; equal values
 *      keep the lower flat index w * n_dir + v first).  For orientation q the
 *      look-up node of entry i is the mesh node closest to R(q) n_{v_i}
 *      (largest dot product in FP64, ties to the lower index) and
 *      Delta(r, q) = sum_i (S^_r[w_i][p(q, i)] - Ref^[w_i][v_i])^2.  The
 *      window of the strong entry is carried along (the paper has one window
 *      per signature).  R(q) rather than R(q)^T: a reference feature at node
 *      u appears at R(q) n_u in the image rotated as in R10.
 *  R13 sub-lattice signatures (Sec. 3.1, the Al3Sc discussion; supplement,
 *      Al-Li-Mg specimens): the signature of a set of atom types is the
 *      signature computed from the atoms of those types only (the selection
 *      itself lives in the NumPy front end, signatures_typed).
 *  R14 reciprocal-space signatures on a cubic grid (Sec. 2.2, FSP paragraph,
 *      Eq. (2); supplement, reciprocal-space costs): amp(k) = |sum_w
 *      exp(-2 pi i k . d_w)| at the L^3 points k = (a - L/2, b - L/2,
 *      c - L/2) * dk, dk = 2 k_max / L, a, b, c in [0, L) (k in cycles per
 *      length unit, the origin on the grid).  The paper's k in [-2 pi, 2 pi]^3
 *      is read as 2 pi k with |k| <= 1 per Angstrom, i.e. k_max = 10 per nm.
 *  R15 adaptive ROI-grid refinement (Sec. 3.5, aluminium bicrystal;
 *      supplement, local grid refinement): the intensity of coarse ROI r in
 *      window w is I[r][w] = max_v img[r][w][v] / N_r (0 for an empty ROI),
 *      the per-atom peak amplitude.  The kappa threshold on normalised
 *      intensity is read against the distribution over all coarse ROIs: r
 *      is kept iff for a selected window I[r][w] >= kappa * max_r' I[r'][w].
 *      Each kept ROI's
 *      grid cell (edge h, centred on the ROI) is split into s^3 cells
 *      (s = 5 in the main text; the supplement's 0.5 nm and 64x imply 4)
 *      whose centres c + h (2i + 1 - s) / (2s) are the refined ROIs, in
 *      order (kept ROI, i along x, j along y, k along z); each offset is
 *      evaluated in FP64, rounded to FP32 and added in FP32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------------- */
/* Eq. (1) constants (reading R1/R2)                                        */
/* ---------------------------------------------------------------------- */
void orc_bin_constants(float radius, int32_t nbins, float *shift, float *scale, double *bin_width)
{
    double R = (double)radius;
    double dR = R / (double)(nbins / 2 - 1);
    *shift = (float)(R + dR);
    *scale = (float)((double)nbins / (2.0 * R + 2.0 * dR));
    if (bin_width) *bin_width = dR;
}

/* Reading R5.  Returns 0 on success, -1 when the window holds no index or
 * leaves [1, nbins/2]. */
int orc_window_bins(double radius, int32_t nbins, double d_min, double d_max, int32_t *k_lo, int32_t *k_hi)
{
    double dR = radius / (double)(nbins / 2 - 1);
    double L = 2.0 * radius + 2.0 * dR;
    double lo = ceil(L / d_max);
    double hi = floor(L / d_min);
    *k_lo = (int32_t)lo;
    *k_hi = (int32_t)hi;
    if (!(d_min > 0.0) || !(d_max >= d_min)) return -1;
    if (lo > hi || lo < 1.0 || hi > (double)(nbins / 2)) return -1;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* ROI query (reading R3), brute force over every atom                      */
/* ---------------------------------------------------------------------- */
static int orc_in_roi(const float *p, const float *c, float R2, float *d)
{
    float dx = p[0] - c[0];
    float dy = p[1] - c[1];
    float dz = p[2] - c[2];
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    d[0] = dx; d[1] = dy; d[2] = dz;
    return r2 <= R2;
}

/* Relative coordinates of every atom inside the ROI, in atom order.
 * Writes at most `cap` rows to rel (may be NULL); returns the count. */
int64_t orc_roi_gather(const float *positions, int64_t n_atoms, const float *centre, float radius,
                       float *rel, int64_t cap)
{
    float R2 = (float)((double)radius * (double)radius);
    int64_t n = 0;
    for (int64_t i = 0; i < n_atoms; ++i) {
        float d[3];
        if (orc_in_roi(positions + 3 * i, centre, R2, d)) {
            if (rel && n < cap) { rel[3 * n] = d[0]; rel[3 * n + 1] = d[1]; rel[3 * n + 2] = d[2]; }
            ++n;
        }
    }
    return n;
}

/* ---------------------------------------------------------------------- */
/* Eq. (1): one spatial distribution map (histogram) per direction          */
/* ---------------------------------------------------------------------- */
void orc_sdm_hist(const float *rel, int64_t n_w, const float *v, float radius, int32_t nbins, int32_t *hist)
{
    float shift, scale;
    orc_bin_constants(radius, nbins, &shift, &scale, NULL);
    memset(hist, 0, sizeof(int32_t) * (size_t)nbins);
    for (int64_t i = 0; i < n_w; ++i) {
        const float *d = rel + 3 * i;
        float s = fmaf(v[2], d[2], fmaf(v[1], d[1], v[0] * d[0]));
        float t = (s + shift) * scale;
        float f = fminf(fmaxf(floorf(t), 0.0f), (float)(nbins - 1));
        hist[(int32_t)f] += 1;
    }
}

/* ---------------------------------------------------------------------- */
/* Reading R4: amplitudes of the unnormalised DFT, by its definition         */
/* X_k = sum_n h_n exp(-2 pi i k n / N), with k n reduced mod N exactly.     */
/* ---------------------------------------------------------------------- */
typedef struct { int32_t n; double *c; double *s; } orc_twiddles;

static void orc_twiddles_make(orc_twiddles *t, int32_t n)
{
    t->n = n;
    t->c = (double *)malloc(sizeof(double) * (size_t)n);
    t->s = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t j = 0; j < n; ++j) {
        t->c[j] = cos(2.0 * ORC_PI * (double)j / (double)n);
        t->s[j] = sin(2.0 * ORC_PI * (double)j / (double)n);
    }
}

static void orc_twiddles_free(orc_twiddles *t) { free(t->c); free(t->s); }

static double orc_dft_amp(const int32_t *hist, const orc_twiddles *t, int32_t k)
{
    int32_t N = t->n;
    double re = 0.0, im = 0.0;
    for (int32_t n = 0; n < N; ++n) {
        if (!hist[n]) continue;
        int32_t j = (int32_t)(((int64_t)k * (int64_t)n) % N);
        re += (double)hist[n] * t->c[j];
        im -= (double)hist[n] * t->s[j];
    }
    return sqrt(re * re + im * im);
}

/* Full one-sided amplitude spectrum, amp[0 .. nbins/2]. */
void orc_amplitudes(const int32_t *hist, int32_t nbins, double *amp)
{
    orc_twiddles t;
    orc_twiddles_make(&t, nbins);
    for (int32_t k = 0; k <= nbins / 2; ++k) amp[k] = orc_dft_amp(hist, &t, k);
    orc_twiddles_free(&t);
}

/* ---------------------------------------------------------------------- */
/* Signatures: images[r][w][v] = max_{k in window w} A_k (readings R5, R6)   */
/* ---------------------------------------------------------------------- */
void orc_signatures(const float *positions, int64_t n_atoms, const float *centres, int64_t n_roi,
                    float radius, const float *dirs, int32_t n_dir, int32_t nbins,
                    const int32_t *windows, int32_t n_win, double *images, int32_t *counts,
                    int32_t n_threads)
{
    orc_twiddles t;
    orc_twiddles_make(&t, nbins);
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int64_t r = 0; r < n_roi; ++r) {
        int64_t n_w = orc_roi_gather(positions, n_atoms, centres + 3 * r, radius, NULL, 0);
        float *rel = (float *)malloc(sizeof(float) * 3 * (size_t)(n_w > 0 ? n_w : 1));
        orc_roi_gather(positions, n_atoms, centres + 3 * r, radius, rel, n_w);
        int32_t *hist = (int32_t *)malloc(sizeof(int32_t) * (size_t)nbins);
        if (counts) counts[r] = (int32_t)n_w;
        for (int32_t v = 0; v < n_dir; ++v) {
            orc_sdm_hist(rel, n_w, dirs + 3 * v, radius, nbins, hist);
            for (int32_t w = 0; w < n_win; ++w) {
                double best = 0.0;
                for (int32_t k = windows[2 * w]; k <= windows[2 * w + 1]; ++k) {
                    double a = orc_dft_amp(hist, &t, k);
                    if (a > best) best = a;
                }
                images[((size_t)r * n_win + w) * n_dir + v] = best;
            }
        }
        free(hist);
        free(rel);
    }
    orc_twiddles_free(&t);
}

/* Histograms and full spectra for one ROI given as relative coordinates. */
void orc_sdm_debug(const float *rel, int64_t n_w, float radius, const float *dirs, int32_t n_dir,
                   int32_t nbins, int32_t *hist_out, double *amp_out)
{
    orc_twiddles t;
    orc_twiddles_make(&t, nbins);
    int32_t *hist = (int32_t *)malloc(sizeof(int32_t) * (size_t)nbins);
    for (int32_t v = 0; v < n_dir; ++v) {
        orc_sdm_hist(rel, n_w, dirs + 3 * v, radius, nbins, hist);
        if (hist_out) memcpy(hist_out + (size_t)v * nbins, hist, sizeof(int32_t) * (size_t)nbins);
        if (amp_out)
            for (int32_t k = 0; k <= nbins / 2; ++k)
                amp_out[(size_t)v * (nbins / 2 + 1) + k] = orc_dft_amp(hist, &t, k);
    }
    free(hist);
    orc_twiddles_free(&t);
}

/* ---------------------------------------------------------------------- */
/* Indexing (readings R7, R8): Eq. S1 over all nodes, FP64                  */
/* ---------------------------------------------------------------------- */
void orc_normalise(const float *images, int64_t n, int32_t n_win, int32_t n_dir, double *out)
{
    for (int64_t r = 0; r < n; ++r)
        for (int32_t w = 0; w < n_win; ++w) {
            const float *src = images + ((size_t)r * n_win + w) * n_dir;
            double *dst = out + ((size_t)r * n_win + w) * n_dir;
            double m = 0.0;
            for (int32_t v = 0; v < n_dir; ++v) if ((double)src[v] > m) m = (double)src[v];
            for (int32_t v = 0; v < n_dir; ++v) dst[v] = m > 0.0 ? (double)src[v] / m : 0.0;
        }
}

/* For every ROI row of S: the k library rows of L with the smallest
 * Delta = sum_j (S_j - L_j)^2, ascending by (Delta, library index). */
void orc_index_topk(const double *S, int64_t n_roi, const double *L, int64_t n_lib, int64_t K,
                    int32_t k, int32_t *top_idx, double *top_score, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int64_t r = 0; r < n_roi; ++r) {
        const double *s = S + (size_t)r * K;
        int32_t *bi = top_idx + (size_t)r * k;
        double *bs = top_score + (size_t)r * k;
        int32_t filled = 0;
        for (int64_t l = 0; l < n_lib; ++l) {
            const double *x = L + (size_t)l * K;
            double delta = 0.0;
            for (int64_t j = 0; j < K; ++j) { double e = s[j] - x[j]; delta += e * e; }
            /* insertion into the sorted list; equal Delta keeps the lower index first */
            int32_t pos = filled;
            while (pos > 0 && bs[pos - 1] > delta) --pos;
            if (pos >= k) continue;
            int32_t last = filled < k ? filled : k - 1;
            for (int32_t m = last; m > pos; --m) { bs[m] = bs[m - 1]; bi[m] = bi[m - 1]; }
            bs[pos] = delta; bi[pos] = (int32_t)l;
            if (filled < k) ++filled;
        }
        for (int32_t m = filled; m < k; ++m) { bs[m] = INFINITY; bi[m] = -1; }
    }
}

/* Delta for explicit (roi, library) pairs. */
void orc_ssd_pairs(const double *S, const double *L, int64_t K, const int64_t *roi, const int64_t *lib,
                   int64_t n_pairs, double *out)
{
    for (int64_t p = 0; p < n_pairs; ++p) {
        const double *s = S + (size_t)roi[p] * K;
        const double *x = L + (size_t)lib[p] * K;
        double delta = 0.0;
        for (int64_t j = 0; j < K; ++j) { double e = s[j] - x[j]; delta += e * e; }
        out[p] = delta;
    }
}

/* ---------------------------------------------------------------------- */
/* Quaternions (w, x, y, z), active crystal -> lab                          */
/* ---------------------------------------------------------------------- */
static void orc_qmul(const double *a, const double *b, double *o)
{
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

static void orc_qmatrix(const double *q_in, double *M)
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
    M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
    M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

/* The 24 proper rotations of the cubic group m-3m as quaternions: identity,
 * 3 x 180 deg about <100>, 6 x +-90 deg about <100>, 6 x 180 deg about <110>,
 * 8 x +-120 deg about <111>. */
static void orc_cubic_group(double S[24][4])
{
    const double h = sqrt(0.5);
    int n = 0;
    S[n][0] = 1; S[n][1] = 0; S[n][2] = 0; S[n][3] = 0; ++n;
    for (int a = 0; a < 3; ++a) {                   /* 180 about x, y, z */
        S[n][0] = 0; S[n][1] = 0; S[n][2] = 0; S[n][3] = 0; S[n][1 + a] = 1; ++n;
    }
    for (int a = 0; a < 3; ++a)                     /* +-90 about x, y, z */
        for (int sg = -1; sg <= 1; sg += 2) {
            S[n][0] = h; S[n][1] = 0; S[n][2] = 0; S[n][3] = 0; S[n][1 + a] = sg * h; ++n;
        }
    for (int a = 0; a < 3; ++a)                     /* 180 about <110>: (1,+-1,0) and perms */
        for (int sg = -1; sg <= 1; sg += 2) {
            int i = a, j = (a + 1) % 3;
            S[n][0] = 0; S[n][1] = 0; S[n][2] = 0; S[n][3] = 0;
            S[n][1 + i] = h; S[n][1 + j] = sg * h; ++n;
        }
    for (int sx = -1; sx <= 1; sx += 2)             /* +-120 about <111> */
        for (int sy = -1; sy <= 1; sy += 2)
            for (int sz = -1; sz <= 1; sz += 2) {
                S[n][0] = 0.5; S[n][1] = 0.5 * sx; S[n][2] = 0.5 * sy; S[n][3] = 0.5 * sz; ++n;
            }
}

/* Reading R9, degrees. */
void orc_disorientation_cubic(const double *qa, const double *qb, int64_t n, double *deg)
{
    double S[24][4];
    orc_cubic_group(S);
    for (int64_t i = 0; i < n; ++i) {
        const double *a = qa + 4 * i, *b = qb + 4 * i;
        double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
        double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + b[3] * b[3]);
        double ai[4] = {a[0] / na, -a[1] / na, -a[2] / na, -a[3] / na};
        double bn[4] = {b[0] / nb, b[1] / nb, b[2] / nb, b[3] / nb};
        double m[4], best = 0.0;
        orc_qmul(ai, bn, m);
        for (int s = 0; s < 24; ++s) {
            double t[4];
            orc_qmul(m, S[s], t);
            double c = fabs(t[0]);
            if (c > best) best = c;
        }
        if (best > 1.0) best = 1.0;
        deg[i] = 2.0 * acos(best) * 180.0 / ORC_PI;
    }
}

/* All 24 symmetry quaternions, for tests. */
void orc_cubic_group_out(double *out)
{
    double S[24][4];
    orc_cubic_group(S);
    memcpy(out, S, sizeof(S));
}

/* ---------------------------------------------------------------------- */
/* Rotated reference library (reading R10)                                  */
/* ---------------------------------------------------------------------- */
/* lut[l][v] = index u of the node with the largest n_u . (R(q_l)^T n_v),
 * FP64, exhaustive, ties to the lower index. */
void orc_rotated_nodes(const double *quats, int64_t n_lib, const float *dirs, int32_t n_dir, int32_t *lut,
                       int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int64_t l = 0; l < n_lib; ++l) {
        double M[9];
        orc_qmatrix(quats + 4 * l, M);
        for (int32_t v = 0; v < n_dir; ++v) {
            double x = dirs[3 * v], y = dirs[3 * v + 1], z = dirs[3 * v + 2];
            /* R^T n */
            double rx = M[0] * x + M[3] * y + M[6] * z;
            double ry = M[1] * x + M[4] * y + M[7] * z;
            double rz = M[2] * x + M[5] * y + M[8] * z;
            double best = -INFINITY;
            int32_t arg = 0;
            for (int32_t u = 0; u < n_dir; ++u) {
                double d = rx * dirs[3 * u] + ry * dirs[3 * u + 1] + rz * dirs[3 * u + 2];
                if (d > best) { best = d; arg = u; }
            }
            lut[(size_t)l * n_dir + v] = arg;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Structure-factor score on spherical shells (reading R11), FP64            */
/* ---------------------------------------------------------------------- */
/* amp[w][v] = |sum_j exp(-2 pi i f_w (R(q) n_v) . x_j)| / N_w */
void orc_sf_amplitudes(const float *rel, int64_t n_w, const double *q, const float *dirs, int32_t n_dir,
                       const double *freqs, int32_t n_freq, double *amp)
{
    double M[9];
    orc_qmatrix(q, M);
    for (int32_t v = 0; v < n_dir; ++v) {
        double x = dirs[3 * v], y = dirs[3 * v + 1], z = dirs[3 * v + 2];
        double u0 = M[0] * x + M[1] * y + M[2] * z;
        double u1 = M[3] * x + M[4] * y + M[5] * z;
        double u2 = M[6] * x + M[7] * y + M[8] * z;
        for (int32_t w = 0; w < n_freq; ++w) {
            double re = 0.0, im = 0.0;
            for (int64_t j = 0; j < n_w; ++j) {
                double s = u0 * rel[3 * j] + u1 * rel[3 * j + 1] + u2 * rel[3 * j + 2];
                double th = 2.0 * ORC_PI * freqs[w] * s;
                re += cos(th);
                im -= sin(th);
            }
            amp[(size_t)w * n_dir + v] = n_w > 0 ? sqrt(re * re + im * im) / (double)n_w : 0.0;
        }
    }
}

double orc_sf_score(const float *rel, int64_t n_w, const double *q, const float *dirs, int32_t n_dir,
                    const double *freqs, int32_t n_freq, const double *target)
{
    double *amp = (double *)malloc(sizeof(double) * (size_t)n_freq * n_dir);
    orc_sf_amplitudes(rel, n_w, q, dirs, n_dir, freqs, n_freq, amp);
    double J = 0.0;
    for (int64_t i = 0; i < (int64_t)n_freq * n_dir; ++i) { double e = amp[i] - target[i]; J += e * e; }
    free(amp);
    return J;
}

/* Central finite differences of J(q) in the four quaternion components. */
void orc_sf_grad_fd(const float *rel, int64_t n_w, const double *q, const float *dirs, int32_t n_dir,
                    const double *freqs, int32_t n_freq, const double *target, double h, double *grad)
{
    for (int c = 0; c < 4; ++c) {
        double qp[4] = {q[0], q[1], q[2], q[3]}, qm[4] = {q[0], q[1], q[2], q[3]};
        qp[c] += h; qm[c] -= h;
        double jp = orc_sf_score(rel, n_w, qp, dirs, n_dir, freqs, n_freq, target);
        double jm = orc_sf_score(rel, n_w, qm, dirs, n_dir, freqs, n_freq, target);
        grad[c] = (jp - jm) / (2.0 * h);
    }
}

/* Refinement trajectory (reading R11 plus the stated update rule, FP64 with
 * central-difference gradients): per iteration a trial q' = normalise(q -
 * a g/|g|) is accepted iff J(q') <= J(q) - 1e-4 a |g| (then a *= 1.5, the
 * gradient is re-evaluated at q'), else a *= 0.5.  `steps` trials. */
double orc_sf_refine(const float *rel, int64_t n_w, double *q, const float *dirs, int32_t n_dir,
                     const double *freqs, int32_t n_freq, const double *target, int32_t steps, double a0, double h)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) q[i] /= n;
    double J = orc_sf_score(rel, n_w, q, dirs, n_dir, freqs, n_freq, target);
    double g[4];
    orc_sf_grad_fd(rel, n_w, q, dirs, n_dir, freqs, n_freq, target, h, g);
    double a = a0;
    for (int it = 0; it < steps; ++it) {
        double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3]);
        if (gn == 0.0) break;
        double t[4];
        for (int i = 0; i < 4; ++i) t[i] = q[i] - a * g[i] / gn;
        double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + t[3] * t[3]);
        for (int i = 0; i < 4; ++i) t[i] /= tn;
        double Jt = orc_sf_score(rel, n_w, t, dirs, n_dir, freqs, n_freq, target);
        if (Jt <= J - 1e-4 * a * gn) {
            for (int i = 0; i < 4; ++i) q[i] = t[i];
            J = Jt;
            orc_sf_grad_fd(rel, n_w, q, dirs, n_dir, freqs, n_freq, target, h, g);
            a *= 1.5;
        } else {
            a *= 0.5;
        }
    }
    return J;
}

/* ---------------------------------------------------------------------- */
/* Sparse look-up-table indexing (reading R12), FP64                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    double v;
    int32_t i;
} orc_ranked;

/* decreasing value, then increasing flat index */
static int orc_ranked_cmp(const void *a, const void *b)
{
    const orc_ranked *x = (const orc_ranked *)a, *y = (const orc_ranked *)b;
    if (x->v > y->v) return -1;
    if (x->v < y->v) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

/* Per phase: the n_hat strongest entries of the window-normalised reference.
 * strong_idx[c][i] = w * n_dir + v, strong_val[c][i] = x / max (FP64). */
void orc_sparse_strong(const float *ref, int32_t n_phase, int32_t n_win, int32_t n_dir, int32_t n_hat,
                       int32_t *strong_idx, double *strong_val)
{
    const int64_t K = (int64_t)n_win * n_dir;
    orc_ranked *e = (orc_ranked *)malloc(sizeof(orc_ranked) * (size_t)K);
    for (int32_t c = 0; c < n_phase; ++c) {
        for (int32_t w = 0; w < n_win; ++w) {
            const float *src = ref + ((size_t)c * n_win + w) * n_dir;
            double m = 0.0;
            for (int32_t v = 0; v < n_dir; ++v) if ((double)src[v] > m) m = (double)src[v];
            for (int32_t v = 0; v < n_dir; ++v) {
                e[(size_t)w * n_dir + v].v = m > 0.0 ? (double)src[v] / m : 0.0;
                e[(size_t)w * n_dir + v].i = w * n_dir + v;
            }
        }
        qsort(e, (size_t)K, sizeof(orc_ranked), orc_ranked_cmp);
        for (int32_t i = 0; i < n_hat; ++i) {
            strong_idx[(size_t)c * n_hat + i] = e[i].i;
            strong_val[(size_t)c * n_hat + i] = e[i].v;
        }
    }
    free(e);
}

/* lut[l][i] = index u of the node with the largest n_u . (R(q_l) n_v),
 * v = node of strong entry i of phase[l]; FP64, ties to the lower index. */
void orc_sparse_lut(const double *quats, const int32_t *phase, int64_t n_lib, const int32_t *strong_idx,
                    int32_t n_hat, const float *dirs, int32_t n_dir, int32_t *lut, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int64_t l = 0; l < n_lib; ++l) {
        double M[9];
        orc_qmatrix(quats + 4 * l, M);
        for (int32_t i = 0; i < n_hat; ++i) {
            const int32_t v = strong_idx[(size_t)phase[l] * n_hat + i] % n_dir;
            double x = dirs[3 * v], y = dirs[3 * v + 1], z = dirs[3 * v + 2];
            /* R n */
            double rx = M[0] * x + M[1] * y + M[2] * z;
            double ry = M[3] * x + M[4] * y + M[5] * z;
            double rz = M[6] * x + M[7] * y + M[8] * z;
            double best = -INFINITY;
            int32_t arg = 0;
            for (int32_t u = 0; u < n_dir; ++u) {
                double d = rx * dirs[3 * u] + ry * dirs[3 * u + 1] + rz * dirs[3 * u + 2];
                if (d > best) { best = d; arg = u; }
            }
            lut[(size_t)l * n_hat + i] = arg;
        }
    }
}

/* Eq. S1 (sparse) for one (ROI, library entry) pair. */
static double orc_sparse_delta(const double *s, int32_t n_dir, const int32_t *strong_idx, const double *strong_val,
                               const int32_t *lut_row, int32_t n_hat)
{
    double delta = 0.0;
    for (int32_t i = 0; i < n_hat; ++i) {
        const int32_t w = strong_idx[i] / n_dir;
        double e = s[(size_t)w * n_dir + lut_row[i]] - strong_val[i];
        delta += e * e;
    }
    return delta;
}

/* For every normalised ROI image Sh[r][n_win][n_dir]: the k library entries
 * with the smallest sparse Delta, ascending by (Delta, library index). */
void orc_sparse_index_topk(const double *Sh, int64_t n_roi, int32_t n_win, int32_t n_dir, const int32_t *strong_idx,
                           const double *strong_val, const int32_t *phase, const int32_t *lut, int64_t n_lib,
                           int32_t n_hat, int32_t k, int32_t *top_idx, double *top_score, int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int64_t r = 0; r < n_roi; ++r) {
        const double *s = Sh + (size_t)r * n_win * n_dir;
        int32_t *bi = top_idx + (size_t)r * k;
        double *bs = top_score + (size_t)r * k;
        int32_t filled = 0;
        for (int64_t l = 0; l < n_lib; ++l) {
            const size_t c = (size_t)phase[l];
            double delta = orc_sparse_delta(s, n_dir, strong_idx + c * n_hat, strong_val + c * n_hat,
                                            lut + (size_t)l * n_hat, n_hat);
            int32_t pos = filled;
            while (pos > 0 && bs[pos - 1] > delta) --pos;
            if (pos >= k) continue;
            int32_t last = filled < k ? filled : k - 1;
            for (int32_t m = last; m > pos; --m) { bs[m] = bs[m - 1]; bi[m] = bi[m - 1]; }
            bs[pos] = delta; bi[pos] = (int32_t)l;
            if (filled < k) ++filled;
        }
        for (int32_t m = filled; m < k; ++m) { bs[m] = INFINITY; bi[m] = -1; }
    }
}

/* Sparse Delta for explicit (roi, library) pairs; lut rows of the listed
 * library entries are passed in lut_rows[p][n_hat]. */
void orc_sparse_pairs(const double *Sh, int32_t n_win, int32_t n_dir, const int32_t *strong_idx,
                      const double *strong_val, const int32_t *pair_phase, const int32_t *lut_rows, int32_t n_hat,
                      const int64_t *roi, int64_t n_pairs, double *out)
{
    for (int64_t p = 0; p < n_pairs; ++p) {
        const size_t c = (size_t)pair_phase[p];
        out[p] = orc_sparse_delta(Sh + (size_t)roi[p] * n_win * n_dir, n_dir, strong_idx + c * n_hat,
                                  strong_val + c * n_hat, lut_rows + (size_t)p * n_hat, n_hat);
    }
}

/* ---------------------------------------------------------------------- */
/* Reciprocal-space signatures on a cubic grid (reading R14), FP64          */
/* ---------------------------------------------------------------------- */
/* amp at explicit k vectors (cycles per length unit): |sum_w exp(-2 pi i k.d_w)| */
void orc_fsp_at(const float *rel, int64_t n_w, const double *k, int64_t n_k, double *amp)
{
    for (int64_t q = 0; q < n_k; ++q) {
        double re = 0.0, im = 0.0;
        for (int64_t w = 0; w < n_w; ++w) {
            double t = k[3 * q] * rel[3 * w] + k[3 * q + 1] * rel[3 * w + 1] + k[3 * q + 2] * rel[3 * w + 2];
            re += cos(2.0 * ORC_PI * t);
            im -= sin(2.0 * ORC_PI * t);
        }
        amp[q] = sqrt(re * re + im * im);
    }
}

/* amp[a][b][c] on the L^3 grid of reading R14 */
void orc_fsp_grid(const float *rel, int64_t n_w, int32_t L, double k_max, double *amp, int32_t n_threads)
{
    const double dk = 2.0 * k_max / (double)L;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int32_t a = 0; a < L; ++a)
        for (int32_t b = 0; b < L; ++b)
            for (int32_t c = 0; c < L; ++c) {
                double k[3] = {(a - L / 2) * dk, (b - L / 2) * dk, (c - L / 2) * dk};
                orc_fsp_at(rel, n_w, k, 1, amp + ((size_t)a * L + b) * L + c);
            }
}

/* ---------------------------------------------------------------------- */
/* Adaptive ROI-grid refinement (reading R15)                               */
/* ---------------------------------------------------------------------- */
/* keep[r] = 1 if ROI r passes the kappa test on a window of window_mask.
 * Returns the number of kept ROIs; refined centres are written for them
 * (cap ROIs at most, parent index of each).  Returns -1 without writing
 * anything when n_win is outside [1, 32] (the window mask has 32 bits) or
 * split < 1. */
int64_t orc_refine_roi_grid(const float *centres, const double *img, const int32_t *counts, int64_t n_roi,
                            int32_t n_win, int32_t n_dir, uint32_t window_mask, double kappa, double h, int32_t split,
                            int32_t *keep, float *out_centres, int32_t *out_parent, int64_t cap)
{
    double best[32];
    if (n_win < 1 || n_win > 32 || split < 1) return -1;
    double *I = (double *)malloc(sizeof(double) * (size_t)(n_roi > 0 ? n_roi : 1) * n_win);
    for (int32_t w = 0; w < n_win; ++w) best[w] = 0.0;
    for (int64_t r = 0; r < n_roi; ++r)
        for (int32_t w = 0; w < n_win; ++w) {
            double m = 0.0;
            for (int32_t v = 0; v < n_dir; ++v) {
                double x = img[((size_t)r * n_win + w) * n_dir + v];
                if (x > m) m = x;
            }
            double val = counts[r] > 0 ? m / (double)counts[r] : 0.0;
            I[(size_t)r * n_win + w] = val;
            if (val > best[w]) best[w] = val;
        }
    int64_t n_keep = 0, n_out = 0;
    for (int64_t r = 0; r < n_roi; ++r) {
        int k = 0;
        for (int32_t w = 0; w < n_win; ++w)
            if (((window_mask >> w) & 1u) && best[w] > 0.0 && I[(size_t)r * n_win + w] >= kappa * best[w]) k = 1;
        keep[r] = k;
        if (!k) continue;
        ++n_keep;
        for (int32_t i = 0; i < split; ++i)
            for (int32_t j = 0; j < split; ++j)
                for (int32_t q = 0; q < split; ++q) {
                    if (n_out < cap) {
                        int32_t id[3] = {i, j, q};
                        for (int a = 0; a < 3; ++a) {
                            float off = (float)(h * (double)(2 * id[a] + 1 - split) / (double)(2 * split));
                            out_centres[3 * n_out + a] = centres[3 * r + a] + off;
                        }
                        out_parent[n_out] = (int32_t)r;
                    }
                    ++n_out;
                }
    }
    free(I);
    return n_keep;
}
