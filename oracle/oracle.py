"""NumPy front end of the C reference oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It loads `liboracle.so`, built from `araullo_oracle.c` with gcc
(`build()`), and marshals NumPy arrays; all arithmetic is in the C file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "araullo_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]


# Host sanitizer build of the same source (memory errors and undefined
# behaviour abort the process).  Loaded instead of LIB when the environment
# variable ARAULLO_ORACLE_SANITIZED=1 is set; the Python process must then run
# with the sanitizer runtime preloaded (see tests/test_oracle_sanitized.py).
LIB_SANITIZED = os.path.join(HERE, "liboracle_sanitized.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitized: bool = False) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    out = LIB_SANITIZED if sanitized else LIB
    flags = [f for f in CFLAGS if not (sanitized and f == "-O2")] + (SANITIZE_FLAGS if sanitized else [])
    tmp = out + ".tmp"
    cmd = ["gcc", *flags, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None

F32P = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
I32P = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
I64P = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
c_i32, c_i64, c_f32, c_f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        sanitized = os.environ.get("ARAULLO_ORACLE_SANITIZED") == "1"
        path = LIB_SANITIZED if sanitized else LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(sanitized=sanitized)
        L = ctypes.CDLL(path)
        L.orc_bin_constants.argtypes = [c_f32, c_i32, ctypes.POINTER(c_f32), ctypes.POINTER(c_f32),
                                        ctypes.POINTER(c_f64)]
        L.orc_window_bins.argtypes = [c_f64, c_i32, c_f64, c_f64, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]
        L.orc_window_bins.restype = c_i32
        L.orc_roi_gather.argtypes = [F32P, c_i64, F32P, c_f32, ctypes.c_void_p, c_i64]
        L.orc_roi_gather.restype = c_i64
        L.orc_sdm_hist.argtypes = [F32P, c_i64, F32P, c_f32, c_i32, I32P]
        L.orc_amplitudes.argtypes = [I32P, c_i32, F64P]
        L.orc_signatures.argtypes = [F32P, c_i64, F32P, c_i64, c_f32, F32P, c_i32, c_i32, I32P, c_i32, F64P,
                                     I32P, c_i32]
        L.orc_sdm_debug.argtypes = [F32P, c_i64, c_f32, F32P, c_i32, c_i32, I32P, ctypes.c_void_p]
        L.orc_normalise.argtypes = [F32P, c_i64, c_i32, c_i32, F64P]
        L.orc_index_topk.argtypes = [F64P, c_i64, F64P, c_i64, c_i64, c_i32, I32P, F64P, c_i32]
        L.orc_ssd_pairs.argtypes = [F64P, F64P, c_i64, I64P, I64P, c_i64, F64P]
        L.orc_disorientation_cubic.argtypes = [F64P, F64P, c_i64, F64P]
        L.orc_cubic_group_out.argtypes = [F64P]
        L.orc_rotated_nodes.argtypes = [F64P, c_i64, F32P, c_i32, I32P, c_i32]
        L.orc_sparse_strong.argtypes = [F32P, c_i32, c_i32, c_i32, c_i32, I32P, F64P]
        L.orc_sparse_lut.argtypes = [F64P, I32P, c_i64, I32P, c_i32, F32P, c_i32, I32P, c_i32]
        L.orc_sparse_index_topk.argtypes = [F64P, c_i64, c_i32, c_i32, I32P, F64P, I32P, I32P, c_i64, c_i32,
                                            c_i32, I32P, F64P, c_i32]
        L.orc_sparse_pairs.argtypes = [F64P, c_i32, c_i32, I32P, F64P, I32P, I32P, c_i32, I64P, c_i64, F64P]
        L.orc_fsp_at.argtypes = [F32P, c_i64, F64P, c_i64, F64P]
        L.orc_fsp_grid.argtypes = [F32P, c_i64, c_i32, c_f64, F64P, c_i32]
        L.orc_refine_roi_grid.argtypes = [F32P, F64P, I32P, c_i64, c_i32, c_i32, ctypes.c_uint32, c_f64, c_f64,
                                          c_i32, I32P, F32P, I32P, c_i64]
        L.orc_refine_roi_grid.restype = c_i64
        L.orc_sf_amplitudes.argtypes = [F32P, c_i64, F64P, F32P, c_i32, F64P, c_i32, F64P]
        L.orc_sf_score.argtypes = [F32P, c_i64, F64P, F32P, c_i32, F64P, c_i32, F64P]
        L.orc_sf_score.restype = c_f64
        L.orc_sf_grad_fd.argtypes = [F32P, c_i64, F64P, F32P, c_i32, F64P, c_i32, F64P, c_f64, F64P]
        L.orc_sf_refine.argtypes = [F32P, c_i64, F64P, F32P, c_i32, F64P, c_i32, F64P, c_i32, c_f64, c_f64]
        L.orc_sf_refine.restype = c_f64
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


# ---------------------------------------------------------------- signatures
def bin_constants(radius: float, nbins: int) -> Tuple[float, float, float]:
    s, c, w = c_f32(), c_f32(), c_f64()
    lib().orc_bin_constants(radius, nbins, ctypes.byref(s), ctypes.byref(c), ctypes.byref(w))
    return s.value, c.value, w.value


def window_bins(radius: float, nbins: int, d_min: float, d_max: float) -> Tuple[int, int]:
    lo, hi = c_i32(), c_i32()
    rc = lib().orc_window_bins(radius, nbins, d_min, d_max, ctypes.byref(lo), ctypes.byref(hi))
    if rc != 0:
        raise ValueError(f"empty or out-of-range window for d in [{d_min}, {d_max}]")
    return lo.value, hi.value


def windows_for(radius: float, nbins: int, spacings) -> np.ndarray:
    return np.array([window_bins(radius, nbins, float(a), float(b)) for a, b in np.asarray(spacings)],
                    dtype=np.int32)


def roi_gather(positions, centre, radius: float) -> np.ndarray:
    p = _f32(positions)
    c = _f32(centre).reshape(3)
    n = lib().orc_roi_gather(p, len(p), c, radius, None, 0)
    out = np.zeros((max(n, 1), 3), np.float32)
    lib().orc_roi_gather(p, len(p), c, radius, out.ctypes.data, n)
    return out[:n]


def sdm_hist(rel, v, radius: float, nbins: int) -> np.ndarray:
    rel = _f32(rel).reshape(-1, 3)
    h = np.zeros(nbins, np.int32)
    lib().orc_sdm_hist(rel, len(rel), _f32(v).reshape(3), radius, nbins, h)
    return h


def amplitudes(hist) -> np.ndarray:
    h = _i32(hist)
    a = np.zeros(len(h) // 2 + 1, np.float64)
    lib().orc_amplitudes(h, len(h), a)
    return a


def signatures(positions, centres, radius: float, directions, nbins: int, windows,
               threads: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    p, c, d, w = _f32(positions), _f32(centres).reshape(-1, 3), _f32(directions), _i32(windows).reshape(-1, 2)
    n_roi, n_dir, n_win = len(c), len(d), len(w)
    img = np.zeros((n_roi, n_win, n_dir), np.float64)
    cnt = np.zeros(n_roi, np.int32)
    lib().orc_signatures(p, len(p), c, n_roi, radius, d, n_dir, nbins, w, n_win, img, cnt,
                         threads or default_threads())
    return img, cnt


def signatures_typed(positions, types, type_masks, centres, radius: float, directions, nbins: int, windows,
                     threads: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Reading R13: channel c of every ROI is the signature of the atoms whose
    type t has bit t set in type_masks[c] (0 <= t < 64).
    Returns (images [n_roi][n_ch][n_win][n_dir] float64, counts [n_roi][n_ch])."""
    t = np.asarray(types, np.int64)
    p = np.asarray(positions)
    imgs, cnts = [], []
    for m in type_masks:
        ok = (t >= 0) & (t < 64) & (((np.uint64(m) >> t.clip(0, 63).astype(np.uint64)) & np.uint64(1)) == 1)
        img, cnt = signatures(p[ok], centres, radius, directions, nbins, windows, threads)
        imgs.append(img)
        cnts.append(cnt)
    return np.stack(imgs, axis=1), np.stack(cnts, axis=1)


def sdm_debug(rel, radius: float, directions, nbins: int, spectra: bool = True):
    """Histograms [n_dir][nbins] and (if spectra) amplitudes [n_dir][nbins/2+1]."""
    rel = _f32(rel).reshape(-1, 3)
    d = _f32(directions)
    h = np.zeros((len(d), nbins), np.int32)
    a = np.zeros((len(d), nbins // 2 + 1), np.float64) if spectra else None
    lib().orc_sdm_debug(rel, len(rel), radius, d, len(d), nbins, h, a.ctypes.data if spectra else None)
    return h, a


# ---------------------------------------------------------------- indexing
def normalise(images) -> np.ndarray:
    x = _f32(images)
    n, n_win, n_dir = x.shape
    out = np.zeros_like(x, dtype=np.float64)
    lib().orc_normalise(x, n, n_win, n_dir, out)
    return out


def index_topk(S_hat, L_hat, k: int, threads: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    S = _f64(S_hat).reshape(len(S_hat), -1)
    L = _f64(L_hat).reshape(len(L_hat), -1)
    assert S.shape[1] == L.shape[1]
    idx = np.zeros((len(S), k), np.int32)
    sc = np.zeros((len(S), k), np.float64)
    lib().orc_index_topk(S, len(S), L, len(L), S.shape[1], k, idx, sc, threads or default_threads())
    return idx, sc


def ssd_pairs(S_hat, L_hat, roi, libidx) -> np.ndarray:
    S = _f64(S_hat).reshape(len(S_hat), -1)
    L = _f64(L_hat).reshape(len(L_hat), -1)
    r = np.ascontiguousarray(roi, np.int64)
    l = np.ascontiguousarray(libidx, np.int64)
    out = np.zeros(len(r), np.float64)
    lib().orc_ssd_pairs(S, L, S.shape[1], r, l, len(r), out)
    return out


def disorientation_cubic(qa, qb) -> np.ndarray:
    a = _f64(qa).reshape(-1, 4)
    b = _f64(qb).reshape(-1, 4)
    out = np.zeros(len(a), np.float64)
    lib().orc_disorientation_cubic(a, b, len(a), out)
    return out


def cubic_group() -> np.ndarray:
    out = np.zeros((24, 4), np.float64)
    lib().orc_cubic_group_out(out)
    return out


def rotated_nodes(quats, directions, threads: Optional[int] = None) -> np.ndarray:
    q = _f64(quats).reshape(-1, 4)
    d = _f32(directions)
    lut = np.zeros((len(q), len(d)), np.int32)
    lib().orc_rotated_nodes(q, len(q), d, len(d), lut, threads or default_threads())
    return lut


def library_images(reference, phase_of, quats, directions, threads: Optional[int] = None) -> np.ndarray:
    """Rotated reference images [n_lib][n_win][n_dir]: the value at node v of
    entry l is reference[phase_of[l]][w][lut[l][v]] (nearest rotated node)."""
    ref = np.asarray(reference)
    lut = rotated_nodes(quats, directions, threads)
    ph = np.asarray(phase_of, np.int64)
    out = np.empty((len(lut), ref.shape[1], ref.shape[2]), ref.dtype)
    for l in range(len(lut)):
        out[l] = ref[ph[l]][:, lut[l]]
    return out


# ---------------------------------------------------------------- sparse indexing (reading R12)
def sparse_strong(reference, n_hat: int) -> Tuple[np.ndarray, np.ndarray]:
    """Per phase of reference [n_phase][n_win][n_dir]: the n_hat strongest
    window-normalised entries as flat indices w*n_dir+v (decreasing value,
    ties to the lower index) and their FP64 normalised values."""
    x = _f32(reference)
    n_phase, n_win, n_dir = x.shape
    assert 1 <= n_hat <= n_win * n_dir
    idx = np.zeros((n_phase, n_hat), np.int32)
    val = np.zeros((n_phase, n_hat), np.float64)
    lib().orc_sparse_strong(x, n_phase, n_win, n_dir, n_hat, idx, val)
    return idx, val


def sparse_lut(quats, phase, strong_idx, directions, threads: Optional[int] = None) -> np.ndarray:
    """lut[l][i]: mesh node closest to R(q_l) n_v, v = node of strong entry i
    of phase[l]."""
    q = _f64(quats).reshape(-1, 4)
    ph = _i32(phase)
    si = _i32(strong_idx)
    d = _f32(directions)
    out = np.zeros((len(q), si.shape[1]), np.int32)
    lib().orc_sparse_lut(q, ph, len(q), si, si.shape[1], d, len(d), out, threads or default_threads())
    return out


def sparse_index_topk(S_hat, strong_idx, strong_val, phase, lut, k: int,
                      threads: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    S = _f64(S_hat)
    n_roi, n_win, n_dir = S.shape
    si, sv, ph, lt = _i32(strong_idx), _f64(strong_val), _i32(phase), _i32(lut)
    idx = np.zeros((n_roi, k), np.int32)
    sc = np.zeros((n_roi, k), np.float64)
    lib().orc_sparse_index_topk(S, n_roi, n_win, n_dir, si, sv, ph, lt, len(lt), si.shape[1], k, idx, sc,
                                threads or default_threads())
    return idx, sc


def sparse_pairs(S_hat, strong_idx, strong_val, pair_phase, lut_rows, roi) -> np.ndarray:
    """Sparse Delta of (roi[p], entry with look-up row lut_rows[p] and phase
    pair_phase[p])."""
    S = _f64(S_hat)
    n_roi, n_win, n_dir = S.shape
    si, sv = _i32(strong_idx), _f64(strong_val)
    r = np.ascontiguousarray(roi, np.int64)
    out = np.zeros(len(r), np.float64)
    lib().orc_sparse_pairs(S, n_win, n_dir, si, sv, _i32(pair_phase), _i32(lut_rows), si.shape[1], r, len(r), out)
    return out


# ---------------------------------------------------------------- reciprocal-space grid (reading R14)
def fsp_grid_k(L: int, k_max: float) -> np.ndarray:
    """The grid's k values along one axis (cycles per length unit)."""
    return (np.arange(L) - L // 2) * (2.0 * k_max / L)


def fsp_at(rel, k) -> np.ndarray:
    """|sum_w exp(-2 pi i k . d_w)| at explicit k vectors [n_k][3]."""
    r = _f32(rel).reshape(-1, 3)
    kk = _f64(k).reshape(-1, 3)
    out = np.zeros(len(kk), np.float64)
    lib().orc_fsp_at(r, len(r), kk, len(kk), out)
    return out


def fsp_grid(rel, L: int, k_max: float, threads: Optional[int] = None) -> np.ndarray:
    """Amplitudes [L][L][L] on the cubic grid of reading R14."""
    r = _f32(rel).reshape(-1, 3)
    out = np.zeros((L, L, L), np.float64)
    lib().orc_fsp_grid(r, len(r), L, k_max, out, threads or default_threads())
    return out


# ---------------------------------------------------------------- adaptive ROI grid (reading R15)
def refine_roi_grid(centres, images, counts, window_mask: int, kappa: float, h: float, split: int = 5):
    """-> (keep int32 [n_roi], refined centres float32 [n_keep*split^3][3],
    parent int32 [n_keep*split^3])."""
    c = _f32(centres).reshape(-1, 3)
    img = _f64(images)
    n_roi, n_win, n_dir = img.shape
    if float(np.float32(h)) != float(h):
        # the GPU interface takes h in single precision: callers pass an FP32
        # number to both sides instead of the oracle rounding it
        raise ValueError(f"cell edge {h!r} is not a single-precision number")
    cnt = _i32(counts)
    keep = np.zeros(n_roi, np.int32)
    cap = int(n_roi) * split ** 3
    out = np.zeros((max(cap, 1), 3), np.float32)
    par = np.zeros(max(cap, 1), np.int32)
    n_keep = lib().orc_refine_roi_grid(c, img, cnt, n_roi, n_win, n_dir, window_mask, kappa, float(h),
                                       split, keep, out, par, cap)
    if n_keep < 0:
        raise ValueError(f"n_win {n_win} outside [1, 32] or split {split} < 1")
    n = int(n_keep) * split ** 3
    return keep, out[:n], par[:n]


# ---------------------------------------------------------------- structure factor
def sf_amplitudes(rel, q, directions, freqs) -> np.ndarray:
    rel = _f32(rel).reshape(-1, 3)
    d = _f32(directions)
    f = _f64(freqs)
    out = np.zeros((len(f), len(d)), np.float64)
    lib().orc_sf_amplitudes(rel, len(rel), _f64(q), d, len(d), f, len(f), out)
    return out


def sf_score(rel, q, directions, freqs, target) -> float:
    rel = _f32(rel).reshape(-1, 3)
    d = _f32(directions)
    f = _f64(freqs)
    return lib().orc_sf_score(rel, len(rel), _f64(q), d, len(d), f, len(f), _f64(target))


def sf_grad_fd(rel, q, directions, freqs, target, h: float = 1e-6) -> np.ndarray:
    rel = _f32(rel).reshape(-1, 3)
    d = _f32(directions)
    f = _f64(freqs)
    g = np.zeros(4, np.float64)
    lib().orc_sf_grad_fd(rel, len(rel), _f64(q), d, len(d), f, len(f), _f64(target), h, g)
    return g


def sf_refine(rel, q, directions, freqs, target, steps: int = 50, a0: float = 0.01, h: float = 1e-6):
    """-> (refined unit quaternion float64 [4], final J)."""
    rel = _f32(rel).reshape(-1, 3)
    d = _f32(directions)
    f = _f64(freqs)
    qq = _f64(q).copy()
    J = lib().orc_sf_refine(rel, len(rel), qq, d, len(d), f, len(f), _f64(target), steps, a0, h)
    return qq, J
