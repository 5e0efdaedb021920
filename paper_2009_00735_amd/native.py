"""ctypes binding of libaraullo.so (the C ABI in include/araullo.h).

Argument marshalling only: every function takes/returns torch tensors on the
context's GPU, passes raw device pointers and the current HIP stream to the
C entry point of the same name, and raises AraulloError on a non-zero status.
There is no fallback: if the shared library is missing, importing this
module raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libaraullo.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2009_00735_amd.build`")

_L = ctypes.CDLL(LIB_PATH)

vp, i32, i64, f32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
P = ctypes.POINTER

_SIGS = {
    "ar_last_error": ([vp], ctypes.c_char_p),
    "ar_version": ([], ctypes.c_char_p),
    "ar_context_create": ([ctypes.c_int, P(vp)], ctypes.c_int),
    "ar_context_destroy": ([vp], ctypes.c_int),
    "ar_window_bins": ([f64, i32, f64, f64, P(i32), P(i32)], ctypes.c_int),
    "ar_roi_gather": ([vp, vp, i64, vp, i64, f32, vp, vp, i64, P(i64), vp], ctypes.c_int),
    "araullo_signatures": ([vp, vp, i64, vp, i64, f32, vp, i32, i32, vp, i32, vp, vp, vp], ctypes.c_int),
    "ar_roi_gather_typed": ([vp, vp, vp, i64, vp, i64, f32, ctypes.c_uint64, vp, vp, i64, P(i64), vp], ctypes.c_int),
    "araullo_signatures_typed": ([vp, vp, vp, i64, vp, i64, f32, vp, i32, vp, i32, i32, vp, i32, vp, vp, vp],
                                 ctypes.c_int),
    "araullo_sdm": ([vp, vp, i64, vp, i64, f32, vp, i32, i32, vp, vp, vp], ctypes.c_int),
    "araullo_signatures_csr": ([vp, vp, vp, i64, f32, vp, i32, i32, vp, i32, vp, vp], ctypes.c_int),
    "ar_signature_plan_create": ([vp, i64, i64, i32, i32, i32, P(vp)], ctypes.c_int),
    "ar_signature_plan_destroy": ([vp], ctypes.c_int),
    "ar_signature_plan_tune": ([vp, vp, vp, i64, f32, vp, vp, vp, vp], ctypes.c_int),
    "ar_signature_plan_config": ([vp, P(i32), P(i32), P(i32), P(i32)], ctypes.c_int),
    "ar_signature_plan_set_config": ([vp, i32, i32, i32, i32], ctypes.c_int),
    "ar_signature_plan_run": ([vp, vp, vp, i64, f32, vp, vp, vp, i32, vp], ctypes.c_int),
    "ar_library_create": ([vp, vp, i64, i32, i32, vp, P(vp)], ctypes.c_int),
    "ar_library_destroy": ([vp], ctypes.c_int),
    "ar_library_prepare": ([vp, vp, i64, i32, i32, vp, vp, vp, P(vp)], ctypes.c_int),
    "ar_library_lookup": ([vp, vp, i64, vp, vp, vp], ctypes.c_int),
    "index_orientations": ([vp, vp, i64, vp, i32, vp, vp, vp], ctypes.c_int),
    "ar_index_set_tile": ([vp, i32, i32, i32, i32], ctypes.c_int),
    "ar_sparse_lut_create": ([vp, vp, i32, i32, vp, i32, vp, P(i64), i32, vp, P(vp)], ctypes.c_int),
    "ar_sparse_lut_destroy": ([vp], ctypes.c_int),
    "ar_sparse_lut_export": ([vp, vp, vp, vp, vp], ctypes.c_int),
    "ar_sparse_lut_screen": ([vp, vp], ctypes.c_int),
    "index_orientations_sparse": ([vp, vp, i64, vp, i32, vp, vp, vp], ctypes.c_int),
    "ar_fsp_amplitudes": ([vp, vp, vp, i64, i32, f32, vp, vp], ctypes.c_int),
    "ar_refine_roi_grid": ([vp, vp, vp, vp, i64, i32, i32, ctypes.c_uint32, f32, f32, i32, vp, vp, i64, P(i64), vp],
                           ctypes.c_int),
    "index_orientations_ex": ([vp, vp, i64, vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
    "ar_disorientation_cubic": ([vp, vp, i64, vp, vp], ctypes.c_int),
    "ar_rotate_reference": ([vp, vp, i32, i32, vp, i32, vp, vp, i64, vp, vp], ctypes.c_int),
    "ar_sf_score_grad": ([vp, vp, vp, i64, vp, vp, vp, i32, vp, vp, i32, i32, vp, vp, vp], ctypes.c_int),
    "ar_sf_score_grad_noalloc": ([vp, vp, vp, i64, vp, vp, vp, i32, vp, vp, i32, i32, vp, vp, vp], ctypes.c_int),
    "ar_sf_score_f64": ([vp, vp, vp, i64, vp, vp, vp, i32, vp, vp, i32, i32, vp, vp], ctypes.c_int),
    "ar_sf_amplitudes": ([vp, vp, vp, i64, vp, vp, vp, i32, vp, i32, i32, vp, vp], ctypes.c_int),
    "ar_refine_orientations": ([vp, vp, vp, i64, vp, vp, vp, i32, vp, vp, i32, i32, i32, f32, vp, vp],
                               ctypes.c_int),
    "ar_measure_peaks": ([vp, P(ctypes.c_double), i32], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_L, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


class AraulloError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = _L.ar_last_error(None).decode(errors="replace")
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def _call(name: str, *args) -> None:
    st = getattr(_L, name)(*args)
    if st != 0:
        raise AraulloError(name, st)


def version() -> str:
    return _L.ar_version().decode()


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev(t: torch.Tensor, dtype, device, name: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _shape(t: torch.Tensor, shape, name: str) -> None:
    """Raise ValueError unless t has the given shape (None matches any size)."""
    ok = t.dim() == len(shape) and all(want is None or got == want for got, want in zip(t.shape, shape))
    if not ok:
        want = "[" + "][".join("*" if x is None else str(x) for x in shape) + "]"
        raise ValueError(f"{name} must have shape {want}, got {list(t.shape)}")


# v_sin_f32 / v_cos_f32 take the phase in turns and are specified for
# |t| <= 256; the structure-factor kernels form t = f (u . x) without range
# reduction, so every call checks max|f| * max|x| against that bound.
SF_MAX_TURNS = 256.0


def _sf_domain(rel: torch.Tensor, freqs: torch.Tensor) -> None:
    if rel.numel() == 0:
        return
    turns = float(freqs.detach().abs().max()) * float(torch.linalg.vector_norm(rel[:, :3], dim=1).max())
    if not turns <= SF_MAX_TURNS:
        raise ValueError(f"max|f| * max|x| = {turns:.4g} turns exceeds the {SF_MAX_TURNS:g}-turn domain of the "
                         "hardware sine and cosine")


class Context:
    """ar_context on one GPU."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = vp()
        _call("ar_context_create", device, ctypes.byref(h))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _L.ar_context_destroy(self.handle)
            self.handle = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ar_window_bins(radius: float, nbins: int, d_min: float, d_max: float) -> Tuple[int, int]:
    lo, hi = i32(), i32()
    _call("ar_window_bins", radius, nbins, d_min, d_max, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def windows_for(radius: float, nbins: int, spacings) -> torch.Tensor:
    """Host int32 [n_win][2] from (d_min, d_max) pairs."""
    return torch.tensor([ar_window_bins(radius, nbins, float(a), float(b)) for a, b in spacings], dtype=torch.int32)


def _host_windows(windows) -> torch.Tensor:
    w = torch.as_tensor(windows, dtype=torch.int32).reshape(-1, 2).contiguous()
    if w.device.type != "cpu":
        w = w.cpu()
    return w


def ar_roi_gather(ctx: Context, positions: torch.Tensor, centres: torch.Tensor, radius: float,
                  out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, types: Optional[torch.Tensor] = None,
                  type_mask: int = (1 << 64) - 1):
    """-> (offsets int64 [n_roi+1], rel float32 [total][4]) on the GPU.

    With out=(offsets, rel_buffer) the rows are written into the given
    buffers (rel_buffer must hold the total; the result is a view of it).
    With types (int32 [n_atoms]) only atoms whose type bit is set in
    type_mask are gathered (ar_roi_gather_typed)."""
    d = ctx.device
    _shape(positions, (None, 3), "positions")
    _shape(centres, (None, 3), "centres")
    n_roi = centres.shape[0]
    total = i64()
    pp = _dev(positions, torch.float32, d, "positions") if positions.numel() else None
    cp = _dev(centres, torch.float32, d, "centres")
    s = _stream(d)
    if types is None:
        def gather(offp, relp, cap):
            _call("ar_roi_gather", ctx.handle, pp, positions.shape[0], cp, n_roi, radius, offp, relp, cap,
                  ctypes.byref(total), s)
    else:
        _shape(types, (positions.shape[0],), "types")
        tp = _dev(types, torch.int32, d, "types") if types.numel() else None

        def gather(offp, relp, cap):
            _call("ar_roi_gather_typed", ctx.handle, pp, tp, positions.shape[0], cp, n_roi, radius, type_mask, offp,
                  relp, cap, ctypes.byref(total), s)
    if out is not None:
        offsets, rel = out
        _shape(offsets, (n_roi + 1,), "offsets")
        _shape(rel, (None, 4), "rel")
        _dev(offsets, torch.int64, d, "offsets")
        _dev(rel, torch.float32, d, "rel")
        gather(offsets.data_ptr(), rel.data_ptr(), rel.shape[0])
        return offsets, rel[:total.value]
    offsets = torch.empty(n_roi + 1, dtype=torch.int64, device=d)
    gather(offsets.data_ptr(), None, 0)
    rel = torch.empty((max(total.value, 1), 4), dtype=torch.float32, device=d)
    gather(offsets.data_ptr(), rel.data_ptr(), rel.shape[0])
    return offsets, rel[:total.value]


def araullo_signatures(ctx: Context, positions: torch.Tensor, centres: torch.Tensor, radius: float,
                       directions: torch.Tensor, nbins: int, windows, counts: bool = True):
    """-> images float32 [n_roi][n_win][n_dir] (and int32 counts [n_roi])."""
    d = ctx.device
    _shape(positions, (None, 3), "positions")
    _shape(centres, (None, 3), "centres")
    _shape(directions, (None, 3), "directions")
    w = _host_windows(windows)
    n_roi, n_dir, n_win = centres.shape[0], directions.shape[0], w.shape[0]
    images = torch.empty((n_roi, n_win, n_dir), dtype=torch.float32, device=d)
    cnt = torch.empty(n_roi, dtype=torch.int32, device=d) if counts else None
    _call("araullo_signatures", ctx.handle, _dev(positions, torch.float32, d, "positions") if positions.numel() else None,
          positions.shape[0], _dev(centres, torch.float32, d, "centres"), n_roi, radius,
          _dev(directions, torch.float32, d, "directions"), n_dir, nbins, w.data_ptr(), n_win, images.data_ptr(),
          cnt.data_ptr() if counts else None, _stream(d))
    return (images, cnt) if counts else images


def araullo_signatures_typed(ctx: Context, positions: torch.Tensor, types: torch.Tensor, centres: torch.Tensor,
                             radius: float, directions: torch.Tensor, nbins: int, windows, type_masks: Sequence[int],
                             counts: bool = True):
    """-> images float32 [n_roi][n_ch][n_win][n_dir] (and int32 counts [n_roi][n_ch]):
    one signature channel per atom-type mask."""
    d = ctx.device
    _shape(positions, (None, 3), "positions")
    _shape(types, (positions.shape[0],), "types")
    _shape(centres, (None, 3), "centres")
    _shape(directions, (None, 3), "directions")
    w = _host_windows(windows)
    n_roi, n_dir, n_win, n_ch = centres.shape[0], directions.shape[0], w.shape[0], len(type_masks)
    masks = (ctypes.c_uint64 * n_ch)(*[int(m) for m in type_masks])
    images = torch.empty((n_roi, n_ch, n_win, n_dir), dtype=torch.float32, device=d)
    cnt = torch.empty((n_roi, n_ch), dtype=torch.int32, device=d) if counts else None
    _call("araullo_signatures_typed", ctx.handle,
          _dev(positions, torch.float32, d, "positions") if positions.numel() else None,
          _dev(types, torch.int32, d, "types") if types.numel() else None, positions.shape[0],
          _dev(centres, torch.float32, d, "centres"), n_roi, radius, masks, n_ch,
          _dev(directions, torch.float32, d, "directions"), n_dir, nbins, w.data_ptr(), n_win, images.data_ptr(),
          cnt.data_ptr() if counts else None, _stream(d))
    return (images, cnt) if counts else images


def araullo_sdm(ctx: Context, positions: torch.Tensor, centres: torch.Tensor, radius: float,
                directions: torch.Tensor, nbins: int):
    """-> (hist int32 [n_roi][n_dir][nbins], amp float32 [n_roi][n_dir][nbins/2+1])."""
    d = ctx.device
    _shape(positions, (None, 3), "positions")
    _shape(centres, (None, 3), "centres")
    _shape(directions, (None, 3), "directions")
    n_roi, n_dir = centres.shape[0], directions.shape[0]
    hist = torch.empty((n_roi, n_dir, nbins), dtype=torch.int32, device=d)
    amp = torch.empty((n_roi, n_dir, nbins // 2 + 1), dtype=torch.float32, device=d)
    _call("araullo_sdm", ctx.handle, _dev(positions, torch.float32, d, "positions") if positions.numel() else None,
          positions.shape[0], _dev(centres, torch.float32, d, "centres"), n_roi, radius,
          _dev(directions, torch.float32, d, "directions"), n_dir, nbins, hist.data_ptr(), amp.data_ptr(), _stream(d))
    return hist, amp


def araullo_signatures_csr(ctx: Context, rel: torch.Tensor, offsets: torch.Tensor, radius: float,
                           directions: torch.Tensor, nbins: int, windows, out: Optional[torch.Tensor] = None):
    d = ctx.device
    w = _host_windows(windows)
    _shape(rel, (None, 4), "rel")
    _shape(offsets, (None,), "offsets")
    _shape(directions, (None, 3), "directions")
    n_roi, n_dir, n_win = offsets.shape[0] - 1, directions.shape[0], w.shape[0]
    images = out if out is not None else torch.empty((n_roi, n_win, n_dir), dtype=torch.float32, device=d)
    _shape(images, (n_roi, n_win, n_dir), "out")
    relp = rel if rel.numel() else torch.zeros((1, 4), dtype=torch.float32, device=d)
    _call("araullo_signatures_csr", ctx.handle, _dev(relp, torch.float32, d, "rel"),
          _dev(offsets, torch.int64, d, "offsets"), n_roi, radius, _dev(directions, torch.float32, d, "directions"),
          n_dir, nbins, w.data_ptr(), n_win, _dev(images, torch.float32, d, "images"), _stream(d))
    return images


class SignaturePlan:
    """ar_plan: batched persistent signatures, autotuned, graph-replayed."""

    def __init__(self, ctx: Context, max_roi: int, max_total: int, n_dir: int, nbins: int, n_win: int):
        self.ctx = ctx
        h = vp()
        _call("ar_signature_plan_create", ctx.handle, max_roi, max_total, n_dir, nbins, n_win, ctypes.byref(h))
        self.handle = h
        self.n_dir, self.nbins, self.n_win = n_dir, nbins, n_win

    def _args(self, rel, offsets, directions, images):
        d = self.ctx.device
        _shape(rel, (None, 4), "rel")
        _shape(offsets, (None,), "offsets")
        _shape(directions, (self.n_dir, 3), "directions")
        _shape(images, (offsets.shape[0] - 1, self.n_win, self.n_dir), "images")
        relp = rel if rel.numel() else torch.zeros((1, 4), dtype=torch.float32, device=d)
        return (_dev(relp, torch.float32, d, "rel"), _dev(offsets, torch.int64, d, "offsets"), offsets.shape[0] - 1,
                _dev(directions, torch.float32, d, "directions"), _dev(images, torch.float32, d, "images"))

    def _out(self, offsets, out):
        if out is not None:
            return out
        return torch.empty((offsets.shape[0] - 1, self.n_win, self.n_dir), dtype=torch.float32,
                           device=self.ctx.device)

    def tune(self, rel, offsets, radius, directions, windows, out=None):
        images = self._out(offsets, out)
        w = _host_windows(windows)
        r, o, n, dp, ip = self._args(rel, offsets, directions, images)
        _call("ar_signature_plan_tune", self.handle, r, o, n, radius, dp, w.data_ptr(), ip, _stream(self.ctx.device))
        return images

    def config(self) -> Tuple[int, int, int, int]:
        """(dirs_per_item, atoms_per_stage, blocks_per_cu, min_waves)."""
        a, b, c, d = i32(), i32(), i32(), i32()
        _call("ar_signature_plan_config", self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
              ctypes.byref(d))
        return a.value, b.value, c.value, d.value

    def set_config(self, dirs_per_item: int, atoms_per_stage: int, blocks_per_cu: int, min_waves: int = 1):
        _call("ar_signature_plan_set_config", self.handle, dirs_per_item, atoms_per_stage, blocks_per_cu,
              min_waves)

    def run(self, rel, offsets, radius, directions, windows, out=None, use_graph: bool = True):
        images = self._out(offsets, out)
        w = _host_windows(windows)
        self._w = w  # keep the host array alive for the call
        r, o, n, dp, ip = self._args(rel, offsets, directions, images)
        _call("ar_signature_plan_run", self.handle, r, o, n, radius, dp, w.data_ptr(), ip, int(use_graph),
              _stream(self.ctx.device))
        return images

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _L.ar_signature_plan_destroy(self.handle)
            self.handle = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Library:
    """ar_library: normalised BF16 reference images + norms (keeps ref alive).
    With quats (float64 [n_lib][4]) and phase (int32 [n_lib]) it is made by
    ar_library_prepare and can map indexing results to orientations."""

    def __init__(self, ctx: Context, ref_images: torch.Tensor, quats: Optional[torch.Tensor] = None,
                 phase: Optional[torch.Tensor] = None):
        self.ctx = ctx
        _shape(ref_images, (None, None, None), "ref_images")
        n_lib, n_win, n_dir = ref_images.shape
        self.ref = ref_images
        self.n_lib, self.n_win, self.n_dir = n_lib, n_win, n_dir
        d = ctx.device
        h = vp()
        if (quats is None) != (phase is None):
            raise ValueError("give both quats and phase, or neither")
        if quats is None:
            _call("ar_library_create", ctx.handle, _dev(ref_images, torch.float32, d, "ref_images"), n_lib,
                  n_win, n_dir, _stream(d), ctypes.byref(h))
        else:
            _shape(quats, (n_lib, 4), "quats")
            _shape(phase, (n_lib,), "phase")
            _call("ar_library_prepare", ctx.handle, _dev(ref_images, torch.float32, d, "ref_images"), n_lib, n_win,
                  n_dir, _dev(quats, torch.float64, d, "quats"), _dev(phase, torch.int32, d, "phase"), _stream(d),
                  ctypes.byref(h))
        self.handle = h

    def lookup(self, idx: torch.Tensor):
        """-> (quats float64 [*idx.shape][4], phase int32 [*idx.shape]) of the
        entries idx (int32; -1 gives NaN and phase -1)."""
        d = self.ctx.device
        q = torch.empty((*idx.shape, 4), dtype=torch.float64, device=d)
        ph = torch.empty(idx.shape, dtype=torch.int32, device=d)
        _call("ar_library_lookup", self.handle, _dev(idx, torch.int32, d, "idx"), idx.numel(), q.data_ptr(),
              ph.data_ptr(), _stream(d))
        return q, ph

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _L.ar_library_destroy(self.handle)
            self.handle = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ar_index_set_tile(ctx: Context, waves: int, wtm: int, wtn: int, bk: int) -> None:
    """Correlation tile of this context's index calls (see include/araullo.h)."""
    _call("ar_index_set_tile", ctx.handle, waves, wtm, wtn, bk)


def index_orientations(ctx: Context, images: torch.Tensor, library: Library, k: int = 16):
    """-> (top_idx int32 [n_roi][k], top_score float32 [n_roi][k])."""
    d = ctx.device
    _shape(images, (None, library.n_win, library.n_dir), "images")
    n_roi = images.shape[0]
    idx = torch.empty((n_roi, k), dtype=torch.int32, device=d)
    sc = torch.empty((n_roi, k), dtype=torch.float32, device=d)
    _call("index_orientations", ctx.handle, _dev(images, torch.float32, d, "images"), n_roi, library.handle, k,
          idx.data_ptr(), sc.data_ptr(), _stream(d))
    return idx, sc


def index_orientations_ex(ctx: Context, images: torch.Tensor, library: Library, k: int, cand: int):
    """-> (top_idx, top_score, cand_idx int32 [n_roi][cand])."""
    d = ctx.device
    _shape(images, (None, library.n_win, library.n_dir), "images")
    n_roi = images.shape[0]
    idx = torch.empty((n_roi, k), dtype=torch.int32, device=d)
    sc = torch.empty((n_roi, k), dtype=torch.float32, device=d)
    ci = torch.empty((n_roi, cand), dtype=torch.int32, device=d)
    _call("index_orientations_ex", ctx.handle, _dev(images, torch.float32, d, "images"), n_roi, library.handle, k,
          cand, idx.data_ptr(), sc.data_ptr(), ci.data_ptr(), _stream(d))
    return idx, sc, ci


class SparseLUT:
    """ar_sparse_lut: the n_hat strongest entries of each phase's reference
    and the rotated-node look-up table for every library orientation (the
    orientations of phase c are the phase_count[c] rows after those of the
    phases before it)."""

    def __init__(self, ctx: Context, reference: torch.Tensor, directions: torch.Tensor, quats: torch.Tensor,
                 phase_count: Sequence[int], n_hat: int):
        self.ctx = ctx
        d = ctx.device
        _shape(reference, (None, None, None), "reference")
        n_phase, n_win, n_dir = reference.shape
        _shape(directions, (n_dir, 3), "directions")
        if len(phase_count) != n_phase:
            raise ValueError("phase_count needs one entry per phase")
        counts = (i64 * n_phase)(*[int(c) for c in phase_count])
        self.n_phase, self.n_win, self.n_dir, self.n_hat = n_phase, n_win, n_dir, n_hat
        self.n_lib = int(sum(int(c) for c in phase_count))
        if quats.shape != (self.n_lib, 4):
            raise ValueError(f"quats must be [{self.n_lib}][4]")
        h = vp()
        _call("ar_sparse_lut_create", ctx.handle, _dev(reference, torch.float32, d, "reference"), n_phase, n_win,
              _dev(directions, torch.float32, d, "directions"), n_dir, _dev(quats, torch.float64, d, "quats"), counts,
              n_hat, _stream(d), ctypes.byref(h))
        self.handle = h

    def export(self):
        """-> (strong_idx int32 [n_phase][n_hat], strong_val float32 [n_phase][n_hat],
        nodes int32 [n_lib][n_hat])."""
        d = self.ctx.device
        si = torch.empty((self.n_phase, self.n_hat), dtype=torch.int32, device=d)
        sv = torch.empty((self.n_phase, self.n_hat), dtype=torch.float32, device=d)
        nodes = torch.empty((self.n_lib, self.n_hat), dtype=torch.int32, device=d)
        _call("ar_sparse_lut_export", self.handle, si.data_ptr(), sv.data_ptr(), nodes.data_ptr(), _stream(d))
        return si, sv, nodes

    @property
    def screen(self):
        """ROIs per LDS read of the screen: 8 (8-bit codes), 2 or 1 (FP16)."""
        out = ctypes.c_int32()
        _call("ar_sparse_lut_screen", self.handle, ctypes.byref(out))
        return out.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _L.ar_sparse_lut_destroy(self.handle)
            self.handle = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def index_orientations_sparse(ctx: Context, images: torch.Tensor, lut: SparseLUT, k: int = 16):
    """-> (top_idx int32 [n_roi][k], top_score float32 [n_roi][k]): sparse Eq. S1."""
    d = ctx.device
    _shape(images, (None, lut.n_win, lut.n_dir), "images")
    n_roi = images.shape[0]
    idx = torch.empty((n_roi, k), dtype=torch.int32, device=d)
    sc = torch.empty((n_roi, k), dtype=torch.float32, device=d)
    _call("index_orientations_sparse", ctx.handle, _dev(images, torch.float32, d, "images"), n_roi, lut.handle, k,
          idx.data_ptr(), sc.data_ptr(), _stream(d))
    return idx, sc


def ar_fsp_amplitudes(ctx: Context, rel: torch.Tensor, offsets: torch.Tensor, L: int, k_max: float,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """-> amplitudes float32 [n_roi][L][L][L] of Eq. (2) on the cubic grid."""
    d = ctx.device
    _shape(rel, (None, 4), "rel")
    _shape(offsets, (None,), "offsets")
    n_roi = offsets.shape[0] - 1
    if out is None:
        out = torch.empty((n_roi, L, L, L), dtype=torch.float32, device=d)
    _shape(out, (n_roi, L, L, L), "out")
    _call("ar_fsp_amplitudes", ctx.handle, _dev(rel, torch.float32, d, "rel"), _dev(offsets, torch.int64, d, "offsets"),
          n_roi, L, k_max, _dev(out, torch.float32, d, "out"), _stream(d))
    return out


def ar_refine_roi_grid(ctx: Context, centres: torch.Tensor, images: torch.Tensor, counts: torch.Tensor,
                       window_mask: int, kappa: float, h: float, split: int = 5):
    """-> (refined centres float32 [n][3], parent int32 [n]) of the coarse ROIs
    that pass the kappa test (see include/araullo.h)."""
    d = ctx.device
    _shape(images, (None, None, None), "images")
    n_roi, n_win, n_dir = images.shape
    _shape(centres, (n_roi, 3), "centres")
    _shape(counts, (n_roi,), "counts")
    cap = n_roi * split ** 3
    out = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=d)
    par = torch.empty(max(cap, 1), dtype=torch.int32, device=d)
    n = i64()
    _call("ar_refine_roi_grid", ctx.handle, _dev(centres, torch.float32, d, "centres"),
          _dev(images, torch.float32, d, "images"), _dev(counts, torch.int32, d, "counts"), n_roi, n_win, n_dir,
          window_mask, kappa, h, split, out.data_ptr(), par.data_ptr(), cap, ctypes.byref(n), _stream(d))
    return out[:n.value], par[:n.value]


def ar_disorientation_cubic(qa: torch.Tensor, qb: torch.Tensor) -> torch.Tensor:
    d = qa.device
    n = qa.shape[0]
    _shape(qa, (n, 4), "qa")
    _shape(qb, (n, 4), "qb")
    out = torch.empty(n, dtype=torch.float64, device=d)
    _call("ar_disorientation_cubic", _dev(qa, torch.float64, d, "qa"), _dev(qb, torch.float64, d, "qb"), n,
          out.data_ptr(), _stream(d))
    return out


def ar_rotate_reference(ctx: Context, reference: torch.Tensor, directions: torch.Tensor, quats: torch.Tensor,
                        phase: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    d = ctx.device
    _shape(reference, (None, None, None), "reference")
    n_phase, n_win, n_dir = reference.shape
    n_lib = quats.shape[0]
    _shape(directions, (n_dir, 3), "directions")
    _shape(quats, (n_lib, 4), "quats")
    _shape(phase, (n_lib,), "phase")
    o = out if out is not None else torch.empty((n_lib, n_win, n_dir), dtype=torch.float32, device=d)
    _shape(o, (n_lib, n_win, n_dir), "out")
    _call("ar_rotate_reference", ctx.handle, _dev(reference, torch.float32, d, "reference"), n_phase, n_win,
          _dev(directions, torch.float32, d, "directions"), n_dir, _dev(quats, torch.float64, d, "quats"),
          _dev(phase, torch.int32, d, "phase"), n_lib, _dev(o, torch.float32, d, "out"), _stream(d))
    return o


def _sf_shapes(rel, offsets, quats, phase, directions, freqs, targets=None) -> None:
    """Shape checks shared by the structure-factor calls: the kernels index
    quats[4 r + i], phase[r], freqs[p][w] and targets[p][w][v] directly."""
    _shape(rel, (None, 4), "rel")
    _shape(offsets, (None,), "offsets")
    n_roi = offsets.shape[0] - 1
    _shape(quats, (n_roi, 4), "quats")
    _shape(phase, (n_roi,), "phase")
    _shape(directions, (None, 3), "directions")
    _shape(freqs, (None, None), "freqs")
    if targets is not None:
        _shape(targets, (freqs.shape[0], freqs.shape[1], directions.shape[0]), "targets")
    _sf_domain(rel, freqs)


def ar_sf_score_grad(ctx: Context, rel, offsets, quats, phase, directions, freqs, targets, grad: bool = True):
    """-> (score float32 [n_roi], grad float32 [n_roi][4] or None)."""
    d = ctx.device
    _sf_shapes(rel, offsets, quats, phase, directions, freqs, targets)
    n_roi = offsets.shape[0] - 1
    n_phase, n_freq = freqs.shape
    score = torch.empty(n_roi, dtype=torch.float32, device=d)
    g = torch.empty((n_roi, 4), dtype=torch.float32, device=d) if grad else None
    relp = rel if rel.numel() else torch.zeros((1, 4), dtype=torch.float32, device=d)
    _call("ar_sf_score_grad", ctx.handle, _dev(relp, torch.float32, d, "rel"), _dev(offsets, torch.int64, d, "offsets"),
          n_roi, _dev(quats, torch.float32, d, "quats"), _dev(phase, torch.int32, d, "phase"),
          _dev(directions, torch.float32, d, "directions"), directions.shape[0], _dev(freqs, torch.float32, d, "freqs"),
          _dev(targets, torch.float32, d, "targets"), n_phase, n_freq, score.data_ptr(),
          g.data_ptr() if grad else None, _stream(d))
    return score, g


def ar_sf_score_grad_noalloc(ctx: Context, rel, offsets, quats, phase, directions, freqs, targets,
                             score: torch.Tensor, grad: Optional[torch.Tensor] = None) -> None:
    """ar_sf_score_grad into caller-owned outputs (score float32 [n_roi],
    grad float32 [n_roi][4] or None) through the allocation-free entry point.
    Shape checks only: this wrapper allocates nothing, so the 256-turn sine
    domain (max|f| max|x|) is the caller's to keep."""
    d = ctx.device
    _shape(rel, (None, 4), "rel")
    _shape(offsets, (None,), "offsets")
    n_roi = offsets.shape[0] - 1
    _shape(quats, (n_roi, 4), "quats")
    _shape(phase, (n_roi,), "phase")
    _shape(directions, (None, 3), "directions")
    _shape(freqs, (None, None), "freqs")
    n_phase, n_freq = freqs.shape
    _shape(targets, (n_phase, n_freq, directions.shape[0]), "targets")
    _shape(score, (n_roi,), "score")
    if grad is not None:
        _shape(grad, (n_roi, 4), "grad")
    _call("ar_sf_score_grad_noalloc", ctx.handle, _dev(rel, torch.float32, d, "rel"),
          _dev(offsets, torch.int64, d, "offsets"), n_roi, _dev(quats, torch.float32, d, "quats"),
          _dev(phase, torch.int32, d, "phase"), _dev(directions, torch.float32, d, "directions"), directions.shape[0],
          _dev(freqs, torch.float32, d, "freqs"), _dev(targets, torch.float32, d, "targets"), n_phase, n_freq,
          _dev(score, torch.float32, d, "score"), _dev(grad, torch.float32, d, "grad") if grad is not None else None,
          _stream(d))


def ar_sf_score_f64(ctx: Context, rel, offsets, quats, phase, directions, freqs, targets) -> torch.Tensor:
    d = ctx.device
    _sf_shapes(rel, offsets, quats, phase, directions, freqs, targets)
    n_roi = offsets.shape[0] - 1
    n_phase, n_freq = freqs.shape
    score = torch.empty(n_roi, dtype=torch.float64, device=d)
    relp = rel if rel.numel() else torch.zeros((1, 4), dtype=torch.float32, device=d)
    _call("ar_sf_score_f64", ctx.handle, _dev(relp, torch.float32, d, "rel"), _dev(offsets, torch.int64, d, "offsets"),
          n_roi, _dev(quats, torch.float64, d, "quats"), _dev(phase, torch.int32, d, "phase"),
          _dev(directions, torch.float32, d, "directions"), directions.shape[0], _dev(freqs, torch.float64, d, "freqs"),
          _dev(targets, torch.float64, d, "targets"), n_phase, n_freq, score.data_ptr(), _stream(d))
    return score


def ar_sf_amplitudes(ctx: Context, rel, offsets, quats, phase, directions, freqs) -> torch.Tensor:
    d = ctx.device
    _sf_shapes(rel, offsets, quats, phase, directions, freqs)
    n_roi = offsets.shape[0] - 1
    n_phase, n_freq = freqs.shape
    amp = torch.empty((n_roi, n_freq, directions.shape[0]), dtype=torch.float32, device=d)
    relp = rel if rel.numel() else torch.zeros((1, 4), dtype=torch.float32, device=d)
    _call("ar_sf_amplitudes", ctx.handle, _dev(relp, torch.float32, d, "rel"), _dev(offsets, torch.int64, d, "offsets"),
          n_roi, _dev(quats, torch.float32, d, "quats"), _dev(phase, torch.int32, d, "phase"),
          _dev(directions, torch.float32, d, "directions"), directions.shape[0], _dev(freqs, torch.float32, d, "freqs"),
          n_phase, n_freq, amp.data_ptr(), _stream(d))
    return amp


def ar_refine_orientations(ctx: Context, rel, offsets, quats, phase, directions, freqs, targets, steps: int = 50,
                           a0: float = 1e-3):
    """Refines quats in place; -> final score float32 [n_roi]."""
    d = ctx.device
    _sf_shapes(rel, offsets, quats, phase, directions, freqs, targets)
    n_roi = offsets.shape[0] - 1
    n_phase, n_freq = freqs.shape
    score = torch.empty(n_roi, dtype=torch.float32, device=d)
    relp = rel if rel.numel() else torch.zeros((1, 4), dtype=torch.float32, device=d)
    _call("ar_refine_orientations", ctx.handle, _dev(relp, torch.float32, d, "rel"),
          _dev(offsets, torch.int64, d, "offsets"), n_roi, _dev(quats, torch.float32, d, "quats"),
          _dev(phase, torch.int32, d, "phase"), _dev(directions, torch.float32, d, "directions"), directions.shape[0],
          _dev(freqs, torch.float32, d, "freqs"), _dev(targets, torch.float32, d, "targets"), n_phase, n_freq, steps,
          a0, score.data_ptr(), _stream(d))
    return score


PEAK_NAMES = ("hbm_bytes_per_s", "lds_bytes_per_s", "lds_atomics_per_s", "fp32_fma_flop_per_s", "sin_per_s",
              "sin_beside_fma_time_ratio", "bf16_mfma_flop_per_s", "lds_gather8_per_s", "fp32_mfma_flop_per_s")


def ar_measure_peaks(ctx: Context) -> dict:
    """Measured peak rates (see include/araullo.h), keyed by PEAK_NAMES."""
    out = (ctypes.c_double * len(PEAK_NAMES))()
    _call("ar_measure_peaks", ctx.handle, out, len(PEAK_NAMES))
    return dict(zip(PEAK_NAMES, list(out)))
