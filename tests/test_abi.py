"""The C-ABI library loads, exports every symbol include/araullo.h declares,
and its host-only helpers agree with the oracle (no GPU compute here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "araullo.h")
LIB = os.path.join(ROOT, "paper_2009_00735_amd", "libaraullo.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text,
                       flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("araullo_signatures", "index_orientations", "ar_roi_gather", "ar_library_create",
                 "ar_disorientation_cubic", "ar_sf_score_grad", "ar_signature_plan_run", "ar_refine_orientations"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_2009_00735_amd.build)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2009_00735_amd import native
    assert set(declared_functions()) <= set(native.EXPORTED)


def test_window_bins_matches_oracle(orc):
    from paper_2009_00735_amd import native
    from paper_2009_00735_amd import synth
    for R, nb in ((1.0, 256), (2.0, 256), (2.0, 1024), (2.0, 4096), (3.3, 2048)):
        for dmin, dmax in synth.window_spacings():
            try:
                expect = orc.window_bins(R, nb, dmin, dmax)
            except ValueError:
                with pytest.raises(native.AraulloError):
                    native.ar_window_bins(R, nb, dmin, dmax)
                continue
            assert native.ar_window_bins(R, nb, dmin, dmax) == expect


def test_window_bins_errors():
    from paper_2009_00735_amd import native
    for args in ((2.0, 300, 0.18, 0.22), (2.0, 8192, 0.18, 0.22), (-1.0, 256, 0.18, 0.22),
                 (2.0, 256, 0.3, 0.2), (2.0, 256, 0.001, 0.0011)):
        with pytest.raises(native.AraulloError) as e:
            native.ar_window_bins(*args)
        assert e.value.status == -1
        assert str(e.value)


def test_null_context_is_rejected():
    from paper_2009_00735_amd import native
    st = native._L.araullo_signatures(None, None, 0, None, 1, 2.0, None, 1, 1024, None, 1, None, None, None)
    assert st == -1
    assert b"NULL" in native._L.ar_last_error(None)


class _HostCtx:
    """Stand-in context: the binding's shape checks run before any device
    pointer is taken, so they can be exercised on the CPU."""
    device = "cpu"
    handle = None


def test_binding_rejects_mismatched_shapes():
    import torch
    from paper_2009_00735_amd import native
    c = _HostCtx()
    rel = torch.zeros((10, 4))
    off = torch.tensor([0, 4, 10])
    dirs = torch.zeros((12, 3))
    freqs = torch.ones((1, 4))
    targets = torch.zeros((1, 4, 12))
    good = dict(rel=rel, offsets=off, quats=torch.zeros((2, 4)), phase=torch.zeros(2, dtype=torch.int32),
                directions=dirs, freqs=freqs, targets=targets)
    for key, bad in (("quats", torch.zeros((1, 4))), ("quats", torch.zeros((2, 3))), ("phase", torch.zeros(3)),
                     ("directions", torch.zeros((12, 4))), ("targets", torch.zeros((1, 4, 11))),
                     ("targets", torch.zeros((2, 4, 12))), ("rel", torch.zeros((10, 3)))):
        args = dict(good, **{key: bad})
        with pytest.raises(ValueError, match=key if key != "rel" else "rel"):
            native.ar_sf_score_grad(c, **args)
        with pytest.raises(ValueError):
            native.ar_refine_orientations(c, **args)
    with pytest.raises(ValueError, match="quats"):
        native.ar_rotate_reference(c, torch.zeros((1, 4, 12)), dirs, torch.zeros((5, 3)), torch.zeros(5))
    with pytest.raises(ValueError, match="phase"):
        native.ar_rotate_reference(c, torch.zeros((1, 4, 12)), dirs, torch.zeros((5, 4)), torch.zeros(4))

    class _Lib:
        n_win, n_dir = 4, 12
    with pytest.raises(ValueError, match="images"):
        native.index_orientations(c, torch.zeros((3, 4, 11)), _Lib(), 4)
    with pytest.raises(ValueError, match="counts"):
        native.ar_refine_roi_grid(c, torch.zeros((3, 3)), torch.zeros((3, 4, 12)), torch.zeros(2), 1, 0.75, 1.0)


def test_binding_rejects_phases_beyond_the_sine_domain():
    """max|f| max|x| above 256 turns leaves the domain of the hardware sine
    and cosine, so the structure-factor calls refuse it."""
    import torch
    from paper_2009_00735_amd import native
    c = _HostCtx()
    rel = torch.zeros((10, 4))
    rel[3, :3] = torch.tensor([30.0, 0.0, 0.0])
    args = dict(rel=rel, offsets=torch.tensor([0, 10]), quats=torch.zeros((1, 4)),
                phase=torch.zeros(1, dtype=torch.int32), directions=torch.zeros((12, 3)),
                targets=torch.zeros((1, 4, 12)))
    with pytest.raises(ValueError, match="turns"):
        native.ar_sf_score_grad(c, freqs=torch.full((1, 4), 9.0), **args)
    native._sf_domain(rel, torch.full((1, 4), 8.5))   # 255 turns: inside
