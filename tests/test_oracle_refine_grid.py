"""Pins of the oracle's adaptive ROI-grid refinement (reading R15): a hand
example of the kappa test (per-atom peak against the best ROI, per window,
window mask, empty ROIs), and the geometry of the split (the refined centres
tile the parent cell: spacing h/s, mean at the parent, extent h - h/s)."""
import numpy as np


def test_kappa_selection_hand_example(orc):
    # 4 ROIs (16, 16, 1 and 0 atoms), 2 windows, 3 directions; every value a
    # binary fraction, so every comparison below is exact.  Per-atom peaks:
    #   window 0: 8/16 = 0.5, 4/16 = 0.25, 0.4375, 0 (empty)  -> threshold 0.75 * 0.5 = 0.375
    #   window 1: 1/16 = 0.0625, 12/16 = 0.75, 0.25, 0         -> threshold 0.75 * 0.75 = 0.5625
    img = np.array([[[1, 8, 2], [0, 1, 0.5]],
                    [[4, 1, 0], [12, 2, 1]],
                    [[0.4375, 0.125, 0], [0.25, 0, 0]],
                    [[5, 5, 5], [5, 5, 5]]], np.float64)
    counts = np.array([16, 16, 1, 0], np.int32)
    cen = np.zeros((4, 3), np.float32)
    keep, out, par = orc.refine_roi_grid(cen, img, counts, 0b01, 0.75, 2.0, 2)
    assert keep.tolist() == [1, 0, 1, 0] and par.tolist() == [0] * 8 + [2] * 8
    keep, out, par = orc.refine_roi_grid(cen, img, counts, 0b10, 0.75, 2.0, 2)
    assert keep.tolist() == [0, 1, 0, 0]
    keep, out, par = orc.refine_roi_grid(cen, img, counts, 0b11, 0.75, 2.0, 2)
    assert keep.tolist() == [1, 1, 1, 0] and len(out) == 24
    # exactly at the threshold is kept
    img2 = img.copy()
    img2[1, 0, 0] = 6.0                                          # 6/16 = 0.375 = 0.75 * 0.5
    keep, _, _ = orc.refine_roi_grid(cen, img2, counts, 0b01, 0.75, 2.0, 2)
    assert keep.tolist() == [1, 1, 1, 0]
    # no window selected, or kappa above 1: nothing kept
    assert orc.refine_roi_grid(cen, img, counts, 0, 0.75, 2.0, 2)[0].sum() == 0
    assert orc.refine_roi_grid(cen, img, counts, 0b11, 1.01, 2.0, 2)[0].sum() == 0


def test_split_geometry(orc):
    h = 2.0
    cen = np.array([[1.5, -2.25, 10.0]], np.float32)
    img = np.ones((1, 1, 4))
    for s in (2, 4, 5):
        keep, out, par = orc.refine_roi_grid(cen, img, [7], 1, 0.75, h, s)
        assert keep.tolist() == [1] and len(out) == s ** 3
        g = out.astype(np.float64).reshape(s, s, s, 3)
        assert np.allclose(g.mean(axis=(0, 1, 2)), cen[0], atol=1e-5)
        assert np.allclose(np.diff(g[:, 0, 0, 0]), h / s, atol=1e-5)      # i along x
        assert np.allclose(np.diff(g[0, :, 0, 1]), h / s, atol=1e-5)      # j along y
        assert np.allclose(np.diff(g[0, 0, :, 2]), h / s, atol=1e-5)      # k along z
        assert np.allclose(g[-1, -1, -1] - g[0, 0, 0], h - h / s, atol=1e-5)


def test_invalid_arguments_are_refused(orc):
    import pytest
    cen = np.zeros((1, 3), np.float32)
    with pytest.raises(ValueError):                       # 33 windows: the mask has 32 bits
        orc.refine_roi_grid(cen, np.ones((1, 33, 4)), [7], 1, 0.75, 2.0, 2)
    with pytest.raises(ValueError):
        orc.refine_roi_grid(cen, np.ones((1, 1, 4)), [7], 1, 0.75, 2.0, 0)
    with pytest.raises(ValueError):                       # not a single-precision number
        orc.refine_roi_grid(cen, np.ones((1, 1, 4)), [7], 1, 0.75, 0.1, 2)
    keep, out, _ = orc.refine_roi_grid(cen, np.ones((1, 32, 4)), [7], 1 << 31, 0.75, float(np.float32(0.1)), 2)
    assert keep.tolist() == [1] and len(out) == 8
