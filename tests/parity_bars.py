"""Tolerances shared by the GPU parity tests.

Images (window maxima of the amplitude spectrum, Sec. 2.2 and the
supplement's reconstruction parameters) are compared per value at relative
1e-5, with an absolute floor of 1e-6 A_0 (A_0 = N_w, the zero-frequency
amplitude and the largest of every spectrum) so that values near zero,
where a relative bar is ill-posed, are held to a fraction of the spectrum's
scale.  Whole spectra are compared per spectrum at 1e-5 A_0."""
import numpy as np

IMAGE_REL = 1e-5
IMAGE_FLOOR = 1e-6
SPECTRUM_REL = 1e-5


def image_excess(got, ref, n_w):
    """Largest |got - ref| / (1e-5 |ref| + 1e-6 n_w) over the arrays (<= 1 passes)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    bar = IMAGE_REL * np.abs(ref) + IMAGE_FLOOR * np.maximum(np.asarray(n_w, np.float64), 1.0)
    return float(np.max(np.abs(got - ref) / bar)) if got.size else 0.0


def assert_images(got, ref, n_w, what=""):
    """Per-value image bar: |got - ref| <= 1e-5 |ref| + 1e-6 max(n_w, 1).
    n_w broadcasts against the arrays (a scalar, or per-ROI counts shaped to
    the leading axis)."""
    e = image_excess(got, ref, n_w)
    assert e <= 1.0, f"{what} image error {e:.3g} x the bar (relative 1e-5 + 1e-6 N_w)"


def assert_spectra(got, ref, n_w, what=""):
    """Per-spectrum bar: max_k |A_gpu[k] - A_orc[k]| <= 1e-5 A_0."""
    err = float(np.max(np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))))
    assert err <= SPECTRUM_REL * max(float(n_w), 1.0), f"{what} spectrum error {err:.3g}"
