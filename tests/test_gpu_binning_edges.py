"""Eq. (1) at its edge cases, GPU against the oracle (Sec. 2.2, Eq. (1);
supplement, "Controlled windowing of the SDMs"): atoms placed exactly on bin
edges and one or two ulps to either side, exactly at +-R along the
directions, and at the ROI centre.  Histograms must be bit-exact and every
direction must conserve the ROI's atom count.

Placement is drawn by hypothesis (derandomized, so every run draws the same
cases).  For an axis direction the projection s equals the coordinate along
that axis, so a coordinate s_k = k / inv - (R + dR), rounded to FP32 and
nudged by whole ulps, puts the atom at the FP32 boundary between bins k - 1
and k of the canonical sequence t = (s + (R + dR)) * inv."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

pytestmark = pytest.mark.gpu

DIRS = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1],
                 [1, 1, 0], [1, -1, 0], [1, 1, 1], [-1, 1, 1], [0.36, -0.48, 0.8], [2, 3, 6]], np.float64)
DIRS = (DIRS / np.linalg.norm(DIRS, axis=1, keepdims=True)).astype(np.float32)


@pytest.fixture(scope="module")
def nat():
    from paper_2009_00735_amd import native
    return native


@pytest.fixture(scope="module")
def ctx(nat):
    return nat.Context(0)


def _nudge(x, ulps):
    x = np.float32(x)
    step = np.float32(np.inf) if ulps > 0 else np.float32(-np.inf)
    for _ in range(abs(ulps)):
        x = np.nextafter(x, step)
    return x


def _edge_coordinate(R, nb, k, ulps):
    dR = R / (nb / 2 - 1)
    hi = np.float32(R + dR)
    inv = np.float32(nb / (2 * R + 2 * dR))
    return _nudge(np.float64(k) / np.float64(inv) - np.float64(hi), ulps)


atom = st.one_of(
    st.tuples(st.just("edge"), st.integers(1, 4095), st.integers(-2, 2), st.integers(0, 2),
              st.floats(-0.25, 0.25, width=32), st.floats(-0.25, 0.25, width=32)),
    st.tuples(st.just("radius"), st.integers(0, len(DIRS) - 1), st.integers(-2, 2), st.sampled_from([-1, 1])),
    st.just(("centre",)),
)


@settings(derandomize=True, max_examples=40, deadline=None, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(nb=st.sampled_from([256, 1024, 4096]), R=st.sampled_from([1.0, 1.7, 2.0, 2.5]),
       centre=st.sampled_from([(0.0, 0.0, 0.0), (10.25, -3.5, 7.0), (0.1, 0.2, 0.3)]),
       atoms=st.lists(atom, min_size=1, max_size=64))
def test_bin_edges_bitexact(nat, ctx, orc, nb, R, centre, atoms):
    c = np.array(centre, np.float32)
    rows = []
    for a in atoms:
        if a[0] == "edge":
            _, k, ulps, axis, y, z = a
            k = 1 + (k - 1) % (nb - 1)             # interior edges: |s| <= R
            d = np.zeros(3, np.float32)
            d[axis] = _edge_coordinate(R, nb, k, ulps)
            d[(axis + 1) % 3] = np.float32(y)
            d[(axis + 2) % 3] = np.float32(z)
        elif a[0] == "radius":
            _, v, ulps, sign = a
            d = np.array([_nudge(np.float32(sign * R * x), ulps) for x in DIRS[v].astype(np.float64)], np.float32)
        else:
            d = np.zeros(3, np.float32)
        rows.append(d + c if np.any(c) else d)    # FP32 sum: the kernel recovers d as p - c in FP32
    pos = np.array(rows, np.float32)
    cen = c[None]
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    hist, _ = nat.araullo_sdm(ctx, dev(pos), dev(cen), R, dev(DIRS), nb)
    rel = orc.roi_gather(pos, cen[0], R)
    h_ref, _ = orc.sdm_debug(rel, R, DIRS, nb, spectra=False)
    h = hist[0].cpu().numpy()
    assert np.array_equal(h, h_ref)
    assert np.all(h.sum(axis=1) == len(rel))
