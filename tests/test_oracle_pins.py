"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), closed forms, invariants, exact rational
arithmetic, NumPy's independent FFT/matmul, or brute force on tiny inputs.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2009_00735_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_worked_examples.json")))


# --------------------------------------------------------------- Eq. (1) constants
def test_frequency_resolution_matches_paper(orc):
    g = GOLDEN["frequency_resolution"]
    _, scale, dR = orc.bin_constants(g["radius_nm"], 2 ** g["m"])
    assert abs(1.0 / dR / 10.0 - g["per_angstrom"]) < 1e-12      # 1/dR in 1/Angstrom
    # 2^m bins of width dR span exactly 2R + 2dR (one pad bin per side)
    assert abs(2 ** g["m"] * dR - (2 * g["radius_nm"] + 2 * dR)) < 1e-12
    assert abs(scale - 1.0 / dR) < 1e-4


def test_fig2_peak_bin_formula(orc):
    g = GOLDEN["fig2_peak_bin"]
    R, nb = g["radius_nm"], 2 ** g["m"]
    _, _, dR = orc.bin_constants(R, nb)
    fs = nb / (2 * (R + dR))
    f = 1.0 / (0.5 * g["lattice_nm_read"])
    assert math.floor(f * nb / fs) == g["bin"]
    # the oracle's window for a +-10 % interval around that spacing holds the bin
    lo, hi = orc.window_bins(R, nb, 0.9 * 0.5 * g["lattice_nm_read"], 1.1 * 0.5 * g["lattice_nm_read"])
    assert lo <= g["bin"] <= hi


def test_al_002_interval_window(orc):
    g = GOLDEN["al_002_interval"]
    lo, hi = orc.window_bins(g["radius_nm"], 2 ** g["m"], g["d_min_nm"], g["d_max_nm"])
    L = 2 * g["radius_nm"] + 2 * g["radius_nm"] / (2 ** (g["m"] - 1) - 1)
    # every index in the window has a spacing L/k inside the printed interval
    for k in range(lo, hi + 1):
        assert g["d_min_nm"] <= L / k <= g["d_max_nm"]
    # and the neighbours outside do not
    assert not (g["d_min_nm"] <= L / (lo - 1) <= g["d_max_nm"])
    assert not (g["d_min_nm"] <= L / (hi + 1) <= g["d_max_nm"])
    assert lo <= GOLDEN["fig2_peak_bin"]["bin"] <= hi


def test_window_bins_rejects_bad_intervals(orc):
    with pytest.raises(ValueError):
        orc.window_bins(2.0, 256, 0.30, 0.20)
    with pytest.raises(ValueError):
        orc.window_bins(2.0, 256, 0.001, 0.002)   # beyond Nyquist
    with pytest.raises(ValueError):
        orc.window_bins(2.0, 256, 10.0, 20.0)     # below index 1


def test_default_windows_separate_the_phases(orc):
    # fcc Al {111},{200},{220},{311} centre the windows; bcc Fe d110/d200/d211
    # fall in windows 2-4 but not window 1.
    w = orc.windows_for(2.0, 1024, synth.window_spacings())
    L = 4.0 + 4.0 / 511
    for j, d in enumerate(synth.WINDOW_SPACINGS_NM):
        assert w[j][0] <= L / d <= w[j][1] + 1
    for d, win in ((0.287 / math.sqrt(2), 1), (0.287 / 2, 2), (0.287 / math.sqrt(6), 3)):
        assert w[win][0] <= round(L / d) <= w[win][1]
    assert not (w[0][0] <= L / (0.287 / math.sqrt(2)) <= w[0][1])


# --------------------------------------------------------------- Eq. (1) binning
def _exact_bin(d, v, R, nb):
    """Eq. (1) in exact rational arithmetic on the float32 inputs."""
    Rf = Fraction(float(np.float32(R)))
    dR = Rf / (nb // 2 - 1)
    s = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, d))
    t = (s + Rf + dR) * nb / (2 * Rf + 2 * dR)
    return math.floor(t), t


def test_eq1_against_exact_rational_arithmetic(orc):
    gen = np.random.default_rng(11)
    R, nb = 2.0, 1024
    dirs = synth.icosphere(2)
    pts = gen.uniform(-1, 1, (4000, 3))
    pts = pts[np.linalg.norm(pts, axis=1) <= 1][:600] * R
    rel = pts.astype(np.float32)
    mism = 0
    for v in dirs[:20]:
        h = orc.sdm_hist(rel, v, R, nb)
        expect = np.zeros(nb, np.int64)
        near_edge = 0
        for d in rel:
            b, t = _exact_bin(d, v, R, nb)
            expect[min(max(b, 0), nb - 1)] += 1
            if abs(t - round(t)) < Fraction(1, 10 ** 4):
                near_edge += 1
        diff = int(np.abs(h - expect).sum())
        assert diff <= 2 * near_edge
        mism += diff
    assert mism <= 4


def test_eq1_hand_placed_atoms(orc):
    """Atoms at hand-chosen bin centres land in the bins Eq. (1) names."""
    R, nb = 2.0, 256
    dR = R / (nb // 2 - 1)
    bins = [1, 2, 64, 127, 128, 129, 200, 254]
    # s_b = -(R + dR) + (b + 1/2) dR, placed along x
    rel = np.array([[-(R + dR) + (b + 0.5) * dR, 0.0, 0.0] for b in bins], np.float32)
    h = orc.sdm_hist(rel, np.array([1, 0, 0], np.float32), R, nb)
    expect = np.zeros(nb, np.int32)
    expect[bins] = 1
    assert np.array_equal(h, expect)
    # the centre of the ROI maps to bin nb/2 (Eq. (1) with s = 0)
    h = orc.sdm_hist(np.zeros((3, 3), np.float32), np.array([0, 0, 1], np.float32), R, nb)
    assert h[nb // 2] == 3 and h.sum() == 3
    # pad bins: no atom inside |s| < R - dR/2 reaches bin 0 or nb-1
    gen = np.random.default_rng(3)
    d = gen.normal(size=(500, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True) * gen.uniform(0, R - dR, (500, 1))).astype(np.float32)
    for v in synth.icosphere(1):
        h = orc.sdm_hist(d, v, R, nb)
        assert h[0] == 0 and h[-1] == 0 and h.sum() == 500


def test_count_conservation_and_gather(orc):
    s = synth.single_roi()
    rel = orc.roi_gather(s.positions, s.centres[0], s.radius)
    # brute force in float64: identical except atoms within 1e-6 nm of the sphere
    r64 = np.linalg.norm(s.positions.astype(np.float64) - s.centres[0].astype(np.float64), axis=1)
    inside = int((r64 <= s.radius).sum())
    boundary = int((np.abs(r64 - s.radius) < 1e-6).sum())
    assert abs(len(rel) - inside) <= boundary
    assert 100 <= len(rel) <= 160
    for v in s.directions[::37]:
        assert orc.sdm_hist(rel, v, s.radius, s.nbins).sum() == len(rel)


# --------------------------------------------------------------- amplitude spectrum
def test_amplitudes_against_numpy_rfft(orc):
    gen = np.random.default_rng(5)
    for nb in (256, 1024, 4096):
        h = gen.integers(0, 40, nb).astype(np.int32)
        a = orc.amplitudes(h)
        ref = np.abs(np.fft.rfft(h.astype(np.float64)))
        assert np.allclose(a, ref, rtol=0, atol=1e-9 * h.sum())


def test_amplitude_invariants(orc):
    gen = np.random.default_rng(6)
    nb = 512
    h = gen.integers(0, 7, nb).astype(np.int32)
    a = orc.amplitudes(h)
    # A_0 = number of atoms and is the spectrum maximum
    assert a[0] == h.sum() and a.max() == a[0]
    # Parseval: N sum h^2 = A_0^2 + 2 sum_{0<k<N/2} A_k^2 + A_{N/2}^2
    lhs = nb * int((h.astype(np.int64) ** 2).sum())
    rhs = a[0] ** 2 + 2 * (a[1:nb // 2] ** 2).sum() + a[nb // 2] ** 2
    assert abs(lhs - rhs) <= 1e-9 * lhs


def test_amplitude_closed_forms(orc):
    nb = 256
    h = np.zeros(nb, np.int32)
    h[37] = 1
    assert np.allclose(orc.amplitudes(h), 1.0, atol=1e-12)        # one atom
    for db in (1, 5, 64, 100):
        h = np.zeros(nb, np.int32)
        h[10] = 1
        h[10 + db] = 1
        k = np.arange(nb // 2 + 1)
        assert np.allclose(orc.amplitudes(h), 2 * np.abs(np.cos(np.pi * k * db / nb)), atol=1e-12)
    # comb of planes every s bins: A at multiples of nb/s equals the atom count
    s = 16
    h = np.zeros(nb, np.int32)
    h[3::s] = 5
    a = orc.amplitudes(h)
    for j in range(0, nb // 2 + 1, nb // s):
        assert abs(a[j] - h.sum()) < 1e-9
    others = [k for k in range(nb // 2 + 1) if k % (nb // s)]
    assert np.all(a[others] < 1e-9)


@pytest.mark.parametrize("kind,a", [("fcc", 0.405), ("bcc", 0.287)])
def test_lattice_plane_peaks(orc, kind, a):
    """Noise-free unrotated crystals: along <100>, <110>, <111> the spectrum
    peaks at the spacing of the first allowed plane family (Sec. 3.1, Fig. 2)."""
    R, nb = 2.0, 1024
    pts = synth.lattice_in_ball(kind, a, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), R + 0.5)
    centre = np.array([0.0137, -0.0071, 0.0049], np.float32)      # generic in-cell position
    rel = orc.roi_gather(pts.astype(np.float32), centre, R)
    L = 2 * R + 2 * R / (nb // 2 - 1)
    if kind == "fcc":
        spacing = {1: a / 2, 2: a / math.sqrt(8), 3: a / math.sqrt(3)}
    else:
        spacing = {1: a / 2, 2: a / math.sqrt(2), 3: a / math.sqrt(12)}
    for v in synth.cubic_directions_26():
        n_nonzero = int(np.count_nonzero(np.abs(v) > 0.1))
        kstar = L / spacing[n_nonzero]
        amp = orc.amplitudes(orc.sdm_hist(rel, v, R, nb))
        assert amp[0] == len(rel)
        lo = 4
        hi = int(1.5 * kstar)
        kmax = lo + int(np.argmax(amp[lo:hi + 1]))
        assert kmax in (math.floor(kstar), math.ceil(kstar)), (kind, v, kstar, kmax)
        assert amp[kmax] > 0.5 * len(rel)


def test_paper_fig2_bin_on_a_crystal(orc):
    """R = 2 nm, m = 8, fcc Al along [100]: the d200 peak sits in bin 19 or 20
    (the caption's floor rule names 19; k* = 19.91)."""
    g = GOLDEN["fig2_peak_bin"]
    R, nb = g["radius_nm"], 2 ** g["m"]
    pts = synth.lattice_in_ball("fcc", 0.405, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), R + 0.5)
    rel = orc.roi_gather(pts.astype(np.float32), np.array([0.011, 0.003, -0.002], np.float32), R)
    amp = orc.amplitudes(orc.sdm_hist(rel, np.array([1, 0, 0], np.float32), R, nb))
    k = 4 + int(np.argmax(amp[4:30]))
    assert k in (g["bin"], g["bin"] + 1)


def test_signature_images_are_window_maxima(orc):
    s = synth.single_roi()
    w = orc.windows_for(s.radius, s.nbins, s.spacings)
    dirs = s.directions[:16]
    img, cnt = orc.signatures(s.positions, s.centres, s.radius, dirs, s.nbins, w)
    rel = orc.roi_gather(s.positions, s.centres[0], s.radius)
    assert cnt[0] == len(rel)
    hist, amp = orc.sdm_debug(rel, s.radius, dirs, s.nbins)
    for v in range(len(dirs)):
        ref = np.abs(np.fft.rfft(hist[v].astype(np.float64)))
        for j, (lo, hi) in enumerate(w):
            assert abs(img[0, j, v] - ref[lo:hi + 1].max()) < 1e-9 * cnt[0]
    # an empty ROI gives zero images and count 0
    img, cnt = orc.signatures(s.positions, np.array([[50.0, 50, 50]], np.float32), s.radius, dirs, s.nbins, w)
    assert cnt[0] == 0 and np.all(img == 0)


# --------------------------------------------------------------- indexing
def test_normalise(orc):
    gen = np.random.default_rng(8)
    x = gen.uniform(0, 5, (3, 4, 50)).astype(np.float32)
    x[1, 2] = 0
    y = orc.normalise(x)
    m = x.astype(np.float64).max(axis=2, keepdims=True)
    assert np.allclose(y[0], x[0] / m[0], rtol=1e-15)
    assert np.all(y[1, 2] == 0)
    assert np.allclose(np.delete(y.max(axis=2).ravel(), 6), 1.0)


def test_ssd_against_matmul_expansion(orc):
    gen = np.random.default_rng(9)
    S = gen.random((5, 300))
    L = gen.random((40, 300))
    idx, sc = orc.index_topk(S, L, 40)
    full = (S ** 2).sum(1)[:, None] + (L ** 2).sum(1)[None, :] - 2 * S @ L.T
    for r in range(5):
        assert np.allclose(sc[r], full[r, idx[r]], rtol=1e-12, atol=1e-10)
        assert np.all(np.diff(sc[r]) >= 0)
        assert set(idx[r]) == set(range(40))
    pairs = orc.ssd_pairs(S, L, [0, 3, 4], [39, 0, 17])
    assert np.allclose(pairs, [full[0, 39], full[3, 0], full[4, 17]], rtol=1e-12)


def test_index_brute_force_small(orc):
    gen = np.random.default_rng(10)
    S = gen.random((3, 17))
    L = gen.random((10, 17))
    L[7] = L[2]                                   # exact tie: lower index first
    S[1] = L[2]
    idx, sc = orc.index_topk(S, L, 4)
    for r in range(3):
        d = [sum((S[r][j] - L[l][j]) ** 2 for j in range(17)) for l in range(10)]
        order = sorted(range(10), key=lambda l: (d[l], l))[:4]
        assert list(idx[r]) == order
        assert np.allclose(sc[r], [d[l] for l in order], rtol=1e-14)
    assert list(idx[1][:2]) == [2, 7] and sc[1][0] == 0 and sc[1][1] == 0


def test_self_indexing(orc):
    gen = np.random.default_rng(12)
    L = gen.random((30, 64))
    idx, sc = orc.index_topk(L[[4, 9, 22]], L, 3)
    assert list(idx[:, 0]) == [4, 9, 22] and np.all(sc[:, 0] == 0)


# --------------------------------------------------------------- disorientation
def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_cubic_group_is_the_rotation_group_of_the_cube(orc):
    G = orc.cubic_group()
    mats = [synth.quat_matrix(q) for q in G]
    keys = set()
    for M in mats:
        # a signed permutation matrix with determinant +1
        assert np.allclose(np.abs(M).sum(0), 1) and np.allclose(np.abs(M).sum(1), 1)
        assert np.allclose(np.round(M), M, atol=1e-12) and abs(np.linalg.det(M) - 1) < 1e-12
        keys.add(tuple(np.round(M).astype(int).ravel()))
    assert len(keys) == 24                         # all 24 distinct rotations


def test_disorientation_special_cases(orc):
    I = np.array([1.0, 0, 0, 0])
    cases = [
        (synth.quat_axis_angle([0, 0, 1], 90), 0.0),
        (synth.quat_axis_angle([1, 1, 1], 120), 0.0),
        (synth.quat_axis_angle([1, 1, 0], 180), 0.0),
        (synth.quat_axis_angle([1, 1, 1], 60), 60.0),          # Sigma 3 twin
        (synth.quat_axis_angle([0, 0, 1], 45), 45.0),
        (synth.quat_axis_angle([0, 0, 1], 30), 30.0),
        (synth.quat_axis_angle([1, 0, 0], 80), 10.0),
        (I, 0.0),
    ]
    for q, expect in cases:
        d = orc.disorientation_cubic(I, q)[0]
        assert abs(d - expect) < 1e-9, (q, d, expect)


def test_disorientation_random_pairs(orc):
    g = GOLDEN["mackenzie_max_deg"]
    gen = np.random.default_rng(13)
    qa = synth.shoemake(20000, gen)
    qb = synth.shoemake(20000, gen)
    d = orc.disorientation_cubic(qa, qb)
    assert d.max() <= g["max_deg"] + 0.05
    assert abs(d.mean() - g["mean_deg"]) < 0.3
    # symmetric, and invariant under crystal symmetry on either side
    assert np.allclose(orc.disorientation_cubic(qb[:200], qa[:200]), d[:200], atol=1e-9)
    G = orc.cubic_group()
    qa2 = np.array([_qmul(q, G[i % 24]) for i, q in enumerate(qa[:200])])
    qb2 = np.array([_qmul(q, G[(7 * i) % 24]) for i, q in enumerate(qb[:200])])
    assert np.allclose(orc.disorientation_cubic(qa2, qb2), d[:200], atol=1e-7)
    # brute force over both symmetry sides
    for i in range(50):
        best = 0.0
        inv = qa[i] * np.array([1, -1, -1, -1])
        for Sa in G:
            for Sb in G:
                m = _qmul(_qmul(_qmul(Sa, inv), qb[i]), Sb)
                best = max(best, abs(m[0]))
        assert abs(2 * math.degrees(math.acos(min(1.0, best))) - d[i]) < 1e-7


# --------------------------------------------------------------- rotated references
def test_rotated_nodes_identity_and_mesh_symmetry(orc):
    dirs = synth.icosphere(3)
    lut = orc.rotated_nodes(np.array([[1.0, 0, 0, 0]]), dirs)
    assert np.array_equal(lut[0], np.arange(len(dirs)))
    # 180 deg about z maps the icosphere onto itself: a permutation
    q = synth.quat_axis_angle([0, 0, 1], 180)
    lut = orc.rotated_nodes(q[None], dirs)[0]
    assert len(set(lut)) == len(dirs)
    d64 = dirs.astype(np.float64)
    target = d64 * np.array([-1, -1, 1])
    brute = np.argmax(target @ d64.T, axis=1)
    assert np.array_equal(lut, brute)
    # a generic rotation: nearest node by brute force in NumPy
    qr = synth.random_orientations(3, 1)
    lut = orc.rotated_nodes(qr, dirs)
    for l in range(3):
        rt = d64 @ synth.quat_matrix(qr[l])        # rows: R^T n_v
        assert np.array_equal(lut[l], np.argmax(rt @ d64.T, axis=1))


# --------------------------------------------------------------- structure factor
def test_sf_one_and_two_atoms(orc):
    dirs = synth.icosphere(2)
    q = synth.random_orientations(1, 2)[0]
    f = np.array([4.2767, 4.9383])
    a = orc.sf_amplitudes(np.array([[0.3, -0.2, 0.1]], np.float32), q, dirs, f)
    assert np.allclose(a, 1.0, atol=1e-12)
    x0 = np.array([0.31, -0.12, 0.2], np.float32)
    a = orc.sf_amplitudes(np.stack([x0, -x0]), q, dirs, f)
    u = dirs.astype(np.float64) @ synth.quat_matrix(q).T
    for w in range(2):
        expect = np.abs(np.cos(2 * np.pi * f[w] * (u @ x0.astype(np.float64))))
        assert np.allclose(a[w], expect, atol=1e-12)
    # score is constant (gradient zero) for one atom, zero when T = A
    T = np.full((2, len(dirs)), 0.7)
    g = orc.sf_grad_fd(np.array([[0.3, -0.2, 0.1]], np.float32), q, dirs, f, T)
    assert np.allclose(g, 0, atol=1e-6)
    assert orc.sf_score(np.stack([x0, -x0]), q, dirs, f, a) == 0.0
    # q and -q are the same rotation
    assert abs(orc.sf_score(np.stack([x0, -x0]), -q, dirs, f, T) - orc.sf_score(np.stack([x0, -x0]), q, dirs, f, T)) < 1e-12


def test_sf_fd_gradient_matches_closed_form(orc):
    """Two atoms at +-x0: A_v = |cos(2 pi f u_v.x0)| with u_v = R(q/|q|) n_v.
    The closed-form derivative (chain rule through R(q) written here with
    NumPy) must agree with the oracle's central differences."""
    dirs = synth.icosphere(1)
    f = np.array([4.9383])
    x0 = np.array([0.21, -0.07, 0.13])
    T = np.full((1, len(dirs)), 0.4)
    q = np.array([0.9, 0.2, -0.3, 0.25])
    rel = np.stack([x0, -x0]).astype(np.float32)
    x0 = rel[0].astype(np.float64)

    def J(qq):
        u = dirs.astype(np.float64) @ synth.quat_matrix(qq).T
        return float(((np.abs(np.cos(2 * np.pi * f[0] * (u @ x0))) - T[0]) ** 2).sum())

    # derivative of J(q/|q|) by complex-step-free exact differentiation:
    # dR/dq for the normalised quaternion, then project out the radial part.
    def dR(qn):
        w, x, y, z = qn
        return [np.array([[0, -2 * z, 2 * y], [2 * z, 0, -2 * x], [-2 * y, 2 * x, 0]]),
                np.array([[0, 2 * y, 2 * z], [2 * y, -4 * x, -2 * w], [2 * z, 2 * w, -4 * x]]),
                np.array([[-4 * y, 2 * x, 2 * w], [2 * x, 0, 2 * z], [-2 * w, 2 * z, -4 * y]]),
                np.array([[-4 * z, -2 * w, 2 * x], [2 * w, -4 * z, 2 * y], [2 * x, 2 * y, 0]])]
    nq = np.linalg.norm(q)
    qn = q / nq
    u = dirs.astype(np.float64) @ synth.quat_matrix(qn).T
    ph = 2 * np.pi * f[0] * (u @ x0)
    A = np.abs(np.cos(ph))
    dA_dph = -np.sign(np.cos(ph)) * np.sin(ph)
    coef = 2 * (A - T[0]) * dA_dph * 2 * np.pi * f[0]          # dJ/d(u.x0)
    gn = np.array([float((coef * ((dirs.astype(np.float64) @ D.T) @ x0)).sum()) for D in dR(qn)])
    g = (gn - qn * (qn @ gn)) / nq
    fd = orc.sf_grad_fd(rel, q, dirs, f, T, 1e-6)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)
    assert abs(orc.sf_score(rel, q, dirs, f, T) - J(q)) < 1e-10


def test_sf_minimum_at_true_orientation(orc):
    """Noise-free crystal: J is lower at the true orientation than a few
    degrees away, with the target taken from the unrotated crystal."""
    dirs = synth.icosphere(3)
    f = np.array([4.2767, 4.9383, 6.9838, 8.1892])
    ref = synth.lattice_in_ball("fcc", 0.405, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), 1.5)
    rel0 = orc.roi_gather(ref.astype(np.float32), np.array([0.01, 0.02, -0.015], np.float32), 1.2)
    T = orc.sf_amplitudes(rel0, np.array([1.0, 0, 0, 0]), dirs, f)
    qt = synth.random_orientations(1, 4)[0]
    pts = synth.lattice_in_ball("fcc", 0.405, qt, np.zeros(3), np.zeros(3), 1.5)
    rel = orc.roi_gather(pts.astype(np.float32), np.array([0.0, 0.0, 0.0], np.float32), 1.2)
    j0 = orc.sf_score(rel, qt, dirs, f, T)
    for ax in ([1, 0, 0], [0, 1, 1], [1, -2, 1]):
        qp = _qmul(qt, synth.quat_axis_angle(ax, 4.0))
        assert orc.sf_score(rel, qp, dirs, f, T) > j0


def test_sf_refinement_trajectory_recovers_truth(orc):
    """Noise-free crystal, start 3 degrees off: the FP64 backtracking descent
    ends within 0.1 degree of the true orientation and lowers J."""
    dirs = synth.icosphere(2)
    f = np.array([4.2767, 4.9383, 6.9838, 8.1892])
    ref = synth.lattice_in_ball("fcc", 0.405, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), 2.5)
    rel0 = orc.roi_gather(ref.astype(np.float32), np.array([0.01, 0.02, -0.015], np.float32), 2.0)
    T = orc.sf_amplitudes(rel0, np.array([1.0, 0, 0, 0]), dirs, f)
    qt = synth.random_orientations(1, 4)[0]
    p = synth.lattice_in_ball("fcc", 0.405, qt, np.zeros(3), np.zeros(3), 2.5)
    rel = orc.roi_gather(p.astype(np.float32), np.zeros(3, np.float32), 2.0)
    q0 = _qmul(qt, synth.quat_axis_angle([1, 2, -1], 3.0))
    qr, J = orc.sf_refine(rel, q0, dirs, f, T, steps=40)
    assert J < orc.sf_score(rel, q0, dirs, f, T)
    assert orc.disorientation_cubic(qr, qt)[0] < 0.1
