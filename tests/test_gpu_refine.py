"""Structure-factor score, its hand-written adjoint and the refinement loop:
GPU (FP32) against the FP64 oracle; gradient against FP64 central finite
differences to a relative 1e-3."""
import numpy as np
import pytest
import torch

from paper_2009_00735_amd import synth

pytestmark = pytest.mark.gpu

F_AL = np.array([4.2767, 4.9383, 6.9838, 8.1892])   # 1/d of fcc Al {111},{200},{220},{311}


@pytest.fixture(scope="module")
def nat():
    from paper_2009_00735_amd import native
    return native


@pytest.fixture(scope="module")
def ctx(nat):
    return nat.Context(0)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def make_case(orc, level, n_roi, sigma=0.05, eta=0.5, R=2.0, seed=0, off_deg=3.0, dirs=None):
    """ROIs cut from fcc Al crystals at random true orientations, start
    orientations rotated `off_deg` away; target from the unrotated crystal
    (FP64 oracle, cast to float32 and shared by both sides).  Directions:
    the icosphere of `level` unless `dirs` is given."""
    dirs = synth.icosphere(level) if dirs is None else dirs
    ref = synth.lattice_in_ball("fcc", 0.405, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), R + 0.5)
    rel0 = orc.roi_gather(ref.astype(np.float32), np.array([0.01, 0.02, -0.015], np.float32), R)
    T = orc.sf_amplitudes(rel0, np.array([1.0, 0, 0, 0]), dirs, F_AL).astype(np.float32)
    rels, q0s, qts = [], [], []
    gen = np.random.default_rng(seed)
    for i in range(n_roi):
        qt = synth.random_orientations(1, 300 + seed * 100 + i)[0]
        p = synth.lattice_in_ball("fcc", 0.405, qt, gen.random(3), np.zeros(3), R + 0.5)
        keep = synth.delete_exact(len(p), eta, gen)
        p = (p[keep] + gen.normal(0, sigma, (len(keep), 3))).astype(np.float32)
        rels.append(orc.roi_gather(p, np.zeros(3, np.float32), R))
        axis = gen.normal(size=3)
        q0s.append(qmul(qt, synth.quat_axis_angle(axis, off_deg)))
        qts.append(qt)
    offsets = np.concatenate([[0], np.cumsum([len(r) for r in rels])]).astype(np.int64)
    rel4 = np.zeros((offsets[-1], 4), np.float32)
    rel4[:, :3] = np.concatenate(rels)
    return dirs, T, rels, offsets, rel4, np.array(q0s), np.array(qts)


def gpu_args(dirs, T, offsets, rel4, n_roi):
    return (dev(rel4), dev(offsets, torch.int64), dev(np.zeros(n_roi, np.int32), torch.int32), dev(dirs),
            dev(F_AL[None]), dev(T[None]))


def _antipodal_mesh(n_pairs, seed):
    g = np.random.default_rng(seed).standard_normal((n_pairs, 3))
    g = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    return np.concatenate([g, -g])


@pytest.mark.parametrize("mesh", ["icosphere3", "icosphere4", "pairs271", "pairs272"])
def test_amplitudes_and_score_match_fp64(nat, ctx, orc, mesh):
    """Evaluated directions per ROI: 321 (a last tile of 65, lane per
    direction), 1281 and 271 (last tiles of 1 and 15 directions, atom-parallel
    short-tile kernel), 272 (a last tile of 16, lane per direction)."""
    dirs = {"icosphere3": None, "icosphere4": synth.icosphere(4), "pairs271": _antipodal_mesh(271, 61),
            "pairs272": _antipodal_mesh(272, 62)}[mesh]
    dirs, T, rels, offsets, rel4, q0, qt = make_case(orc, 3, 4, dirs=dirs)
    rel, off, ph, d, f, t = gpu_args(dirs, T, offsets, rel4, 4)
    amp = nat.ar_sf_amplitudes(ctx, rel, off, dev(q0), ph, d, f).cpu().numpy()
    score, _ = nat.ar_sf_score_grad(ctx, rel, off, dev(q0), ph, d, f, t, grad=False)
    q0f = q0.astype(np.float32).astype(np.float64)     # the same quaternion both sides see
    s64 = nat.ar_sf_score_f64(ctx, rel, off, dev(q0f, torch.float64), ph, d, dev(F_AL[None], torch.float64),
                              dev(T[None].astype(np.float64), torch.float64)).cpu().numpy()
    for r in range(4):
        a_ref = orc.sf_amplitudes(rels[r], q0[r].astype(np.float32).astype(np.float64), dirs, F_AL)
        assert np.max(np.abs(amp[r] - a_ref)) <= 1e-5      # A is normalised by N_w: scale 1
        j_ref = orc.sf_score(rels[r], q0[r].astype(np.float32).astype(np.float64), dirs, F_AL, T.astype(np.float64))
        assert abs(float(score[r]) - j_ref) <= 1e-5 * j_ref
        assert abs(s64[r] - j_ref) <= 1e-9 * j_ref


@pytest.mark.parametrize("level", [3, 5])
def test_adjoint_matches_fp64_finite_differences(nat, ctx, orc, level):
    n = 3 if level == 3 else 2
    dirs, T, rels, offsets, rel4, q0, qt = make_case(orc, level, n, seed=level)
    rel, off, ph, d, f, t = gpu_args(dirs, T, offsets, rel4, n)
    qf = q0.astype(np.float32)
    _, g = nat.ar_sf_score_grad(ctx, rel, off, dev(qf), ph, d, f, t, grad=True)
    g = g.cpu().numpy().astype(np.float64)
    # FP64 central differences: oracle (CPU) at level 3, the GPU FP64 forward at level 5
    h = 1e-6
    for r in range(n):
        q64 = qf[r].astype(np.float64)
        if level == 3:
            fd = orc.sf_grad_fd(rels[r], q64, dirs, F_AL, T.astype(np.float64), h)
        else:
            qs = []
            for c in range(4):
                for sgn in (1, -1):
                    qq = q64.copy()
                    qq[c] += sgn * h
                    qs.append(qq)
            qs = np.array(qs)
            reps = 8
            o1 = np.array([offsets[r], offsets[r + 1]])
            relr = rel4[offsets[r]:offsets[r + 1]]
            offr = np.array([k * len(relr) for k in range(reps + 1)], np.int64)
            relrep = np.tile(relr, (reps, 1))
            js = nat.ar_sf_score_f64(ctx, dev(relrep), dev(offr, torch.int64), dev(qs, torch.float64),
                                     dev(np.zeros(reps, np.int32), torch.int32), d, dev(F_AL[None], torch.float64),
                                     dev(T[None].astype(np.float64), torch.float64)).cpu().numpy()
            fd = np.array([(js[2 * c] - js[2 * c + 1]) / (2 * h) for c in range(4)])
        err = np.linalg.norm(g[r] - fd) / np.linalg.norm(fd)
        assert err <= 1e-3, (level, r, g[r], fd, err)


def test_autograd_function_uses_the_adjoint(nat, ctx, orc):
    from paper_2009_00735_amd import refine
    dirs, T, rels, offsets, rel4, q0, qt = make_case(orc, 3, 3, seed=7)
    rel, off, ph, d, f, t = gpu_args(dirs, T, offsets, rel4, 3)
    q = dev(q0).requires_grad_(True)
    J = refine.sf_score(ctx, q, rel, off, ph, d, f, t)
    w = torch.tensor([1.0, 2.0, -0.5], device="cuda")
    (J * w).sum().backward()
    _, g = nat.ar_sf_score_grad(ctx, rel, off, dev(q0), ph, d, f, t, grad=True)
    assert torch.allclose(q.grad, g * w[:, None], rtol=1e-6, atol=0)


def test_degenerate_rois_have_zero_gradient(nat, ctx):
    dirs = synth.icosphere(2)
    T = np.full((1, 4, len(dirs)), 0.3, np.float32)
    rel4 = np.array([[0.3, -0.2, 0.1, 0.0]], np.float32)          # one atom, then an empty ROI
    offsets = np.array([0, 1, 1], np.int64)
    q = synth.random_orientations(2, 1).astype(np.float32)
    score, g = nat.ar_sf_score_grad(ctx, dev(rel4), dev(offsets, torch.int64), dev(q),
                                    dev(np.zeros(2, np.int32), torch.int32), dev(dirs), dev(F_AL[None]), dev(T))
    g = g.cpu().numpy()
    assert np.allclose(g, 0.0, atol=1e-4)
    s = score.cpu().numpy()
    assert abs(s[0] - 4 * len(dirs) * 0.7 ** 2) < 1e-2        # A = 1 for one atom
    assert abs(s[1] - 4 * len(dirs) * 0.3 ** 2) < 1e-3        # A = 0 for no atom


def test_refinement_recovers_orientation_and_tracks_oracle(nat, ctx, orc):
    dirs, T, rels, offsets, rel4, q0, qt = make_case(orc, 3, 6, sigma=0.03, seed=2, off_deg=3.0)
    rel, off, ph, d, f, t = gpu_args(dirs, T, offsets, rel4, 6)
    q = dev(q0)
    nat.ar_refine_orientations(ctx, rel, off, q, ph, d, f, t, steps=50, a0=0.01)
    qr = q.cpu().numpy().astype(np.float64)
    start = orc.disorientation_cubic(q0, qt)
    end = orc.disorientation_cubic(qr, qt)
    assert np.all(end < 0.5 * start) and np.median(end) < 0.5, (start, end)
    # the FP64 oracle trajectory of the same update rule lands on the same orientation
    qo, Jo = orc.sf_refine(rels[0], q0[0].astype(np.float32).astype(np.float64), dirs, F_AL, T.astype(np.float64),
                           steps=50, a0=0.01)
    assert orc.disorientation_cubic(qo, qr[0])[0] < 0.1


def test_unpaired_and_mixed_directions(nat, ctx, orc):
    """Directions without antipodes are evaluated alone; a mixed set (mesh
    plus random extra directions) matches the oracle and FD on both paths.
    The 10-direction set runs entirely in the short-tile kernel."""
    gen = np.random.default_rng(9)
    extra = gen.normal(size=(37, 3))
    extra = (extra / np.linalg.norm(extra, axis=1, keepdims=True)).astype(np.float32)
    for dirs in (extra, extra[:10], np.concatenate([synth.icosphere(2), extra])):
        dirs = np.ascontiguousarray(dirs)
        p = synth.lattice_in_ball("fcc", 0.405, synth.random_orientations(1, 11)[0], gen.random(3), np.zeros(3), 2.5)
        rel = orc.roi_gather(p.astype(np.float32), np.zeros(3, np.float32), 2.0)
        T = gen.random((4, len(dirs))).astype(np.float32) * 0.3
        rel4 = np.zeros((len(rel), 4), np.float32)
        rel4[:, :3] = rel
        q = synth.random_orientations(1, 12).astype(np.float32)
        args = (dev(rel4), dev(np.array([0, len(rel)]), torch.int64), dev(q), dev(np.zeros(1, np.int32), torch.int32),
                dev(dirs), dev(F_AL[None]))
        amp = nat.ar_sf_amplitudes(ctx, *args).cpu().numpy()[0]
        q64 = q[0].astype(np.float64)
        assert np.max(np.abs(amp - orc.sf_amplitudes(rel, q64, dirs, F_AL))) <= 1e-5
        score, g = nat.ar_sf_score_grad(ctx, *args, dev(T[None]))
        j = orc.sf_score(rel, q64, dirs, F_AL, T.astype(np.float64))
        assert abs(float(score[0]) - j) <= 1e-5 * j
        fd = orc.sf_grad_fd(rel, q64, dirs, F_AL, T.astype(np.float64))
        assert np.linalg.norm(g[0].cpu().numpy() - fd) <= 1e-3 * np.linalg.norm(fd)


@pytest.mark.parametrize("freqs", [(8.1892, 4.2767, 6.9838, 4.9383), (4.2767, 0.0, 8.1892, -6.9838),
                                   (4.9383, 8.1892, 4.2767), (0.0, 0.0, 0.0, 0.0), (-5.0,),
                                   (3.0, -7.0, 2.0, 5.0, 1.0, 4.0), (2.0, 3.0, 4.5, 1.0, 0.5, 6.0, 2.5, 7.5)])
def test_frequency_sets(nat, ctx, orc, freqs):
    """The kernel forms the phase of the largest |f| from the dot product and
    the others by the ratio f / f_max: any order, zero and negative
    frequencies, other counts (1, 3, 6 and the maximum 8), and all-zero
    frequencies (A = 1, no gradient) match the FP64 oracle; 81 evaluated directions run in the
    lane-per-direction kernel, 10 unpaired ones in the short-tile kernel."""
    f = np.array(freqs, np.float64)
    gen = np.random.default_rng(21)
    extra = gen.normal(size=(10, 3))
    extra = (extra / np.linalg.norm(extra, axis=1, keepdims=True)).astype(np.float32)
    for dirs in (synth.icosphere(2), extra):
        dirs = np.ascontiguousarray(dirs)
        p = synth.lattice_in_ball("fcc", 0.405, synth.random_orientations(1, 23)[0], gen.random(3), np.zeros(3), 2.5)
        rel = orc.roi_gather(p.astype(np.float32), np.zeros(3, np.float32), 2.0)
        T = gen.random((len(f), len(dirs))).astype(np.float32) * 0.3
        rel4 = np.zeros((len(rel), 4), np.float32)
        rel4[:, :3] = rel
        q = synth.random_orientations(1, 24).astype(np.float32)
        args = (dev(rel4), dev(np.array([0, len(rel)]), torch.int64), dev(q), dev(np.zeros(1, np.int32), torch.int32),
                dev(dirs), dev(f[None]))
        q64 = q[0].astype(np.float64)
        f32 = f.astype(np.float32).astype(np.float64)      # the frequencies both sides see
        amp = nat.ar_sf_amplitudes(ctx, *args).cpu().numpy()[0]
        assert np.max(np.abs(amp - orc.sf_amplitudes(rel, q64, dirs, f32))) <= 1e-5
        score, g = nat.ar_sf_score_grad(ctx, *args, dev(T[None]))
        j = orc.sf_score(rel, q64, dirs, f32, T.astype(np.float64))
        assert abs(float(score[0]) - j) <= 1e-5 * j
        g = g[0].cpu().numpy()
        if not f.any():
            assert np.allclose(amp, 1.0, rtol=0, atol=1e-6) and np.allclose(g, 0.0, rtol=0, atol=1e-6)
        else:
            fd = orc.sf_grad_fd(rel, q64, dirs, f32, T.astype(np.float64))
            assert np.linalg.norm(g - fd) <= 1e-3 * np.linalg.norm(fd)


def test_refinement_zero_and_one_step(nat, ctx, orc):
    """The update rule on its first steps, against host arithmetic on the
    score and gradient entry point.  steps = 0: one score-only evaluation,
    quaternions unchanged, score J(q0).  steps = 1: one adjoint evaluation at
    q0 and a score-only one at q1 = normalise(q0 - a0 g/|g|); q1 is kept iff
    J(q1) <= J(q0) - 1e-4 a0 |g| (a small step that is kept, a large one that
    is refused)."""
    dirs, T, rels, offsets, rel4, q0, qt = make_case(orc, 3, 3, seed=13)
    rel, off, ph, d, f, t = gpu_args(dirs, T, offsets, rel4, 3)
    q0 = q0.astype(np.float32)
    J0, g0 = nat.ar_sf_score_grad(ctx, rel, off, dev(q0), ph, d, f, t, grad=True)
    J0s, _ = nat.ar_sf_score_grad(ctx, rel, off, dev(q0), ph, d, f, t, grad=False)
    J0, J0s, g0 = J0.cpu().numpy(), J0s.cpu().numpy(), g0.cpu().numpy().astype(np.float64)
    assert np.allclose(J0s, J0, rtol=1e-6, atol=0)

    q = dev(q0)
    score = nat.ar_refine_orientations(ctx, rel, off, q, ph, d, f, t, steps=0, a0=0.01).cpu().numpy()
    assert np.array_equal(q.cpu().numpy(), q0)
    assert np.array_equal(score, J0s)                     # the same score-only kernels

    for a0, kept in ((0.002, True), (1.5, False)):
        gn = np.linalg.norm(g0, axis=1, keepdims=True)
        q1 = q0 - a0 * g0 / gn
        q1 /= np.linalg.norm(q1, axis=1, keepdims=True)
        J1, _ = nat.ar_sf_score_grad(ctx, rel, off, dev(q1), ph, d, f, t, grad=False)
        J1 = J1.cpu().numpy()
        accept = J1 <= J0 - 1e-4 * a0 * gn[:, 0]
        assert np.all(accept == kept), (a0, J0, J1)
        q = dev(q0)
        score = nat.ar_refine_orientations(ctx, rel, off, q, ph, d, f, t, steps=1, a0=a0).cpu().numpy()
        qr = q.cpu().numpy()
        if kept:
            assert np.allclose(qr, q1, rtol=0, atol=2e-6), (qr, q1)
            assert np.allclose(score, J1, rtol=1e-5, atol=0)
        else:
            assert np.array_equal(qr, q0)
            assert np.array_equal(score, J0)
