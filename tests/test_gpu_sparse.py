"""Sparse Eq. S1 indexing on the GPU against the FP64 oracle.

Look-up table: strongest-entry lists and rotated-node tables bit-exact
(including exact ties of the normalised values, an all-zero window, a phase
with no orientations, odd phase boundaries).  Indexing: GPU top-1 equals the
oracle's top-1 or is a tie within the indexing tolerance, and every returned
FP32 score is within 1e-5 relative (+1e-6) of the FP64 score of the same
(ROI, orientation); sizes span several orientation chunks, a ragged ROI
group and all three screens (8-bit codes with 8 ROIs per LDS read, FP16 with
2 and with 1).  The bench configuration
(2000 ROIs, 20000 orientations, 1000 strong entries, 10242 nodes, 4 windows)
is checked on sampled ROIs and orientations."""
import numpy as np
import pytest
import torch

from paper_2009_00735_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    from paper_2009_00735_amd import native
    return native


@pytest.fixture(scope="module")
def ctx(nat):
    return nat.Context(0)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def phases_of(counts):
    return np.repeat(np.arange(len(counts), dtype=np.int32), counts)


def build(nat, ctx, ref, dirs, q, counts, n_hat):
    lut = nat.SparseLUT(ctx, dev(ref), dev(dirs), dev(q, torch.float64), counts, n_hat)
    si, sv, nodes = (t.cpu().numpy() for t in lut.export())
    return lut, si, sv, nodes


def check_lut(orc, ref, dirs, q, counts, n_hat, si, sv, nodes, rows=None):
    osi, osv = orc.sparse_strong(ref, n_hat)
    assert np.array_equal(si, osi)
    assert np.array_equal(sv, osv.astype(np.float32))      # (float) of the same FP64 quotient
    ph = phases_of(counts)
    rows = np.arange(len(q)) if rows is None else np.asarray(rows)
    olut = orc.sparse_lut(q[rows], ph[rows], osi, dirs)
    assert np.array_equal(nodes[rows], olut)
    return osi, osv, olut


def check_index(orc, S, osi, osv, ph, olut, gidx, gsc, k):
    """GPU top-k vs the oracle's over all orientations (olut covers all)."""
    Sh = orc.normalise(S)
    oi, osc = orc.sparse_index_topk(Sh, osi, osv, ph, olut, k)
    ties = 0
    for r in range(len(S)):
        d64 = orc.sparse_pairs(Sh, osi, osv, ph[gidx[r]], olut[gidx[r]], np.full(k, r))
        assert np.all(np.abs(gsc[r] - d64) <= 1e-5 * d64 + 1e-6), (r, gsc[r], d64)
        assert np.all(np.diff(gsc[r]) >= 0)
        if gidx[r, 0] != oi[r, 0]:
            assert d64[0] - osc[r, 0] <= 1e-5 * osc[r, 0] + 1e-6, (r, gidx[r, 0], oi[r, 0], d64[0], osc[r, 0])
            ties += 1
    return ties


def test_lut_bit_exact_small(nat, ctx, orc):
    dirs = synth.icosphere(3)
    gen = np.random.default_rng(31)
    ref = (gen.integers(0, 17, (2, 4, len(dirs))) / 16.0).astype(np.float32)   # many exact ties
    ref[1, 2] = 0.0                                                            # all-zero window
    counts = [1025, 1151]
    q = synth.random_orientations(sum(counts), 32)
    lut, si, sv, nodes = build(nat, ctx, ref, dirs, q, counts, 300)
    check_lut(orc, ref, dirs, q, counts, 300, si, sv, nodes)


@pytest.mark.parametrize("counts,n_hat", [([5, 0, 3], 4 * 162), ([1], 1), ([2, 7], 37)])
def test_lut_edge_cases(nat, ctx, orc, counts, n_hat):
    """Every entry kept (n_hat = n_win * n_dir), a phase without
    orientations, a single orientation with one entry."""
    dirs = synth.icosphere(2)
    gen = np.random.default_rng(33 + n_hat)
    ref = gen.random((len(counts), 4, len(dirs))).astype(np.float32)
    ref[0, 1] = 0.0
    q = synth.random_orientations(sum(counts), 34)
    lut, si, sv, nodes = build(nat, ctx, ref, dirs, q, counts, n_hat)
    check_lut(orc, ref, dirs, q, counts, n_hat, si, sv, nodes)


def test_lut_argument_checks(nat, ctx):
    dirs = synth.icosphere(1)
    ref = np.ones((2, 2, len(dirs)), np.float32)
    q = synth.random_orientations(4, 35)
    for counts, n_hat in [([2, 2], 0), ([2, 2], 2 * len(dirs) + 1), ([3, -1], 5), ([0, 0], 5)]:
        with pytest.raises((nat.AraulloError, ValueError)):
            nat.SparseLUT(ctx, dev(ref), dev(dirs), dev(q[:max(0, sum(counts))], torch.float64), counts, n_hat)


def _qmul(a, b):
    return np.stack([a[:, 0] * b[:, 0] - a[:, 1] * b[:, 1] - a[:, 2] * b[:, 2] - a[:, 3] * b[:, 3],
                     a[:, 0] * b[:, 1] + a[:, 1] * b[:, 0] + a[:, 2] * b[:, 3] - a[:, 3] * b[:, 2],
                     a[:, 0] * b[:, 2] - a[:, 1] * b[:, 3] + a[:, 2] * b[:, 0] + a[:, 3] * b[:, 1],
                     a[:, 0] * b[:, 3] + a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1] + a[:, 3] * b[:, 0]], axis=1)


def _planted(dirs, counts, q, n_roi, seed):
    """Signature-like ROI images: ROI r is its phase's crystal seen in the
    orientation of a seeded library entry truth[r] turned by 1.5 deg about a
    random axis, with a per-window gain and 5 % multiplicative noise.  ROI 1
    has an all-zero window and the last ROI is entirely zero."""
    gen = np.random.default_rng(seed)
    ph = phases_of(counts)
    truth = gen.integers(0, len(q), n_roi)
    axis = gen.standard_normal((n_roi, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    h = np.radians(1.5) / 2
    jitter = np.concatenate([np.full((n_roi, 1), np.cos(h)), np.sin(h) * axis], axis=1)
    qt = _qmul(q[truth], jitter)
    gain = gen.uniform(0.5, 2.0, (n_roi, 4))
    S = synth.bump_images(dirs, qt, ph[truth], 4, gain=gain, noise=0.05, seed=seed)
    S[1, 2] = 0.0
    S[-1] = 0.0
    return S, truth, qt


@pytest.fixture(scope="module")
def chunks_world(nat, ctx, orc):
    """10242 nodes (the 8-bit screen, eight ROIs per workgroup), 2 phases
    with 2500 + 1701 orientations (chunks of 2048, an odd phase start), 300
    strong entries, 45 ROIs (a ragged last group of five)."""
    dirs = synth.icosphere(5)
    counts = [2500, 1701]
    ref = synth.bump_images(dirs, np.tile([1.0, 0, 0, 0], (2, 1)), [0, 1], 4)
    q = synth.library_orientations(sum(counts), 7)
    lut, si, sv, nodes = build(nat, ctx, ref, dirs, q, counts, 300)
    assert lut.screen == 8
    osi, osv, olut = check_lut(orc, ref, dirs, q, counts, 300, si, sv, nodes)
    S, truth, qt = _planted(dirs, counts, q, 45, 41)
    return dict(lut=lut, osi=osi, osv=osv, olut=olut, S=S, ph=phases_of(counts), q=q, qt=qt)


@pytest.mark.parametrize("k", [16, 1, 32])
def test_index_parity_several_chunks(nat, ctx, orc, chunks_world, k):
    w = chunks_world
    gidx, gsc = nat.index_orientations_sparse(ctx, dev(w["S"]), w["lut"], k)
    gidx, gsc = gidx.cpu().numpy(), gsc.cpu().numpy()
    ties = check_index(orc, w["S"], w["osi"], w["osv"], w["ph"], w["olut"], gidx, gsc, k)
    dis = orc.disorientation_cubic(w["q"][gidx[:-1, 0]], w["qt"][:-1])
    print(f"\nk={k}: ties with the oracle's top-1 {ties}/45; top-1 disorientation median {np.median(dis):.2f} deg",
          flush=True)


@pytest.mark.parametrize("n_hat", [150, 4 * 642])
def test_index_parity_empty_window_and_all_entries(nat, ctx, orc, n_hat):
    """642 nodes, 2 phases (700 + 650 orientations); phase 1's reference has
    an all-zero window, which gets no strong entry at N^ = 150 (an empty
    screen segment) and 642 zero-valued entries when all 4 x 642 entries are
    kept (segments of 642 rows, padded to 644)."""
    dirs = synth.icosphere(3)
    counts = [700, 650]
    ref = synth.bump_images(dirs, np.tile([1.0, 0, 0, 0], (2, 1)), [0, 1], 4)
    ref[1, 2] = 0.0
    q = synth.library_orientations(sum(counts), 9)
    lut, si, sv, nodes = build(nat, ctx, ref, dirs, q, counts, n_hat)
    assert lut.screen == 8
    osi, osv, olut = check_lut(orc, ref, dirs, q, counts, n_hat, si, sv, nodes)
    if n_hat == 150:
        assert not np.any(osi[1] // len(dirs) == 2)
    S, truth, qt = _planted(dirs, counts, q, 20, 47)
    gidx, gsc = nat.index_orientations_sparse(ctx, dev(S), lut, 16)
    check_index(orc, S, osi, osv, phases_of(counts), olut, gidx.cpu().numpy(), gsc.cpu().numpy(), 16)


@pytest.mark.parametrize("mesh", ["random30000", "icosphere6"])
def test_index_parity_wide_meshes(nat, ctx, orc, mesh):
    """Meshes too large for the 8-bit screen: 30000 random unit directions
    (FP16, two ROIs per workgroup) and the paper's 40962-node mesh (FP16, one
    ROI per workgroup)."""
    if mesh == "icosphere6":
        dirs = synth.icosphere(6)
    else:
        g = np.random.default_rng(36).standard_normal((30000, 3))
        dirs = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    counts = [300, 301]
    ref = synth.bump_images(dirs, np.tile([1.0, 0, 0, 0], (2, 1)), [0, 1], 4)
    q = synth.library_orientations(sum(counts), 8)
    lut, si, sv, nodes = build(nat, ctx, ref, dirs, q, counts, 200)
    assert lut.screen == (2 if mesh == "random30000" else 1)
    osi, osv, olut = check_lut(orc, ref, dirs, q, counts, 200, si, sv, nodes)
    S, truth, qt = _planted(dirs, counts, q, 9, 42)
    gidx, gsc = nat.index_orientations_sparse(ctx, dev(S), lut, 16)
    check_index(orc, S, osi, osv, phases_of(counts), olut, gidx.cpu().numpy(), gsc.cpu().numpy(), 16)


def test_index_bench_configuration_sampled(nat, ctx, orc):
    """2000 ROIs x 20000 orientations of one phase, 1000 strong entries,
    10242 nodes, 4 windows (the benchmark's launch configuration).  On 6
    sampled ROIs: every returned score equals the FP64 score of the same
    orientation (the oracle builds those look-up rows itself), and the GPU
    top-1 is no worse than the FP64 score of 600 sampled orientations plus
    the seeded one; on 2 of them the GPU top-1 equals the oracle's full FP64
    top-1 over all 20000 orientations or is a tie; look-up rows bit-exact on
    sampled orientations."""
    dirs = synth.icosphere(5)
    n_lib, n_roi, n_hat = 20000, 2000, 1000
    ref = synth.bump_images(dirs, np.array([[1.0, 0, 0, 0]]), [0], 4)
    q = synth.library_orientations(n_lib, 2)
    lut, si, sv, nodes = build(nat, ctx, ref, dirs, q, [n_lib], n_hat)
    rows = np.concatenate([[0, 1, 2047, 2048, n_lib - 1], np.random.default_rng(43).choice(n_lib, 11, replace=False)])
    osi, osv, _ = check_lut(orc, ref, dirs, q, [n_lib], n_hat, si, sv, nodes, rows=rows)
    S, truth, qt = _planted(dirs, [n_lib], q, n_roi, 44)
    gidx, gsc = nat.index_orientations_sparse(ctx, dev(S), lut, 16)
    gidx, gsc = gidx.cpu().numpy(), gsc.cpu().numpy()
    sel = np.random.default_rng(45).choice(n_roi - 1, 6, replace=False)
    Sh = orc.normalise(S[sel])
    ph = np.zeros(n_lib, np.int32)
    probe = np.random.default_rng(46).choice(n_lib, 600, replace=False)
    for a, r in enumerate(sel):
        cols = np.concatenate([gidx[r], probe, [truth[r]]])
        olut = orc.sparse_lut(q[cols], ph[cols], osi, dirs)
        d64 = orc.sparse_pairs(Sh, osi, osv, ph[cols], olut, np.full(len(cols), a))
        assert np.all(np.abs(gsc[r] - d64[:16]) <= 1e-5 * d64[:16] + 1e-6), (r, gsc[r], d64[:16])
        assert d64[0] <= d64[16:].min() * (1 + 1e-5) + 1e-6, (r, d64[0], d64[16:].min())
    # two ROIs against the oracle's full sparse top-1 over all 20000
    # orientations (the oracle builds every look-up row itself)
    full = orc.sparse_lut(q, ph, osi, dirs)
    oidx, osc = orc.sparse_index_topk(Sh[:2], osi, osv, ph, full, 1)
    for a in range(2):
        r = sel[a]
        if gidx[r, 0] != oidx[a, 0]:
            d = orc.sparse_pairs(Sh, osi, osv, ph[[gidx[r, 0]]], full[[gidx[r, 0]]], [a])[0]
            assert d - osc[a, 0] <= 1e-5 * osc[a, 0] + 1e-6, (r, gidx[r, 0], oidx[a, 0], d, osc[a, 0])
    # accuracy against the seeded orientation (cubic symmetry)
    dis = orc.disorientation_cubic(q[gidx[:-1, 0]], qt[:-1])
    print(f"\nbench configuration: top-1 disorientation median {np.median(dis):.2f} deg, "
          f"p95 {np.percentile(dis, 95):.2f} deg", flush=True)
    assert np.median(dis) < 5.0
