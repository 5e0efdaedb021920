"""GPU <-> oracle parity of the indexing stage (normalise + BF16 MFMA
correlation + top-k + FP32 rescore), rotated references and disorientation.

Bar (top-1): the GPU's rescored top-1 equals the FP64 oracle's top-1, or is a
tie: Delta_orc(gpu) - Delta_orc(orc) <= 1e-5 Delta_orc(orc) + 1e-6.
FP32 Delta of every returned pair within 1e-5 relative (+1e-6) of FP64."""
import math

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


def check_topk(orc, S, L, gidx, gsc, k, report):
    """S, L raw float32 images; gidx/gsc GPU outputs (numpy)."""
    Sh = orc.normalise(S)
    Lh = orc.normalise(L)
    oidx, osc = orc.index_topk(Sh, Lh, k)
    n = len(S)
    ties = 0
    for r in range(n):
        if gidx[r, 0] != oidx[r, 0]:
            d = orc.ssd_pairs(Sh, Lh, [r], [gidx[r, 0]])[0]
            assert d - osc[r, 0] <= 1e-5 * osc[r, 0] + 1e-6, (r, gidx[r, 0], oidx[r, 0], d, osc[r, 0])
            ties += 1
        # FP32 Delta of every returned pair against FP64
        d64 = orc.ssd_pairs(Sh, Lh, np.full(k, r), gidx[r])
        assert np.all(np.abs(gsc[r] - d64) <= 1e-5 * d64 + 1e-6), (r, gsc[r], d64)
        assert np.all(np.diff(gsc[r]) >= 0)
    report["ties"] = ties
    report["recall_k"] = float(np.mean([len(set(gidx[r]) & set(oidx[r])) / k for r in range(n)]))
    return oidx, osc


def reference_library(orc, R, nbins, dirs, windows, n_lib, cfg):
    pts, offs = synth.reference_rois(0, 16, R=R, cfg=cfg)
    ref, _ = orc.signatures(pts, offs, R, dirs, nbins, windows)
    R0 = ref.mean(axis=0)
    q = synth.library_orientations(n_lib, cfg)
    L = orc.library_images(R0[None], np.zeros(n_lib, np.int32), q, dirs).astype(np.float32)
    return R0, q, L


def test_index_single_roi_rotated_library(nat, ctx, orc):
    """Single ROI: 1000 rotated fcc references (level-3 mesh, 256 bins); the
    single-ROI specimen's ROI plus 36 ROIs of other random crystals (ragged M, N, K)."""
    s = synth.single_roi()
    w = orc.windows_for(s.radius, s.nbins, s.spacings)
    R0, q, L = reference_library(orc, s.radius, s.nbins, s.directions, w, 1000, 1)
    cents = np.zeros((36, 3), np.float32)
    imgs = [orc.signatures(s.positions, s.centres, s.radius, s.directions, s.nbins, w)[0]]
    for i in range(36):
        qt = synth.random_orientations(1, 500 + i)[0]
        p = synth.lattice_in_ball("fcc", 0.405, qt, np.random.default_rng(i).random(3), np.zeros(3), 1.5)
        imgs.append(orc.signatures(p.astype(np.float32), cents[i:i + 1], s.radius, s.directions, s.nbins, w)[0])
    S = np.concatenate(imgs).astype(np.float32)
    lib = nat.Library(ctx, dev(L))
    gidx, gsc = nat.index_orientations(ctx, dev(S), lib, 16)
    rep = {}
    check_topk(orc, S, L, gidx.cpu().numpy(), gsc.cpu().numpy(), 16, rep)
    print("single-ROI indexing:", rep)


def test_index_self(nat, ctx, orc):
    S, L, truth = synth.planted_images(10, 700, 4, 333, seed=3)
    lib = nat.Library(ctx, dev(L))
    rows = np.array([0, 5, 127, 128, 129, 699])
    gidx, gsc = nat.index_orientations(ctx, dev(L[rows]), lib, 4)
    assert np.array_equal(gidx[:, 0].cpu().numpy(), rows)
    assert np.all(gsc[:, 0].cpu().numpy() == 0.0)


@pytest.mark.parametrize("k,cand", [(1, 16), (16, 16), (5, 32), (32, 32)])
def test_index_planted_small(nat, ctx, orc, k, cand):
    S, L, truth = synth.planted_images(300, 1000, 4, 257, seed=k + cand)
    lib = nat.Library(ctx, dev(L))
    gidx, gsc, gcand = nat.index_orientations_ex(ctx, dev(S), lib, k, cand)
    gidx = gidx.cpu().numpy()
    assert np.array_equal(gidx[:, 0], truth)
    rep = {}
    check_topk(orc, S, L, gidx, gsc.cpu().numpy(), k, rep)
    gcand = gcand.cpu().numpy()
    assert np.all([truth[r] in gcand[r] for r in range(len(S))])


def test_index_planted_bench_shape(nat, ctx, orc):
    """The benchmark's indexing shape: 2000 ROIs x 20000 references x
    (4 x 10242) nodes; sampled ROIs against the FP64 oracle."""
    S, L, truth = synth.planted_images(2000, 20000, 4, 10242, seed=11)
    lib = nat.Library(ctx, dev(L))
    Sd = dev(S)
    gidx, gsc = nat.index_orientations(ctx, Sd, lib, 16)
    torch.cuda.synchronize()
    gidx = gidx.cpu().numpy()
    gsc = gsc.cpu().numpy()
    assert np.array_equal(gidx[:, 0], truth)
    sel = np.random.default_rng(0).choice(2000, 10, replace=False)
    rep = {}
    check_topk(orc, S[sel], L, gidx[sel], gsc[sel], 16, rep)
    print("bench-shape indexing:", rep)


def test_rotate_reference_matches_oracle(nat, ctx, orc):
    dirs = synth.icosphere(3)
    gen = np.random.default_rng(4)
    ref = gen.random((2, 4, len(dirs))).astype(np.float32)
    q = synth.library_orientations(300, 9)
    ph = (np.arange(300) % 2).astype(np.int32)
    got = nat.ar_rotate_reference(ctx, dev(ref), dev(dirs), dev(q, torch.float64), dev(ph, torch.int32)).cpu().numpy()
    lut = orc.rotated_nodes(q, dirs)
    expect = np.stack([ref[ph[l]][:, lut[l]] for l in range(300)])
    assert np.array_equal(got, expect)


def _mesh(kind):
    gen = np.random.default_rng(12)
    if kind == "icosphere0":                      # 12 nodes: one cube-map cell per face, every node listed
        return synth.icosphere(0)
    if kind == "clustered":                       # 2000 nodes in a 3 deg cap + 100 elsewhere: lists past the
        c = gen.standard_normal((2000, 3)) * np.radians(1.5)   # cap of 256 fall back to the full scan
        c[:, 2] = 1.0
        o = gen.standard_normal((100, 3))
        d = np.concatenate([c, o])
        return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    if kind == "non_unit":                        # nodes off the unit sphere: the full scan is used
        d = synth.icosphere(2).astype(np.float64)
        return (d * gen.uniform(0.5, 1.5, (len(d), 1))).astype(np.float32)
    d = synth.icosphere(3)                        # duplicated nodes: exact ties go to the lower index
    return np.concatenate([d, d[::7]]).astype(np.float32)


@pytest.mark.parametrize("kind", ["icosphere0", "clustered", "duplicates", "non_unit"])
def test_rotate_reference_nearest_node_edge_meshes(nat, ctx, orc, kind):
    """The reference value of node u is u itself, so the output is the chosen
    node: it must equal the oracle's exhaustive FP32-scan / FP64-re-rank
    choice on meshes that stress the cube-map candidate lists."""
    dirs = _mesh(kind)
    n = len(dirs)
    ref = np.tile(np.arange(n, dtype=np.float32), (1, 1, 1))
    q = synth.library_orientations(200, 13)
    q[0] = [1.0, 0.0, 0.0, 0.0]                   # identity and 180 deg about z: rotated nodes land on nodes
    q[1] = [0.0, 0.0, 0.0, 1.0]
    ph = np.zeros(200, np.int32)
    got = nat.ar_rotate_reference(ctx, dev(ref), dev(dirs), dev(q, torch.float64), dev(ph, torch.int32)).cpu().numpy()
    lut = orc.rotated_nodes(q, dirs)
    assert np.array_equal(got[:, 0, :].astype(np.int64), lut.astype(np.int64))


def test_disorientation_matches_oracle(nat, orc):
    gen = np.random.default_rng(5)
    qa = synth.shoemake(5000, gen)
    qb = synth.shoemake(5000, gen)
    qa[:10] = qb[:10]
    qb[10] = -qa[10]
    got = nat.ar_disorientation_cubic(dev(qa, torch.float64), dev(qb, torch.float64)).cpu().numpy()
    ref = orc.disorientation_cubic(qa, qb)
    assert np.max(np.abs(got - ref)) < 1e-6
    assert np.all(got[:11] < 1e-5)


def test_planted_orientation_end_to_end(nat, ctx, orc):
    """GPU pipeline at the benchmark mesh (level 5, 1024 bins, R = 2 nm):
    reference crystal -> GPU signatures -> GPU rotated library (300 random
    orientations + the true one) -> GPU signatures of noisy ROIs (sigma 0.05,
    half the atoms) -> GPU indexing: the true orientation ranks first."""
    R, nb = 2.0, 1024
    dirs = synth.icosphere(5)
    w = nat.windows_for(R, nb, synth.window_spacings())
    pts, offs = synth.reference_rois(0, 16, R=R, cfg=4)
    ref = nat.araullo_signatures(ctx, dev(pts), dev(offs), R, dev(dirs), nb, w, counts=False).mean(0, keepdim=True)
    qlib = synth.library_orientations(300, 2)
    for seed in range(3):
        qt = synth.random_orientations(1, 100 + seed)[0]
        q = np.concatenate([qlib, qt[None]])
        L = nat.ar_rotate_reference(ctx, ref.contiguous(), dev(dirs), dev(q, torch.float64),
                                    torch.zeros(len(q), dtype=torch.int32, device="cuda"))
        gen = np.random.default_rng(seed)
        p = synth.lattice_in_ball("fcc", 0.405, qt, gen.random(3), np.zeros(3), R + 0.5)
        keep = synth.delete_exact(len(p), 0.5, gen)
        p = (p[keep] + gen.normal(0, 0.05, (len(keep), 3))).astype(np.float32)
        img = nat.araullo_signatures(ctx, dev(p), dev(np.zeros((1, 3))), R, dev(dirs), nb, w, counts=False)
        lib = nat.Library(ctx, L)
        gidx, _ = nat.index_orientations(ctx, img, lib, 16)
        assert int(gidx[0, 0]) == len(q) - 1


def test_index_invalid_arguments(nat, ctx):
    S, L, truth = synth.planted_images(4, 200, 2, 64, seed=1)
    lib = nat.Library(ctx, dev(L))
    with pytest.raises(nat.AraulloError):
        nat.index_orientations(ctx, dev(S), lib, 0)
    with pytest.raises(nat.AraulloError):
        nat.index_orientations(ctx, dev(S), lib, 65)
    with pytest.raises(nat.AraulloError):
        nat.index_orientations_ex(ctx, dev(S), lib, 4, 20)
    with pytest.raises(nat.AraulloError):
        nat.index_orientations_ex(ctx, dev(S), lib, 33, 32)
    with pytest.raises(nat.AraulloError, match="without orientations"):
        lib.lookup(torch.zeros(3, dtype=torch.int32, device="cuda"))


def test_index_unaligned_image_arrays(nat, ctx):
    """Image arrays that start 4 bytes off an 8-byte boundary (a view one
    float into its buffer) take the single-value path of the normalise-and-
    cast kernel; the top-k and scores equal those from aligned arrays."""
    S, L, truth = synth.planted_images(50, 300, 4, 64, seed=5)   # even n_dir: the paired path when aligned

    def shifted(a):
        t = dev(a)
        buf = torch.empty(t.numel() + 1, device="cuda")
        v = buf[1:].view(t.shape)
        v.copy_(t)
        assert v.data_ptr() % 8 == 4
        return v

    lib = nat.Library(ctx, dev(L))
    lib_u = nat.Library(ctx, shifted(L))
    a_idx, a_sc = nat.index_orientations(ctx, dev(S), lib, 16)
    for images, library in ((shifted(S), lib), (dev(S), lib_u), (shifted(S), lib_u)):
        b_idx, b_sc = nat.index_orientations(ctx, images, library, 16)
        assert torch.equal(a_idx, b_idx) and torch.equal(a_sc, b_sc)
    assert np.array_equal(a_idx[:, 0].cpu().numpy(), truth)


def test_library_rejects_rows_beyond_the_panel_offsets(nat, ctx):
    """The correlation addresses 256-row panels of BF16 rows with 32-bit
    byte offsets, so n_win * n_dir above 4194240 is refused before any device
    memory is touched (the image pointer is a stand-in and never read)."""
    import ctypes
    out = ctypes.c_void_p()
    s = torch.cuda.current_stream().cuda_stream
    fake = ctypes.c_void_p(256)
    for n_win, n_dir in ((4, 1048561), (1, 4194241), (64, 65536)):   # 4 x 1048560 would be the largest accepted
        st = nat._L.ar_library_create(ctx.handle, fake, 1, n_win, n_dir, s, ctypes.byref(out))
        assert st == -1 and not out.value, (n_win, n_dir, st)
        assert b"too large" in nat._L.ar_last_error(ctx.handle)


@pytest.mark.parametrize("tile", [(4, 2, 2, 32), (4, 2, 4, 32), (4, 4, 2, 32), (4, 4, 4, 32), (8, 2, 2, 32),
                                  (8, 4, 2, 32), (0, 0, 0, 0)])
def test_every_correlation_tile_gives_identical_results(nat, ctx, tile):
    """Each score accumulates K in the same order whatever the workgroup
    tile, so candidates, indices and FP32 scores are bit-identical, with 16,
    32 and 64 candidates; (0, 0, 0, 0) is the default choice per candidate
    count."""
    S, L, truth = synth.planted_images(333, 1500, 4, 300, seed=21)
    lib = nat.Library(ctx, dev(L))
    try:
        for cand in (16, 32, 64):
            nat.ar_index_set_tile(ctx, 4, 2, 2, 32)
            ref = nat.index_orientations_ex(ctx, dev(S), lib, cand, cand)
            nat.ar_index_set_tile(ctx, *tile)
            got = nat.index_orientations_ex(ctx, dev(S), lib, cand, cand)
            for a, b in zip(ref, got):
                assert torch.equal(a, b)
            assert np.array_equal(got[0][:, 0].cpu().numpy(), truth)
    finally:
        nat.ar_index_set_tile(ctx, 0, 0, 0, 0)


@pytest.mark.parametrize("n_win,n_dir", [(1, 40), (2, 32), (1, 64)])
def test_short_k_every_tile_against_oracle(nat, ctx, orc, n_win, n_dir):
    """K padded to 64 or 128 (two to four K steps, fewer than the LDS ring
    holds): every tile, with 16, 32 and 64 candidates, returns the oracle's
    top-k (or ties) and bit-identical results across tiles."""
    S, L, truth = synth.planted_images(40, 700, n_win, n_dir, seed=n_dir + n_win)
    lib = nat.Library(ctx, dev(L))
    tiles = [(4, 2, 2, 32), (4, 2, 4, 32), (4, 4, 2, 32), (4, 4, 4, 32), (8, 2, 2, 32), (8, 4, 2, 32)]
    try:
        for cand in (16, 32, 64):
            ref = None
            for tile in tiles:
                nat.ar_index_set_tile(ctx, *tile)
                got = nat.index_orientations_ex(ctx, dev(S), lib, cand, cand)
                if ref is None:
                    ref = got
                    rep = {}
                    check_topk(orc, S, L, got[0].cpu().numpy(), got[1].cpu().numpy(), cand, rep)
                else:
                    for a, b in zip(ref, got):
                        assert torch.equal(a, b), (cand, tile)
    finally:
        nat.ar_index_set_tile(ctx, 0, 0, 0, 0)


def test_index_set_tile_rejects_unsupported(nat, ctx):
    for tile in [(8, 4, 4, 32), (4, 2, 2, 16), (2, 2, 2, 32), (0, 0, 0, 32)]:
        with pytest.raises(nat.AraulloError):
            nat.ar_index_set_tile(ctx, *tile)


@pytest.mark.parametrize("k", [64, 40, 33, 17])
def test_index_long_lists_planted_ranking(nat, ctx, orc, k):
    """k above 32 (the paper keeps many near-best solutions per ROI, Sec.
    3.2): 40 ROIs, each with 64 planted library rows at increasing distance
    (ratio 1.08 between neighbours) among 5003 rows, 4 x 642 nodes.  The
    oracle's FP64 top-64 is the planted ranking (checked first); the GPU
    returns exactly the planted first k, its 64 BF16-stage candidates are the
    planted set, and every score is within 1e-5 of FP64."""
    S, L, ranked = synth.ranked_images(40, 5003, 4, 642, 64, seed=5)
    oidx, _ = orc.index_topk(orc.normalise(S), orc.normalise(L), 64)
    assert np.array_equal(oidx, ranked)
    lib = nat.Library(ctx, dev(L))
    gidx, gsc = nat.index_orientations(ctx, dev(S), lib, k)
    gidx = gidx.cpu().numpy()
    assert np.array_equal(gidx, ranked[:, :k])
    check_topk(orc, S, L, gidx, gsc.cpu().numpy(), k, {})
    _, _, gcand = nat.index_orientations_ex(ctx, dev(S), lib, k, 64)
    gcand = gcand.cpu().numpy()
    assert all(set(gcand[r]) == set(ranked[r]) for r in range(len(S)))


def test_index_k64_beyond_the_library(nat, ctx, orc):
    """k = 64 against a 40-entry library: the 40 entries in the oracle's
    order, then index -1 and Delta +inf."""
    S, L, truth = synth.planted_images(7, 40, 4, 300, seed=9)
    lib = nat.Library(ctx, dev(L))
    gidx, gsc = nat.index_orientations(ctx, dev(S), lib, 64)
    gidx, gsc = gidx.cpu().numpy(), gsc.cpu().numpy()
    oidx, _ = orc.index_topk(orc.normalise(S), orc.normalise(L), 40)
    assert np.array_equal(gidx[:, :40], oidx)
    assert np.all(gidx[:, 40:] == -1) and np.all(np.isinf(gsc[:, 40:]))
    check_topk(orc, S, L, gidx[:, :40], gsc[:, :40], 40, {})


def test_library_with_orientations_reports_them(nat, ctx, orc):
    """A library prepared with orientations and phases maps indexing results
    back to them; -1 gives a NaN quaternion and phase -1."""
    s = synth.single_roi()
    w = orc.windows_for(s.radius, s.nbins, s.spacings)
    R0, q, L = reference_library(orc, s.radius, s.nbins, s.directions, w, 300, 1)
    ph = (np.arange(300) % 2).astype(np.int32)
    lib = nat.Library(ctx, dev(L), dev(q, torch.float64), dev(ph, torch.int32))
    img, _ = orc.signatures(s.positions, s.centres, s.radius, s.directions, s.nbins, w)
    gidx, _ = nat.index_orientations(ctx, dev(img.astype(np.float32)), lib, 64)
    plain = nat.Library(ctx, dev(L))
    pidx, _ = nat.index_orientations(ctx, dev(img.astype(np.float32)), plain, 64)
    assert torch.equal(gidx, pidx)
    probe = torch.cat([gidx.reshape(-1), torch.tensor([-1, 300, 299], dtype=torch.int32, device="cuda")])
    gq, gph = lib.lookup(probe)
    gq, gph, probe = gq.cpu().numpy(), gph.cpu().numpy(), probe.cpu().numpy()
    ok = (probe >= 0) & (probe < 300)
    assert np.array_equal(gq[ok], q[probe[ok]]) and np.array_equal(gph[ok], ph[probe[ok]])
    assert np.all(np.isnan(gq[~ok])) and np.all(gph[~ok] == -1)
