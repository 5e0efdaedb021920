"""Pins of the oracle's sparse form of Eq. S1 (supplement, "Indexing
algorithm"): strongest-entry selection, the look-up table of rotated nodes,
the score and its ranking.  Each is checked against something other than the
oracle's own formula: a library sort, exact mesh symmetries, the separately
pinned dense score, and a worked example in exact binary fractions."""
import numpy as np

from paper_2009_00735_amd import synth


def _match(dirs, targets):
    """Index of the mesh node at each target point (must be within 1e-6)."""
    d = dirs.astype(np.float64)
    out = []
    for t in targets:
        dist = np.linalg.norm(d - t, axis=1)
        j = int(np.argmin(dist))
        assert dist[j] < 1e-6
        out.append(j)
    return np.array(out)


def test_sparse_strong_against_lexsort(orc):
    gen = np.random.default_rng(21)
    n_phase, n_win, n_dir, n_hat = 2, 3, 200, 150
    # values on a coarse grid so that many normalised values tie exactly
    ref = (gen.integers(0, 9, (n_phase, n_win, n_dir)) / 8.0).astype(np.float32)
    ref[1, 1] = 0.0                                          # an all-zero window stays zero
    idx, val = orc.sparse_strong(ref, n_hat)
    for c in range(n_phase):
        m = ref[c].astype(np.float64).max(axis=1, keepdims=True)
        v = np.where(m > 0, ref[c].astype(np.float64) / np.where(m > 0, m, 1.0), 0.0).ravel()
        flat = np.arange(n_win * n_dir)
        order = np.lexsort((flat, -v))[:n_hat]                # value descending, then lower index
        assert np.array_equal(idx[c], order)
        assert np.array_equal(val[c], v[order])
    # all entries: a permutation; the first are the window maxima (value 1)
    idx, val = orc.sparse_strong(ref, n_win * n_dir)
    for c in range(n_phase):
        assert np.array_equal(np.sort(idx[c]), np.arange(n_win * n_dir))
        assert np.all(np.diff(val[c]) <= 0)
    assert val[0, 0] == 1.0 and val[1, -1] == 0.0


def test_sparse_lut_mesh_symmetries(orc):
    """The level-3 icosphere in the standard orientation is mapped onto itself
    by 180 deg about z and by +-120 deg about [111] (cyclic coordinate
    permutations): the look-up node of every strong entry is then the node at
    the exactly rotated position.  +120 and -120 deg differ by R vs R^T."""
    dirs = synth.icosphere(3)
    gen = np.random.default_rng(22)
    ref = gen.random((2, 2, len(dirs))).astype(np.float32)
    si, _ = orc.sparse_strong(ref, 300)
    quats = np.array([[1.0, 0, 0, 0], synth.quat_axis_angle([0, 0, 1], 180), [0.5, 0.5, 0.5, 0.5],
                      [0.5, -0.5, -0.5, -0.5]])
    phase = np.array([0, 1, 0, 1], np.int32)
    lut = orc.sparse_lut(quats, phase, si, dirs)
    d64 = dirs.astype(np.float64)
    maps = [lambda p: p, lambda p: p * [-1, -1, 1], lambda p: p[:, [2, 0, 1]], lambda p: p[:, [1, 2, 0]]]
    for l in range(4):
        v = si[phase[l]] % len(dirs)
        assert np.array_equal(lut[l], _match(dirs, maps[l](d64[v]))), l
    # a generic rotation: nearest node to R(q) n_v by brute force
    q = synth.random_orientations(2, 23)
    lut = orc.sparse_lut(q, [1, 0], si, dirs)
    for l, c in enumerate([1, 0]):
        rot = d64[si[c] % len(dirs)] @ synth.quat_matrix(q[l]).T
        assert np.array_equal(lut[l], np.argmax(rot @ d64.T, axis=1))


def test_sparse_delta_all_entries_equals_dense_ssd(orc):
    """With every entry kept and a rotation that permutes the mesh, the sparse
    score equals the dense score against the rotated reference of the dense
    reading (value at node v taken from the node closest to R^T n_v), which is
    pinned on its own: the two readings agree on the rotation direction."""
    dirs = synth.icosphere(2)
    gen = np.random.default_rng(24)
    ref = gen.random((1, 2, len(dirs))).astype(np.float32)
    S = gen.random((3, 2, len(dirs))).astype(np.float32)
    Sh = orc.normalise(S)
    K = 2 * len(dirs)
    si, sv = orc.sparse_strong(ref, K)
    quats = np.array([[1.0, 0, 0, 0], [0.5, 0.5, 0.5, 0.5], synth.quat_axis_angle([0, 0, 1], 180)])
    phase = np.zeros(3, np.int32)
    lut = orc.sparse_lut(quats, phase, si, dirs)
    Lh = orc.normalise(orc.library_images(ref, phase, quats, dirs))
    for r in range(3):
        sparse = orc.sparse_pairs(Sh, si, sv, phase, lut, np.full(3, r))
        dense = orc.ssd_pairs(Sh, Lh, np.full(3, r), np.arange(3))
        assert np.allclose(sparse, dense, rtol=1e-12, atol=0)


def test_sparse_worked_example(orc):
    """Level-0 icosphere (12 vertices), two windows, four strong entries; all
    values are binary fractions, so every score below is exact.

    Reference, window 0: node 5 = 4, node 9 = 2, other nodes 1 -> normalised
    1, 0.5, 0.25; window 1: nodes 0 and 8 = 3, others 0 -> 1, 1, 0.
    Strong entries (value, then flat index w*12+v): 5 (1), 12 (1), 20 (1),
    9 (0.5).
    ROI, window 0: node 4 = 2, node 11 = 1, node 5 = 0.5 -> 1, 0.5, 0.25;
    window 1: nodes 3 and 10 = 5, node 0 = 2.5 -> 1, 1, 0.5.
    Look-up nodes (5, 0, 8, 9) for identity: (5, 0, 8, 9);
    180 deg about z, (x,y,z) -> (-x,-y,z): (4, 3, 10, 11);
    120 deg about [111], (x,y,z) -> (z,x,y): (9, 4, 0, 1).
    Delta: identity (0.25-1)^2 + (0.5-1)^2 + (0-1)^2 + (0-0.5)^2 = 2.0625;
    180z: 0; 120[111]: 1 + 1 + 0.25 + 0.25 = 2.5."""
    dirs = synth.icosphere(0)
    ref = np.ones((1, 2, 12), np.float32)
    ref[0, 0, 5], ref[0, 0, 9] = 4.0, 2.0
    ref[0, 1] = 0.0
    ref[0, 1, 0] = ref[0, 1, 8] = 3.0
    S = np.zeros((1, 2, 12), np.float32)
    S[0, 0, 4], S[0, 0, 11], S[0, 0, 5] = 2.0, 1.0, 0.5
    S[0, 1, 3] = S[0, 1, 10] = 5.0
    S[0, 1, 0] = 2.5
    si, sv = orc.sparse_strong(ref, 4)
    assert si.tolist() == [[5, 12, 20, 9]] and sv.tolist() == [[1.0, 1.0, 1.0, 0.5]]
    quats = np.array([[1.0, 0, 0, 0], synth.quat_axis_angle([0, 0, 1], 180), [0.5, 0.5, 0.5, 0.5]])
    phase = np.zeros(3, np.int32)
    lut = orc.sparse_lut(quats, phase, si, dirs)
    assert lut.tolist() == [[5, 0, 8, 9], [4, 3, 10, 11], [9, 4, 0, 1]]
    idx, sc = orc.sparse_index_topk(orc.normalise(S), si, sv, phase, lut, 3)
    assert idx.tolist() == [[1, 0, 2]] and sc.tolist() == [[0.0, 2.0625, 2.5]]


def test_sparse_topk_brute_force(orc):
    dirs = synth.icosphere(1)
    gen = np.random.default_rng(25)
    ref = gen.random((2, 2, len(dirs))).astype(np.float32)
    si, sv = orc.sparse_strong(ref, 20)
    q = synth.random_orientations(30, 26)
    q[17] = q[3]                                          # same phase below: an exact tie
    phase = np.array([0] * 20 + [1] * 10, np.int32)
    lut = orc.sparse_lut(q, phase, si, dirs)
    S = gen.random((4, 2, len(dirs))).astype(np.float32)
    Sh = orc.normalise(S)
    Sh[2] = 0.0
    Sh[2].reshape(-1)[si[0]] = sv[0]                      # ROI 2 sees exactly the strong values ...
    Sh[2, :, :] = 0.0
    for i in range(20):                                   # ... at the look-up nodes of entry 3
        w = si[0, i] // len(dirs)
        Sh[2, w, lut[3, i]] = sv[0, i]
    idx, sc = orc.sparse_index_topk(Sh, si, sv, phase, lut, 6)
    for r in range(4):
        d = []
        for l in range(30):
            c = phase[l]
            d.append(sum((Sh[r, si[c, i] // len(dirs), lut[l, i]] - sv[c, i]) ** 2 for i in range(20)))
        order = sorted(range(30), key=lambda l: (d[l], l))[:6]
        assert list(idx[r]) == order
        assert np.allclose(sc[r], [d[l] for l in order], rtol=1e-13, atol=0)
    assert list(idx[2, :2]) == [3, 17] and sc[2, 0] == 0.0 and sc[2, 1] == 0.0
