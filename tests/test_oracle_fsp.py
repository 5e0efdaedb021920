"""Pins of the oracle's reciprocal-space grid (Eq. (2) on a cubic k-grid,
reading R14): the origin holds N_w, one atom gives 1 everywhere, two atoms
give 2|cos(2 pi k.x0)|, a perfect lattice gives exactly N_w at its
reciprocal-lattice points, and the fcc structure factor removes (100)."""
import numpy as np

from paper_2009_00735_amd import synth


def test_fsp_closed_forms(orc):
    L, kmax = 32, 10.0
    k = orc.fsp_grid_k(L, kmax)
    assert k[L // 2] == 0.0 and np.isclose(k[1] - k[0], 2 * kmax / L)
    one = orc.fsp_grid(np.array([[0.31, -0.17, 0.42]], np.float32), L, kmax)
    assert np.allclose(one, 1.0, atol=1e-12)
    x0 = np.array([0.123, -0.377, 0.251], np.float32)
    two = orc.fsp_grid(np.stack([x0, -x0]), L, kmax)
    K = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1)
    expect = 2 * np.abs(np.cos(2 * np.pi * (K @ x0.astype(np.float64))))
    assert np.allclose(two, expect, atol=1e-10)
    gen = np.random.default_rng(70)
    pts = gen.uniform(-1, 1, (200, 3)).astype(np.float32)
    g = orc.fsp_grid(pts, L, kmax)
    assert abs(g[L // 2, L // 2, L // 2] - 200) < 1e-9
    # |F(-k)| = |F(k)| (real positions): the grid is symmetric about its origin
    assert np.allclose(g[1:, 1:, 1:], g[1:, 1:, 1:][::-1, ::-1, ::-1], atol=1e-9)
    # explicit k vectors agree with the grid
    idx = gen.integers(0, L, (20, 3))
    kv = k[idx]
    assert np.allclose(orc.fsp_at(pts, kv), g[idx[:, 0], idx[:, 1], idx[:, 2]], atol=1e-10)


def test_fsp_lattice_reflections(orc):
    """A block of 6^3 whole unit cells, a = 0.4 nm (k_max = 10/nm and L = 64
    put 1/a on grid step 8): simple cubic has N_w at (1/a, 0, 0); fcc has 0
    there (its four basis atoms cancel in every whole cell) and N_w at
    (2/a, 0, 0) and (1/a, 1/a, 1/a)."""
    L, kmax, a = 64, 10.0, 0.4
    for kind in ("sc", "fcc"):
        basis = np.zeros((1, 3)) if kind == "sc" else synth.BASIS["fcc"]
        r = np.arange(-3, 3, dtype=np.float64)
        ijk = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 1, 3)
        pts = ((ijk + basis[None]) * a).reshape(-1, 3).astype(np.float32)
        nw = len(pts)
        G = np.array([[1 / a, 0, 0], [2 / a, 0, 0], [1 / a, 1 / a, 1 / a], [0.5 / a, 0, 0]])
        amp = orc.fsp_at(pts, G)
        assert abs(amp[1] - nw) < 1e-6 * nw and abs(amp[2] - nw) < 1e-6 * nw
        if kind == "sc":
            assert abs(amp[0] - nw) < 1e-6 * nw
        else:
            assert amp[0] < 1e-6 * nw
        assert amp[3] < 0.2 * nw                        # half a reciprocal vector: no reflection
