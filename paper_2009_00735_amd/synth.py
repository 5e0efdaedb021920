"""Seeded synthetic atom-probe specimens shaped like the paper's workloads.

This module produces *inputs only*: atom positions, ROI centres, projection
directions, orientations and window spacings.  It contains none of the
method's arithmetic (no projection, binning, Fourier transform, peak picking,
normalisation, matching or disorientation); both the CPU oracle and the GPU
path consume what it returns.

Paper passages the recipes follow (Kuehbach et al., arXiv 2009.00735):
  * fcc Al a = 0.405 nm and bcc lattices, rotated single crystals
    (Sec. 3.1, "Verification of the methods");
  * random deletion to a kept fraction eta and Gaussian displacement noise
    (Sec. 3.1, noise-robustness study);
  * ROI ensembles on a 3D grid or by random sampling, spherical, radius R
    (Sec. 2.1 and Sec. 2.5);
  * directions = nodes of a geodesic sphere mesh (Sec. 2.2, RSP paragraph);
  * Poisson-Voronoi polycrystal with random grain orientations
    (Sec. 3.3, polycrystal verification);
  * peak windows of +-10 % around a lattice-plane spacing (supplement,
    reconstruction parameters of the Al bicrystal: 1.823-2.230 A about
    d200 = 2.025 A).

Seeds: numpy PCG64 seeded with SeedSequence([200900735, config, stream]);
streams 0 orientation, 1 lattice offset, 2 deletion, 3 noise, 4 ROI placement,
5 library orientations, 6 Voronoi seeds, 8 reference offsets.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

SEED_ROOT = 200900735
STREAM_ORIENTATION = 0
STREAM_OFFSET = 1
STREAM_DELETION = 2
STREAM_NOISE = 3
STREAM_ROI = 4
STREAM_LIBRARY = 5
STREAM_VORONOI = 6
STREAM_REFERENCE = 8

A_AL = 0.405   # nm, fcc aluminium
A_FE = 0.287   # nm, bcc iron

A_AL3SC = 0.4105   # nm, L1_2 Al3Sc
A_AL3LI = 0.4010   # nm, L1_2 Al3Li (delta')

BASIS = {
    "fcc": np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]),
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "L12": np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]),
}
# atom type per basis site: L1_2 (Cu3Au type) puts the minority species (Sc,
# Li: type 1) on the cube corner and aluminium (type 0) on the face centres
BASIS_TYPES = {"fcc": np.array([0, 0, 0, 0]), "bcc": np.array([0, 0]), "L12": np.array([1, 0, 0, 0])}
TYPE_AL, TYPE_MINOR = 0, 1

# Lattice-plane spacings (nm) that centre the four peak windows: fcc Al
# {111}, {200}, {220}, {311}.
WINDOW_SPACINGS_NM = (0.405 / math.sqrt(3.0), 0.405 / 2.0, 0.405 / math.sqrt(8.0), 0.405 / math.sqrt(11.0))
WINDOW_HALF_WIDTH = 0.10  # +-10 %, as in the supplement's Al {002} interval


def rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, stream])))


def window_spacings(centres=WINDOW_SPACINGS_NM, half_width=WINDOW_HALF_WIDTH) -> np.ndarray:
    """[n_win][2] (d_min, d_max) in nm: each spacing widened by +-half_width."""
    c = np.asarray(centres, dtype=np.float64)
    return np.stack([c * (1.0 - half_width), c * (1.0 + half_width)], axis=1)


# --------------------------------------------------------------------------
# directions: geodesic (icosphere) mesh nodes
# --------------------------------------------------------------------------
def icosphere(level: int) -> np.ndarray:
    """Unit vertices of an icosahedron subdivided `level` times (10*4^level + 2).

    Built and normalised in float64, returned as float32 [n][3].
    """
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
             (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache: Dict[Tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = v[i] + v[j]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    out = np.array(v, dtype=np.float64)
    out /= np.linalg.norm(out, axis=1, keepdims=True)
    return out.astype(np.float32)


def cubic_directions_26() -> np.ndarray:
    """The 26 symmetric variants of <100>, <110>, <111> as unit float32 vectors."""
    d = []
    for x in (-1, 0, 1):
        for y in (-1, 0, 1):
            for z in (-1, 0, 1):
                if (x, y, z) != (0, 0, 0):
                    d.append((x, y, z))
    d = np.array(d, dtype=np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d.astype(np.float32)


# --------------------------------------------------------------------------
# orientations (quaternions w, x, y, z; active crystal -> lab)
# --------------------------------------------------------------------------
def shoemake(n: int, gen: np.random.Generator) -> np.ndarray:
    """n uniform random unit quaternions (Shoemake 1992), float64 [n][4], w >= 0."""
    u1, u2, u3 = gen.random(n), gen.random(n), gen.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], axis=1)
    q[q[:, 0] < 0] *= -1.0
    return q


def quat_matrix(q: np.ndarray) -> np.ndarray:
    """3x3 rotation matrix of a unit quaternion (w, x, y, z), float64."""
    w, x, y, z = (float(c) for c in np.asarray(q, dtype=np.float64) / np.linalg.norm(q))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_axis_angle(axis, deg: float) -> np.ndarray:
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    h = math.radians(deg) / 2.0
    return np.concatenate([[math.cos(h)], math.sin(h) * axis])


def quat_bunge(phi1: float, Phi: float, phi2: float) -> np.ndarray:
    """Active crystal->lab quaternion of Bunge angles (deg): the transpose of
    the passive matrix Rz(phi2) Rx(Phi) Rz(phi1)."""
    def qz(a):
        return quat_axis_angle([0, 0, 1], a)

    def qx(a):
        return quat_axis_angle([1, 0, 0], a)

    def mul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    # active rotation = Rz(phi1) Rx(Phi) Rz(phi2)
    q = mul(mul(qz(phi1), qx(Phi)), qz(phi2))
    return q if q[0] >= 0 else -q


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------
def lattice_in_ball(kind: str, a: float, q: np.ndarray, offset_frac: np.ndarray,
                    centre: np.ndarray, radius: float) -> np.ndarray:
    """Lattice sites (float64, lab frame) of a crystal rotated by q whose origin
    sits at `centre` + R(q) (offset_frac * a), inside a ball of `radius`."""
    Rm = quat_matrix(q)
    n = int(math.ceil(radius / a)) + 2
    r = np.arange(-n, n + 1, dtype=np.float64)
    ijk = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 1, 3)
    pts = ((ijk + BASIS[kind][None] + np.asarray(offset_frac)[None, None]) * a).reshape(-1, 3)
    lab = pts @ Rm.T
    keep = np.einsum("ij,ij->i", lab, lab) <= radius * radius
    return lab[keep] + np.asarray(centre, dtype=np.float64)


def typed_lattice_in_ball(kind: str, a: float, q: np.ndarray, offset_frac: np.ndarray,
                          centre: np.ndarray, radius: float) -> Tuple[np.ndarray, np.ndarray]:
    """lattice_in_ball with the atom type of every site (BASIS_TYPES)."""
    Rm = quat_matrix(q)
    n = int(math.ceil(radius / a)) + 2
    r = np.arange(-n, n + 1, dtype=np.float64)
    ijk = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 1, 3)
    pts = ((ijk + BASIS[kind][None] + np.asarray(offset_frac)[None, None]) * a).reshape(-1, 3)
    types = np.tile(BASIS_TYPES[kind], len(ijk)).astype(np.int32)
    lab = pts @ Rm.T
    keep = np.einsum("ij,ij->i", lab, lab) <= radius * radius
    return lab[keep] + np.asarray(centre, dtype=np.float64), types[keep]


def l12_specimen(n_roi: int = 64, eta: float = 0.5, sigma: float = 0.03, R: float = 1.0, seed: int = 0,
                 a: float = A_AL3SC):
    """A rotated L1_2 crystal (types 0 = Al, 1 = Sc/Li) in a ball of radius
    3R + 1 nm with kept fraction eta and Gaussian displacements sigma; n_roi
    ROI centres uniform in the ball of radius 3R.  Returns (positions float32,
    types int32, centres float32, q)."""
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 12, seed])))
    q = shoemake(1, gen)[0]
    pos, types = typed_lattice_in_ball("L12", a, q, gen.random(3), np.zeros(3), 3 * R + 1.0)
    keep = delete_exact(len(pos), eta, gen)
    pos, types = pos[keep], types[keep]
    pos = pos + gen.normal(0.0, sigma, pos.shape)
    c = gen.normal(size=(n_roi, 3))
    c *= (3 * R * gen.random(n_roi) ** (1 / 3) / np.linalg.norm(c, axis=1))[:, None]
    return pos.astype(np.float32), types, c.astype(np.float32), q


def lattice_in_box(kind: str, a: float, q: np.ndarray, offset_frac: np.ndarray,
                   lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Lattice sites of a rotated crystal inside the axis-aligned box [lo, hi);
    the crystal origin sits at the box centre + R(q) (offset_frac * a).
    Enumerates the integer cells covering the box's crystal-frame bounding box."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = 0.5 * (lo + hi)
    Rm = quat_matrix(q)
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])]) - c
    xc = corners @ Rm                                   # crystal-frame coordinates (R^T p)
    off = np.asarray(offset_frac, dtype=np.float64)
    i0 = np.floor(xc.min(0) / a - off).astype(int) - 1
    i1 = np.ceil(xc.max(0) / a - off).astype(int) + 1
    out = []
    basis = BASIS[kind]
    # slab by slab along the first axis to bound temporaries
    j = np.arange(i0[1], i1[1] + 1, dtype=np.float64)
    k = np.arange(i0[2], i1[2] + 1, dtype=np.float64)
    J, K = np.meshgrid(j, k, indexing="ij")
    JK = np.stack([J.ravel(), K.ravel()], axis=1)
    for i in range(i0[0], i1[0] + 1):
        cell = np.concatenate([np.full((len(JK), 1), float(i)), JK], axis=1)
        pts = ((cell[:, None, :] + basis[None] + off[None, None]) * a).reshape(-1, 3)
        lab = pts @ Rm.T + c
        keep = np.all((lab >= lo) & (lab < hi), axis=1)
        if keep.any():
            out.append(lab[keep])
    return np.concatenate(out) if out else np.zeros((0, 3))


def delete_exact(n: int, eta: float, gen: np.random.Generator) -> np.ndarray:
    """Sorted indices of round(eta*n) atoms kept, drawn without replacement."""
    k = int(round(eta * n))
    return np.sort(gen.choice(n, size=k, replace=False))


def gaussian_noise(n: int, sigma_xy: float, sigma_z: float, gen: np.random.Generator) -> np.ndarray:
    e = gen.standard_normal((n, 3))
    e[:, 0:2] *= sigma_xy
    e[:, 2] *= sigma_z
    return e


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Specimen:
    positions: np.ndarray            # float32 [n_atoms][3] nm
    centres: np.ndarray              # float32 [n_roi][3] nm
    radius: float                    # nm
    directions: np.ndarray           # float32 [n_dir][3] unit
    nbins: int
    spacings: np.ndarray             # float64 [n_win][2] (d_min, d_max) nm
    truth_q: np.ndarray              # float64 [n_roi][4]
    truth_phase: np.ndarray          # int32 [n_roi] (0 fcc Al, 1 bcc Fe)
    truth_share: np.ndarray          # float64 [n_roi] atom share of the dominant grain
    atom_grain: Optional[np.ndarray] = None
    grain_q: Optional[np.ndarray] = None
    grain_phase: Optional[np.ndarray] = None
    name: str = ""


PHASES = (("fcc", A_AL), ("bcc", A_FE))


def single_roi(nbins: int = 256, level: int = 3) -> Specimen:
    """Single ROI R = 1 nm in a rotated fcc Al crystal, 50 % deletion, sigma 0.05 nm."""
    cfg = 1
    q = shoemake(1, rng(cfg, STREAM_ORIENTATION))[0]
    off = rng(cfg, STREAM_OFFSET).random(3)
    R = 1.0
    pts = lattice_in_ball("fcc", A_AL, q, off, np.zeros(3), R + 0.5)
    keep = delete_exact(len(pts), 0.5, rng(cfg, STREAM_DELETION))
    pts = pts[keep] + gaussian_noise(len(keep), 0.05, 0.05, rng(cfg, STREAM_NOISE))
    return Specimen(positions=pts.astype(np.float32), centres=np.zeros((1, 3), np.float32), radius=R,
                    directions=icosphere(level), nbins=nbins, spacings=window_spacings(),
                    truth_q=q[None], truth_phase=np.zeros(1, np.int32), truth_share=np.ones(1),
                    name="single ROI R=1 nm fcc Al, 642 directions, 256 bins")


def single_grain_box(level: int = 5, nbins: int = 1024, grid: Tuple[int, int, int] = (10, 10, 20)) -> Specimen:
    """Single-grain fcc Al box 20x20x40 nm at 30 atoms/nm^3, ROIs on a 2 nm grid."""
    cfg = 2
    q = shoemake(1, rng(cfg, STREAM_ORIENTATION))[0]
    off = rng(cfg, STREAM_OFFSET).random(3)
    R = 2.0
    gx, gy, gz = grid
    lo = np.array([-2.0, -2.0, -2.0])
    hi = np.array([2.0 * gx + 2.0, 2.0 * gy + 2.0, 2.0 * gz + 2.0])
    pts = lattice_in_box("fcc", A_AL, q, off, lo, hi)
    eta = 30.0 * A_AL ** 3 / 4.0
    keep = delete_exact(len(pts), eta, rng(cfg, STREAM_DELETION))
    pts = pts[keep] + gaussian_noise(len(keep), 0.05, 0.05, rng(cfg, STREAM_NOISE))
    i, j, k = np.meshgrid(np.arange(gx), np.arange(gy), np.arange(gz), indexing="ij")
    centres = np.stack([1.0 + 2.0 * i, 1.0 + 2.0 * j, 1.0 + 2.0 * k], axis=-1).reshape(-1, 3)
    n = len(centres)
    return Specimen(positions=pts.astype(np.float32), centres=centres.astype(np.float32), radius=R,
                    directions=icosphere(level), nbins=nbins, spacings=window_spacings(),
                    truth_q=np.repeat(q[None], n, 0), truth_phase=np.zeros(n, np.int32),
                    truth_share=np.ones(n),
                    name=f"single-grain fcc Al box {2*gx}x{2*gy}x{2*gz} nm, {n} ROIs R=2 nm, "
                         f"{len(icosphere(level)) if level < 6 else 40962} directions, {nbins} bins")


# truncated cone: axis z in [0, H], radius r(z) = r_top + (H - z) tan(half_angle)
CONE_H = 60.0
CONE_R_TOP = 15.0
CONE_HALF_ANGLE_DEG = 10.0


def cone_radius(z):
    return CONE_R_TOP + (CONE_H - z) * math.tan(math.radians(CONE_HALF_ANGLE_DEG))


def in_cone(p: np.ndarray) -> np.ndarray:
    z = p[:, 2]
    r2 = p[:, 0] ** 2 + p[:, 1] ** 2
    return (z >= 0.0) & (z < CONE_H) & (r2 < cone_radius(z) ** 2)


def in_cone_dilated(p: np.ndarray, margin: float) -> np.ndarray:
    """Points within `margin` (radially and axially) of the cone."""
    z = p[:, 2]
    r2 = p[:, 0] ** 2 + p[:, 1] ** 2
    return (z >= -margin) & (z < CONE_H + margin) & (r2 < (cone_radius(np.clip(z, 0.0, CONE_H)) + margin) ** 2)


def uniform_in_cone(n: int, gen: np.random.Generator, margin: float = 0.0) -> np.ndarray:
    """n points uniform in the cone dilated by `margin` (rejection sampling)."""
    rb = cone_radius(0.0) + margin
    out = []
    got = 0
    while got < n:
        m = max(2 * (n - got), 64)
        p = np.stack([gen.uniform(-rb, rb, m), gen.uniform(-rb, rb, m),
                      gen.uniform(-margin, CONE_H + margin, m)], axis=1)
        p = p[in_cone_dilated(p, margin) if margin > 0 else in_cone(p)]
        out.append(p)
        got += len(p)
    return np.concatenate(out)[:n]


_POLY_CACHE: Dict[Tuple, Tuple] = {}


def polycrystal(n_grains: int = 20, eta: float = 0.5, sigma: float = 0.05, cfg: int = 3):
    """20-grain Poisson-Voronoi polycrystal in the truncated cone; even grains
    fcc Al, odd grains bcc Fe; each grain its own random orientation/offset.

    Returns (positions float32 [n][3], atom_grain int32 [n], grain_q, grain_phase)."""
    key = (n_grains, eta, sigma, cfg)
    if key in _POLY_CACHE:
        return _POLY_CACHE[key]
    from scipy.spatial import cKDTree
    seeds = uniform_in_cone(n_grains, rng(cfg, STREAM_VORONOI))
    seed_tree = cKDTree(seeds)
    gq = shoemake(n_grains, rng(cfg, STREAM_ORIENTATION))
    goff = rng(cfg, STREAM_OFFSET).random((n_grains, 3))
    gphase = (np.arange(n_grains) % 2).astype(np.int32)
    # coarse voxel assignment to bound each grain's extent
    rb = cone_radius(0.0)
    h = 1.0
    xs = np.arange(-rb - h, rb + h, h) + 0.5 * h
    zs = np.arange(-h, CONE_H + h, h) + 0.5 * h
    X, Y, Z = np.meshgrid(xs, xs, zs, indexing="ij")
    vox = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    z = vox[:, 2]
    near_cone = (z > -2 * h) & (z < CONE_H + 2 * h) & (
        vox[:, 0] ** 2 + vox[:, 1] ** 2 < (cone_radius(np.clip(z, 0.0, CONE_H)) + 2 * h) ** 2)
    vox = vox[near_cone]
    near = seed_tree.query(vox, workers=-1)[1]
    all_pts, all_g = [], []
    for g in range(n_grains):
        vg = vox[near == g]
        if len(vg) == 0:
            continue
        lo = vg.min(0) - 2.0 * h
        hi = vg.max(0) + 2.0 * h
        kind, a = PHASES[gphase[g]]
        pts = lattice_in_box(kind, a, gq[g], goff[g], lo, hi)
        pts = pts[in_cone(pts)]
        # nearest seed must be g
        pts = pts[seed_tree.query(pts, workers=-1)[1] == g]
        all_pts.append(pts)
        all_g.append(np.full(len(pts), g, np.int32))
    pts = np.concatenate(all_pts)
    grain = np.concatenate(all_g)
    keep = delete_exact(len(pts), eta, rng(cfg, STREAM_DELETION))
    pts = pts[keep] + gaussian_noise(len(keep), sigma, sigma, rng(cfg, STREAM_NOISE))
    out = (pts.astype(np.float32), grain[keep], gq, gphase)
    _POLY_CACHE[key] = out
    return out


def _roi_truth(tree, pos64, grain, centres, R):
    counts = np.zeros(len(centres), np.int64)
    dom = np.zeros(len(centres), np.int32)
    share = np.zeros(len(centres))
    for i, idx in enumerate(tree.query_ball_point(centres, R, workers=-1)):
        counts[i] = len(idx)
        if len(idx):
            b = np.bincount(grain[idx])
            dom[i] = int(np.argmax(b))
            share[i] = b[dom[i]] / len(idx)
    return counts, dom, share


def polycrystal_rois(n_roi: int, min_atoms: int = 100, max_atoms: Optional[int] = None,
                     min_share: float = 0.0, cfg: int = 3, R: float = 2.0,
                     stream: int = STREAM_ROI):
    """ROI centres drawn uniformly in the cone (surface-clipped ROIs kept)
    whose atom count lies in [min_atoms, max_atoms] and whose dominant-grain
    share is >= min_share. Returns (centres float32, dominant grain, share, counts)."""
    from scipy.spatial import cKDTree
    pos, grain, gq, gphase = polycrystal(cfg=3)
    tree = cKDTree(pos.astype(np.float64))
    gen = rng(cfg, stream)
    acc_c, acc_g, acc_s, acc_n = [], [], [], []
    got = 0
    while got < n_roi:
        # centres up to 0.9 R outside the surface: clipped ROIs keep >= min_atoms
        cand = uniform_in_cone(max(2 * (n_roi - got), 256), gen, margin=0.9 * R)
        counts, dom, share = _roi_truth(tree, pos, grain, cand, R)
        ok = counts >= min_atoms
        if max_atoms is not None:
            ok &= counts <= max_atoms
        ok &= share >= min_share
        acc_c.append(cand[ok]); acc_g.append(dom[ok]); acc_s.append(share[ok]); acc_n.append(counts[ok])
        got += int(ok.sum())
    c = np.concatenate(acc_c)[:n_roi]
    return (c.astype(np.float32), np.concatenate(acc_g)[:n_roi], np.concatenate(acc_s)[:n_roi],
            np.concatenate(acc_n)[:n_roi])


def polycrystal_cone(n_roi: int = 8000, level: int = 5, nbins: int = 1024) -> Specimen:
    """Fcc Al / bcc Fe Voronoi polycrystal in a truncated cone; uneven,
    surface-clipped ROIs of R = 2 nm with at least 100 atoms."""
    pos, grain, gq, gphase = polycrystal(cfg=3)
    centres, dom, share, counts = polycrystal_rois(n_roi)
    return Specimen(positions=pos, centres=centres, radius=2.0, directions=icosphere(level), nbins=nbins,
                    spacings=window_spacings(), truth_q=gq[dom], truth_phase=gphase[dom].astype(np.int32),
                    truth_share=share, atom_grain=grain, grain_q=gq, grain_phase=gphase,
                    name=f"20-grain fcc Al + bcc Fe cone, {n_roi} uneven ROIs R=2 nm")


def refinement_rois(n_roi: int = 4096):
    """ROIs of the polycrystal with 800-1200 atoms and dominant share >= 0.9."""
    pos, grain, gq, gphase = polycrystal(cfg=3)
    centres, dom, share, counts = polycrystal_rois(n_roi, min_atoms=800, max_atoms=1200, min_share=0.9,
                                                   stream=STREAM_ROI + 100)
    return centres, gq[dom], gphase[dom].astype(np.int32), share


# --------------------------------------------------------------------------
# reference crystals (noise-free, eta = 1, identity orientation)
# --------------------------------------------------------------------------
def reference_rois(phase: int, n_offsets: int = 16, R: float = 2.0, cfg: int = 4):
    """Per phase: a noise-free unrotated crystal ball of radius R + 0.5 and
    `n_offsets` ROI centres at seeded in-cell offsets from its origin.
    Returns (positions float32, centres float32 [n_offsets][3])."""
    kind, a = PHASES[phase]
    pts = lattice_in_ball(kind, a, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), R + a * 2 + 0.5)
    offs = rng(cfg, STREAM_REFERENCE + phase).random((n_offsets, 3)) * a
    return pts.astype(np.float32), offs.astype(np.float32)


def library_orientations(n: int, cfg: int) -> np.ndarray:
    return shoemake(n, rng(cfg, STREAM_LIBRARY))


def random_orientations(n: int, seed: int) -> np.ndarray:
    return shoemake(n, np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 999, seed]))))


def planted_images(n_roi: int, n_lib: int, n_win: int, n_dir: int, seed: int, noise: float = 0.05):
    """Seeded non-negative image sets with a planted match per ROI (inputs for
    exercising the indexing boundary at full sizes without rotated
    references): library rows are random; ROI r is the library row truth[r]
    with a random per-window gain and multiplicative noise.
    Returns (S float32 [n_roi][n_win][n_dir], L float32 [n_lib][n_win][n_dir],
    truth int64 [n_roi])."""
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 777, seed])))
    L = np.empty((n_lib, n_win, n_dir), np.float32)
    for s in range(0, n_lib, 1024):
        blk = gen.random((min(1024, n_lib - s), n_win, n_dir), dtype=np.float32)
        L[s:s + len(blk)] = blk * blk
    truth = gen.integers(0, n_lib, n_roi)
    gain = gen.uniform(0.5, 2.0, (n_roi, n_win, 1)).astype(np.float32)
    jitter = 1.0 + noise * gen.standard_normal((n_roi, n_win, n_dir), dtype=np.float32)
    S = np.abs(L[truth] * gain * jitter).astype(np.float32)
    return S, L, truth


def ranked_images(n_roi: int, n_lib: int, n_win: int, n_dir: int, n_ranked: int, seed: int):
    """Seeded image sets with a planted ranking per ROI (inputs for checking
    long candidate lists): ROI r is a random non-negative image B_r; n_ranked
    library rows (distinct per ROI, at random positions) are B_r * (1 - e_j
    |n_r|) with e_j = 0.01 * 1.04^j and one noise pattern n_r per ROI that is
    zero at every window's largest node, so that each row keeps B_r's window
    maxima and its squared distance to B_r after per-window normalisation is
    e_j^2 times a constant of ROI r: rank j.  The other rows are random.
    Returns (S float32 [n_roi][n_win][n_dir], L float32 [n_lib][n_win][n_dir],
    ranked int64 [n_roi][n_ranked], the planted rows nearest first)."""
    if n_roi * n_ranked > n_lib:
        raise ValueError("n_roi * n_ranked must not exceed n_lib")
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 778, seed])))
    L = gen.random((n_lib, n_win, n_dir), dtype=np.float32) ** 2
    S = 0.05 + gen.random((n_roi, n_win, n_dir), dtype=np.float32) ** 2
    rows = gen.permutation(n_lib)[:n_roi * n_ranked].reshape(n_roi, n_ranked)
    eps = 0.01 * 1.04 ** np.arange(n_ranked)
    for r in range(n_roi):
        n = np.abs(gen.standard_normal((n_win, n_dir))).clip(0.0, 3.0)
        n[np.arange(n_win), np.argmax(S[r], axis=1)] = 0.0
        L[rows[r]] = (S[r][None] * (1.0 - eps[:, None, None] * 0.3 * n[None])).astype(np.float32)
    return S.astype(np.float32), L, rows.astype(np.int64)


# --------------------------------------------------------------------------
# signature-like spherical images (indexing inputs without running the
# signature path): peaks at the crystal directions of each window's
# lattice-plane family, the shape real window-maximum images have
# --------------------------------------------------------------------------
def _family(hkl) -> np.ndarray:
    """One unit vector per antipodal pair of the cubic family {hkl}."""
    out = []
    vals = set()
    h = [abs(x) for x in hkl]
    for perm in itertools.permutations(h):
        for sg in itertools.product((-1, 1), repeat=3):
            v = tuple(a * b for a, b in zip(perm, sg))
            if v == (0, 0, 0):
                continue
            neg = tuple(-a for a in v)
            if neg not in vals:
                vals.add(v)
    for v in sorted(vals):
        out.append(np.array(v, np.float64) / np.linalg.norm(v))
    return np.array(out)


# plane-normal families behind the four windows: fcc {111} {200} {220} {311},
# bcc {110} {200} {211} {220}
BUMP_FAMILIES = {0: [(1, 1, 1), (1, 0, 0), (1, 1, 0), (3, 1, 1)], 1: [(1, 1, 0), (1, 0, 0), (2, 1, 1), (1, 1, 0)]}


def bump_images(directions: np.ndarray, quats: np.ndarray, phase: np.ndarray, n_win: int, width: float = 0.02,
                background: float = 0.1, gain: Optional[np.ndarray] = None, noise: float = 0.0,
                seed: int = 0) -> np.ndarray:
    """Images [n][n_win][n_dir] float32: window w of image i is
    background + sum_a exp((|u . a| - 1) / width) over the directions a of
    family w of phase[i], u = R(q_i)^T n_v (the crystal rotated by q_i seen at
    node v), times gain[i][w] and (1 + noise * N(0,1)) clipped at 0."""
    d = np.asarray(directions, np.float64)
    q = np.asarray(quats, np.float64).reshape(-1, 4)
    ph = np.asarray(phase).reshape(-1)
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 778, seed])))
    fams = {c: [_family(BUMP_FAMILIES[c][w % 4]) for w in range(n_win)] for c in BUMP_FAMILIES}
    out = np.empty((len(q), n_win, len(d)), np.float32)
    for i in range(len(q)):
        u = d @ quat_matrix(q[i])                 # rows R^T n_v
        for w in range(n_win):
            a = fams[int(ph[i])][w]
            x = background + np.exp((np.abs(u @ a.T) - 1.0) / width).sum(axis=1)
            if gain is not None:
                x *= gain[i][w]
            if noise > 0:
                x *= np.maximum(0.0, 1.0 + noise * gen.standard_normal(len(d)))
            out[i, w] = x
    return out


# --------------------------------------------------------------------------
# reciprocal-space benchmark input (supplement, reciprocal-space benchmark:
# 1e4 ROIs of R = 20 A in synthetic aluminium single crystals)
# --------------------------------------------------------------------------
def fsp_specimen(n_roi: int = 10000, R: float = 2.0, box: float = 24.0, eta: float = 1.0, seed: int = 0):
    """A full-density (eta = 1) fcc Al single crystal in a cube of edge `box`
    nm, rotated by a seeded orientation, and n_roi ROI centres uniform in the
    cube shrunk by R (every ROI complete).  Returns (positions float32,
    centres float32, q)."""
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 21, seed])))
    q = shoemake(1, gen)[0]
    lo, hi = np.zeros(3), np.full(3, box)
    pos = lattice_in_box("fcc", A_AL, q, gen.random(3), lo, hi)
    if eta < 1.0:
        pos = pos[delete_exact(len(pos), eta, gen)]
    cen = R + gen.random((n_roi, 3)) * (box - 2 * R)
    return pos.astype(np.float32), cen.astype(np.float32), q


# --------------------------------------------------------------------------
# coarse ROI grids and a bicrystal (Sec. 3.5: ROIs on a cubic grid over an
# aluminium bicrystal, then local refinement)
# --------------------------------------------------------------------------
def roi_grid(lo, hi, h: float) -> np.ndarray:
    """ROI centres lo + h (i + 1/2) along each axis inside [lo, hi), float32 [n][3]."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n = np.floor((hi - lo) / h).astype(int)
    axes = [lo[a] + h * (np.arange(n[a]) + 0.5) for a in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.float32)


def bicrystal(box: float = 12.0, eta: float = 0.5, sigma: tuple = (0.02, 0.08), seed: int = 0):
    """Two fcc Al grains filling the cube [0, box)^3, split at x = box/2, with
    seeded orientations; grain 0 is displaced by sigma[0], grain 1 by sigma[1]
    (a sharp and a blurred grain).  Returns (positions float32, grain int32, q [2][4])."""
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, 31, seed])))
    q = shoemake(2, gen)
    parts, gid = [], []
    for g in range(2):
        lo = np.array([g * box / 2, 0.0, 0.0])
        hi = np.array([(g + 1) * box / 2, box, box])
        p = lattice_in_box("fcc", A_AL, q[g], gen.random(3), lo, hi)
        p = p[delete_exact(len(p), eta, gen)]
        p = p + gen.normal(0.0, sigma[g], p.shape)
        parts.append(p)
        gid.append(np.full(len(p), g, np.int32))
    return np.concatenate(parts).astype(np.float32), np.concatenate(gid), q
