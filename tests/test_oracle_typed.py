"""Pins of the oracle's sub-lattice signatures (Sec. 3.1, the Al3Sc case:
one amplitude spectrum per sub-lattice).  Closed forms of the L1_2 (Cu3Au
type) structure: along <100> and <110> the whole crystal has no superlattice
peak at d = a and d = a/sqrt(2) (equal plane densities), the minority
sub-lattice (simple cubic) has the full peak, and the aluminium sub-lattice
(plane densities alternating 1 : 2) has one third of it; along <111> every
sub-lattice is in phase."""
import math

import numpy as np

from paper_2009_00735_amd import synth


def _amp_ratio(orc, rel, v, k, R, nb):
    vv = np.asarray(v, np.float32) / np.linalg.norm(v)
    amp = orc.amplitudes(orc.sdm_hist(rel, vv, R, nb))
    return amp[int(k) - 1:int(k) + 3].max() / len(rel)


def test_l12_sublattice_peaks(orc):
    R, nb = 2.0, 1024
    a = synth.A_AL3SC
    pts, ty = synth.typed_lattice_in_ball("L12", a, np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3), R + 0.5)
    centre = np.array([0.0137, -0.0071, 0.0049], np.float32)
    L = 2 * R + 2 * R / (nb // 2 - 1)
    rel = {name: orc.roi_gather(pts[sel].astype(np.float32), centre, R)
           for name, sel in (("all", np.ones(len(ty), bool)), ("Al", ty == synth.TYPE_AL),
                             ("minor", ty == synth.TYPE_MINOR))}
    assert len(rel["all"]) == len(rel["Al"]) + len(rel["minor"])
    assert abs(len(rel["Al"]) / len(rel["all"]) - 0.75) < 0.03
    for v, d in (((1, 0, 0), a), ((1, 1, 0), a / math.sqrt(2))):
        k = L / d
        assert _amp_ratio(orc, rel["all"], v, k, R, nb) < 0.05
        assert 0.25 < _amp_ratio(orc, rel["Al"], v, k, R, nb) < 0.40
        assert _amp_ratio(orc, rel["minor"], v, k, R, nb) > 0.85
        for name in rel:                                          # the fundamental at d/2
            assert _amp_ratio(orc, rel[name], v, 2 * k, R, nb) > 0.7
    k111 = L / (a / math.sqrt(3))
    for name in rel:
        assert _amp_ratio(orc, rel[name], (1, 1, 1), k111, R, nb) > 0.9


def test_typed_channels_partition_the_atoms(orc):
    pos, types, cen, q = synth.l12_specimen(n_roi=6, R=1.0, seed=3)
    types = types.copy()
    types[::97] = -1                                              # out-of-range types are never selected
    types[1::101] = 64
    dirs = synth.icosphere(1)
    w = orc.windows_for(1.0, 256, [(0.9 * synth.A_AL3SC, 1.1 * synth.A_AL3SC)] + list(synth.window_spacings()[:2]))
    masks = [(1 << 64) - 1, 1 << synth.TYPE_AL, 1 << synth.TYPE_MINOR, 0]
    img, cnt = orc.signatures_typed(pos, types, masks, cen, 1.0, dirs, 256, w)
    assert img.shape == (6, 4, 3, len(dirs)) and cnt.shape == (6, 4)
    assert np.array_equal(cnt[:, 0], cnt[:, 1] + cnt[:, 2])
    assert np.all(cnt[:, 3] == 0) and np.all(img[:, 3] == 0)
    valid = (types >= 0) & (types < 64)
    ref, rcnt = orc.signatures(pos[valid], cen, 1.0, dirs, 256, w)
    assert np.array_equal(cnt[:, 0], rcnt) and np.array_equal(img[:, 0], ref)
    al, acnt = orc.signatures(pos[types == synth.TYPE_AL], cen, 1.0, dirs, 256, w)
    assert np.array_equal(cnt[:, 1], acnt) and np.array_equal(img[:, 1], al)
