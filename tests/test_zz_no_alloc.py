"""The allocation-free structure-factor entry point (ar_sf_score_grad_noalloc,
workspace in a fixed per-GPU device array) against ar_sf_score_grad (the
same kernels with the context's workspace), called through the C ABI: two
calls in a row, the second with fewer ROIs and directions than the first,
each with and without the gradient.  The two entry points run the same
kernels in the same order, so score and gradient must be bit-identical; the
score of sampled ROIs is also held to the FP64 oracle at relative 1e-5 (the
structure-factor score bar, Sec. 2.2, Eq. (2))."""
import numpy as np
import pytest
import torch

from paper_2009_00735_amd import synth

pytestmark = pytest.mark.gpu

F = np.array([[4.2767, 4.9383, 6.9838, 8.1892],      # fcc Al {111},{200},{220},{311}
              [4.9276, 6.9686, 8.5347, 9.8552]])     # bcc Fe {110},{200},{211},{220}


@pytest.fixture(scope="module")
def nat():
    from paper_2009_00735_amd import native
    return native


@pytest.fixture(scope="module")
def ctx(nat):
    return nat.Context(0)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def case(orc, n_roi, level, seed):
    """Ragged two-phase ROIs (fcc Al / bcc Fe, R = 2 nm, 50 % deletion,
    sigma = 0.05 nm, one empty ROI), random orientations and targets."""
    gen = np.random.default_rng(seed)
    dirs = synth.icosphere(level)
    qs = synth.random_orientations(n_roi, seed)
    phase = (np.arange(n_roi) % 2).astype(np.int32)
    rels = []
    for i in range(n_roi):
        if i == n_roi // 2:
            rels.append(np.zeros((0, 3), np.float32))
            continue
        kind, a = synth.PHASES[phase[i]]
        p = synth.lattice_in_ball(kind, a, qs[i], gen.random(3), np.zeros(3), 2.5)
        keep = synth.delete_exact(len(p), 0.5, gen)
        p = (p[keep] + gen.normal(0, 0.05, (len(keep), 3))).astype(np.float32)
        rels.append(orc.roi_gather(p, np.zeros(3, np.float32), float(gen.uniform(1.2, 2.0))))
    offsets = np.concatenate([[0], np.cumsum([len(r) for r in rels])]).astype(np.int64)
    rel4 = np.zeros((offsets[-1], 4), np.float32)
    rel4[:, :3] = np.concatenate(rels)
    T = gen.uniform(0.0, 0.6, (2, 4, len(dirs))).astype(np.float32)
    q0 = np.array([synth.random_orientations(1, 1000 + seed * 97 + i)[0] for i in range(n_roi)], np.float32)
    return dirs, rels, offsets, rel4, q0, phase, T


@pytest.mark.parametrize("n_roi, level", [(64, 5), (5, 3)])
def test_noalloc_matches_allocating_entry_point(nat, ctx, orc, n_roi, level):
    dirs, rels, offsets, rel4, q0, phase, T = case(orc, n_roi, level, seed=n_roi + level)
    args = (dev(rel4), dev(offsets, torch.int64), dev(q0), dev(phase, torch.int32), dev(dirs), dev(F), dev(T))
    s_ref, g_ref = nat.ar_sf_score_grad(ctx, *args, grad=True)
    s0_ref, _ = nat.ar_sf_score_grad(ctx, *args, grad=False)
    score = torch.full((n_roi,), float("nan"), device="cuda")
    grad = torch.full((n_roi, 4), float("nan"), device="cuda")
    nat.ar_sf_score_grad_noalloc(ctx, *args, score, grad)
    score0 = torch.full((n_roi,), float("nan"), device="cuda")
    nat.ar_sf_score_grad_noalloc(ctx, *args, score0, None)
    torch.cuda.synchronize()
    assert torch.equal(score, s_ref) and torch.equal(grad, g_ref)
    assert torch.equal(score0, s0_ref)
    for r in (0, n_roi // 2, n_roi - 1):
        j = orc.sf_score(rels[r], q0[r].astype(np.float64), dirs, F[phase[r]], T[phase[r]].astype(np.float64))
        assert abs(float(score[r]) - j) <= 1e-5 * j, (r, float(score[r]), j)


def test_noalloc_rejects_calls_beyond_the_fixed_workspace(nat, ctx):
    """25000 ROIs at 10242 directions need about 41 MB of partials: refused
    before anything is queued, outputs untouched."""
    n_roi = 25000
    dirs = dev(synth.icosphere(5))
    score = torch.full((n_roi,), -1.0, device="cuda")
    with pytest.raises(nat.AraulloError, match="fixed workspace"):
        nat.ar_sf_score_grad_noalloc(ctx, torch.zeros((1, 4), device="cuda"),
                                     torch.zeros(n_roi + 1, dtype=torch.int64, device="cuda"),
                                     torch.zeros((n_roi, 4), device="cuda"),
                                     torch.zeros(n_roi, dtype=torch.int32, device="cuda"), dirs, dev(F),
                                     torch.zeros((2, 4, dirs.shape[0]), device="cuda"), score, None)
    torch.cuda.synchronize()
    assert bool((score == -1.0).all())
