"""Batched persistent signatures (uneven, surface-clipped ROIs; one
persistent launch replayed as a HIP graph; autotuned tile): identical images
to the plain per-launch kernel, and oracle parity on sampled ROIs."""
import numpy as np
import pytest
import torch

from paper_2009_00735_amd import synth
from parity_bars import assert_images

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    from paper_2009_00735_amd import native
    return native


@pytest.fixture(scope="module")
def ctx(nat):
    return nat.Context(0)


@pytest.fixture(scope="module")
def cone(nat, ctx):
    s = synth.polycrystal_cone()
    pos = torch.from_numpy(s.positions).cuda()
    cen = torch.from_numpy(s.centres).cuda()
    dirs = torch.from_numpy(s.directions).cuda()
    off, rel = nat.ar_roi_gather(ctx, pos, cen, s.radius)
    w = nat.windows_for(s.radius, s.nbins, s.spacings)
    return s, pos, cen, dirs, off, rel, w


def test_plan_equals_plain_and_replays(nat, ctx, cone):
    s, pos, cen, dirs, off, rel, w = cone
    counts = torch.diff(off).cpu().numpy()
    assert counts.min() >= 100 and counts.max() > 1000
    plain = nat.araullo_signatures_csr(ctx, rel, off, s.radius, dirs, s.nbins, w)
    plan = nat.SignaturePlan(ctx, len(s.centres), int(off[-1]), len(s.directions), s.nbins, len(w))
    img = plan.run(rel, off, s.radius, dirs, w, use_graph=False)
    assert torch.equal(img, plain)
    tuned = plan.tune(rel, off, s.radius, dirs, w)
    assert torch.equal(tuned, plain)
    dpi, cap, bpc, occ = plan.config()
    assert dpi >= 1 and cap % 256 == 0 and 256 <= cap <= 4096 and bpc >= 1 and occ in (1, 4)
    out = torch.empty_like(plain)
    for rep in range(3):
        out.fill_(-1.0)
        plan.run(rel, off, s.radius, dirs, w, out=out, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(out, plain), rep
        # unrelated eager work between replays
        _ = (plain * 2.0).sum().item()


@pytest.mark.parametrize("dpi,cap,bpc,occ", [(7, 256, 2, 1), (64, 512, 4, 4), (33, 1024, 3, 1), (128, 4096, 1, 4)])
def test_every_plan_configuration_is_bit_identical(nat, ctx, cone, dpi, cap, bpc, occ):
    """Stages smaller than the largest ROI stream atoms in chunks (workgroup
    barriers per refill); direction chunks that do not divide the mesh leave
    idle wavefronts in the last round.  Histograms are exact and the
    transform code is shared, so every configuration writes the same bits."""
    s, pos, cen, dirs, off, rel, w = cone
    plain = nat.araullo_signatures_csr(ctx, rel, off, s.radius, dirs, s.nbins, w)
    plan = nat.SignaturePlan(ctx, len(s.centres), int(off[-1]), len(s.directions), s.nbins, len(w))
    plan.set_config(dpi, cap, bpc, occ)
    assert plan.config() == (dpi, cap, bpc, occ)
    for graph in (False, True):
        img = plan.run(rel, off, s.radius, dirs, w, use_graph=graph)
        torch.cuda.synchronize()
        assert torch.equal(img, plain), graph


def test_plan_sampled_oracle_parity(nat, ctx, orc, cone):
    s, pos, cen, dirs, off, rel, w = cone
    plan = nat.SignaturePlan(ctx, len(s.centres), int(off[-1]), len(s.directions), s.nbins, len(w))
    img = plan.run(rel, off, s.radius, dirs, w, use_graph=True)
    torch.cuda.synchronize()
    counts = torch.diff(off).cpu().numpy()
    pick = [int(np.argmin(counts)), int(np.argmax(counts)), int(np.argsort(counts)[len(counts) // 2])]
    dsel = np.sort(np.random.default_rng(3).choice(len(s.directions), 400, replace=False))
    ref, rcnt = orc.signatures(s.positions, s.centres[pick], s.radius, s.directions[dsel], s.nbins, w.numpy())
    got = img[torch.as_tensor(pick).cuda()][:, :, torch.as_tensor(dsel).cuda()].cpu().numpy().astype(np.float64)
    assert np.array_equal(counts[pick], rcnt)
    for i in range(len(pick)):
        assert_images(got[i], ref[i], rcnt[i], f"ROI {pick[i]}")


def test_plan_argument_checks(nat, ctx, cone):
    s, pos, cen, dirs, off, rel, w = cone
    plan = nat.SignaturePlan(ctx, 10, 100, len(s.directions), s.nbins, len(w))
    with pytest.raises(nat.AraulloError):
        plan.run(rel, off, s.radius, dirs, w, use_graph=False)      # n_roi above the plan capacity
    for bad in [(0, 256, 4, 1), (32, 300, 4, 1), (32, 8192, 4, 1), (32, 256, 0, 1), (32, 256, 4, 2)]:
        with pytest.raises(nat.AraulloError):
            plan.set_config(*bad)
