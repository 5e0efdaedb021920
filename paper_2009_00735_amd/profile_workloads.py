"""Single-stage workloads for profiling one kernel family under rocprofv3.

    python -m paper_2009_00735_amd.profile_workloads indexing [--reps 5]
    python -m paper_2009_00735_amd.profile_workloads indexing_two_phase [--reps 2]
    python -m paper_2009_00735_amd.profile_workloads signatures [--reps 5]
    python -m paper_2009_00735_amd.profile_workloads sparse [--reps 5]
    python -m paper_2009_00735_amd.profile_workloads fsp [--reps 5]

`indexing`: the config-2 indexing shape (2000 ROI images x 20000 references,
4 x 10242 nodes) on seeded random non-negative images generated on the
device; calls `index_orientations(k = 16)` `reps` times.

`indexing_two_phase`: the two-phase indexing shape (20000 ROI images x
100000 references, 4 x 10242 nodes), seeded random non-negative images
generated on the device; `index_orientations(k = 16)` `reps` times.

`signatures`: config 2 (2000 ROIs of about 1000 atoms, 10242 directions,
1024 bins): one ROI query, then the autotuned persistent signature plan
replayed `reps` times.

`sparse`: the config-2 sparse indexing shape: the fcc Al reference (mean
signature of 16 unrotated crystal ROIs), 20000 library orientations, 1000
strongest entries; the look-up table is built once, then
`index_orientations_sparse(k = 16)` runs `reps` times on seeded random
non-negative ROI images (2000 x 4 x 10242) generated on the device.

`fsp`: Eq. (2) on the 64^3 grid (k_max = 10/nm) for 10^4 ROIs of R = 2 nm in
full-density fcc Al (`synth.fsp_specimen`); `ar_fsp_amplitudes` runs `reps`
times into one output buffer.

Every call goes through the C ABI (`native`); nothing here computes any part
of the method.  Prints one line per repetition with the wall time.
"""
from __future__ import annotations

import argparse
import time

import torch

from . import native as nat
from . import synth


def _timed(label: str, fn, reps: int) -> None:
    for i in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        print(f"{label} rep {i}: {(time.perf_counter() - t0) * 1e3:.2f} ms", flush=True)


def indexing(reps: int) -> None:
    ctx = nat.Context(0)
    gen = torch.Generator(device="cuda").manual_seed(5)
    L = torch.rand((20000, 4, 10242), device="cuda", generator=gen) ** 2
    S = torch.rand((2000, 4, 10242), device="cuda", generator=gen) ** 2
    lib = nat.Library(ctx, L)
    _timed("index_orientations", lambda: nat.index_orientations(ctx, S, lib, 16), reps)


def indexing_two_phase(reps: int) -> None:
    ctx = nat.Context(0)
    gen = torch.Generator(device="cuda").manual_seed(6)
    L = torch.rand((100000, 4, 10242), device="cuda", generator=gen) ** 2
    S = torch.rand((20000, 4, 10242), device="cuda", generator=gen) ** 2
    lib = nat.Library(ctx, L)
    _timed("index_orientations", lambda: nat.index_orientations(ctx, S, lib, 16), reps)


def signatures(reps: int) -> None:
    ctx = nat.Context(0)
    s = synth.single_grain_box()
    w = nat.windows_for(s.radius, s.nbins, s.spacings)
    pos = torch.from_numpy(s.positions).cuda()
    cen = torch.from_numpy(s.centres).cuda()
    dirs = torch.from_numpy(s.directions).cuda()
    off, rel = nat.ar_roi_gather(ctx, pos, cen, s.radius)
    plan = nat.SignaturePlan(ctx, len(s.centres), rel.shape[0], len(s.directions), s.nbins, len(w))
    out = plan.tune(rel, off, s.radius, dirs, w)
    print("plan", plan.config(), flush=True)
    _timed("signature plan", lambda: plan.run(rel, off, s.radius, dirs, w, out=out, use_graph=True), reps)


def sparse(reps: int) -> None:
    ctx = nat.Context(0)
    s = synth.single_grain_box()
    w = nat.windows_for(s.radius, s.nbins, s.spacings)
    dirs = torch.from_numpy(s.directions).cuda()
    rpos, roffs = synth.reference_rois(0, 16, R=s.radius, cfg=4)
    ref = nat.araullo_signatures(ctx, torch.from_numpy(rpos).cuda(), torch.from_numpy(roffs).cuda(), s.radius, dirs,
                                 s.nbins, w, counts=False).mean(0, keepdim=True).contiguous()
    q = torch.from_numpy(synth.library_orientations(20000, 2)).cuda()
    lut = nat.SparseLUT(ctx, ref, dirs, q, [20000], 1000)
    gen = torch.Generator(device="cuda").manual_seed(6)
    S = torch.rand((2000, len(w), len(s.directions)), device="cuda", generator=gen) ** 2
    _timed("index_orientations_sparse", lambda: nat.index_orientations_sparse(ctx, S, lut, 16), reps)


def fsp(reps: int) -> None:
    ctx = nat.Context(0)
    pos, cen, _ = synth.fsp_specimen(10000, 2.0)
    off, rel = nat.ar_roi_gather(ctx, torch.from_numpy(pos).cuda(), torch.from_numpy(cen).cuda(), 2.0)
    rel = rel.contiguous()
    out = torch.empty((len(cen), 64, 64, 64), dtype=torch.float32, device="cuda")
    _timed("ar_fsp_amplitudes", lambda: nat.ar_fsp_amplitudes(ctx, rel, off, 64, 10.0, out=out), reps)


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload", choices=["indexing", "indexing_two_phase", "signatures", "sparse", "fsp"])
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    {"indexing": indexing, "indexing_two_phase": indexing_two_phase, "signatures": signatures, "sparse": sparse,
     "fsp": fsp}[a.workload](a.reps)


if __name__ == "__main__":
    main()
