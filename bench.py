#!/usr/bin/env python3
"""Benchmark of the real-space signature + orientation indexing hot path on
one MI355X, on the single-grain fcc Al workload (the benchmark
definition): a 20 x 20 x 40 nm box at 30 atoms/nm^3, sigma = 0.05 nm,
2000 ROIs of R = 2 nm on a 2 nm grid, 10242 icosphere directions, 1024 bins,
4 peak windows, indexed against 20000 rotated fcc references.

One step = the whole hot path over that batch, inputs resident in HBM:
  a1      ROI query (ar_roi_gather)
  a2-a5   Eq. (1) histograms + FFT + window maxima, persistent autotuned
          launch replayed as a HIP graph (ar_signature_plan_run)
  a6-a8   normalise + BF16 MFMA correlation + top-16 + FP32 rescore
          (index_orientations)
  a9      FP64 cubic disorientation of the top-1 against the ground truth
  a10     50-step structure-factor refinement of the top-1 orientation
          (ar_refine_orientations)

Prints one JSON line.  `--gpus N` with N > 1 exits: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12      # MI355X datasheet, FLOP/s (packed FP32 counted)
PEAK_BF16_DENSE = 2.5e15         # MI355X datasheet, FLOP/s dense
PEAK_HBM = 8.0e12                # B/s
F_AL = (4.2767, 4.9383, 6.9838, 8.1892)   # 1/d of fcc Al {111},{200},{220},{311}, nm^-1
F_FE = (4.9276, 6.9686, 8.5347, 9.8552)   # 1/d of bcc Fe {110},{200},{211},{220}, nm^-1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(profile: str, source: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        vals = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and l.split(": ", 1)[0] in
                    ("traffic_bytes_per_launch", "source_sha256"))
        sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
        if vals.get("source_sha256") != sha:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--refine-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config-legs", action="store_true",
                    help="skip the batched-polycrystal, two-phase indexing and 4096-ROI refinement legs")
    ap.add_argument("--leg-reps", type=int, default=3, help="timed repetitions of each config leg")
    ap.add_argument("--cpu-sample-rois", type=int, default=16)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB (scale factor for HBM counters)")
    ap.add_argument("--compare", action="store_true",
                    help="instead of the step: plain vs batched signatures (single-grain box, polycrystal cone) and BF16-MFMA vs "
                         "plain FP32 indexing on the same GPU; prints one JSON line")
    return ap.parse_args()


def cpu_info():
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return model


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path. "
              "ROIs would shard across GPUs with no exchange; a sharded library would need one all-gather of "
              "the per-GPU top-k candidates.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_00735_amd import native as nat
    from paper_2009_00735_amd import synth

    dev = torch.device("cuda", 0)
    if args.copy_probe:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}))
        return
    if args.compare:
        compare(nat, synth, torch, dev)
        return

    # ------------------------------------------------------------ setup (untimed)
    t_setup = time.perf_counter()
    s = synth.single_grain_box()
    n_roi, n_dir, nb, R = len(s.centres), len(s.directions), s.nbins, s.radius
    ctx = nat.Context(0)
    peaks = nat.ar_measure_peaks(ctx)      # measured roofline denominators (probe loops, ~1 s)
    pos = torch.from_numpy(s.positions).to(dev)
    cen = torch.from_numpy(s.centres).to(dev)
    dirs = torch.from_numpy(s.directions).to(dev)
    windows = nat.windows_for(R, nb, s.spacings)
    n_win = windows.shape[0]
    # reference (noise-free, unrotated fcc Al, 16 in-cell offsets) and library
    rpos, roffs = synth.reference_rois(0, 16, R=R, cfg=4)
    rpos_d, roffs_d = torch.from_numpy(rpos).to(dev), torch.from_numpy(roffs).to(dev)
    ref = nat.araullo_signatures(ctx, rpos_d, roffs_d, R, dirs, nb, windows, counts=False).mean(0, keepdim=True)
    n_lib = 20000
    lib_q = synth.library_orientations(n_lib, 2)
    lib_q_d = torch.from_numpy(lib_q).to(dev)
    L = nat.ar_rotate_reference(ctx, ref.contiguous(), dirs, lib_q_d, torch.zeros(n_lib, dtype=torch.int32, device=dev))
    lib = nat.Library(ctx, L)
    # structure-factor target: amplitudes of the reference ROIs at identity
    ident = torch.tensor([[1.0, 0, 0, 0]], device=dev).repeat(len(roffs), 1).contiguous()
    roff_csr, rrel = nat.ar_roi_gather(ctx, rpos_d, roffs_d, R)
    freqs = torch.tensor([F_AL], dtype=torch.float32, device=dev)
    T = nat.ar_sf_amplitudes(ctx, rrel.contiguous(), roff_csr, ident, torch.zeros(len(roffs), dtype=torch.int32,
                                                                                   device=dev), dirs, freqs)
    T = T.mean(0, keepdim=True).contiguous()
    truth_q = torch.from_numpy(s.truth_q).to(dev)
    phase = torch.zeros(n_roi, dtype=torch.int32, device=dev)
    # gather buffers and the signature plan (autotuned once)
    off_buf = torch.empty(n_roi + 1, dtype=torch.int64, device=dev)
    off_buf, rel0 = nat.ar_roi_gather(ctx, pos, cen, R)
    total = rel0.shape[0]
    rel_buf = torch.empty((int(total * 1.05) + 64, 4), dtype=torch.float32, device=dev)
    images = torch.empty((n_roi, n_win, n_dir), dtype=torch.float32, device=dev)
    plan = nat.SignaturePlan(ctx, n_roi, rel_buf.shape[0], n_dir, nb, n_win)
    _, rel = nat.ar_roi_gather(ctx, pos, cen, R, out=(off_buf, rel_buf))
    plan.tune(rel, off_buf, R, dirs, windows, out=images)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    log(f"setup {t_setup:.1f} s: {n_roi} ROIs, {total} gathered atoms, library {n_lib}, plan {plan.config()}")

    stream = torch.cuda.current_stream(dev)
    ev = {}

    def mark(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        ev.setdefault(name, []).append(e)

    out = {}

    def step():
        mark("a1")
        _, rel = nat.ar_roi_gather(ctx, pos, cen, R, out=(off_buf, rel_buf))
        mark("a2_a5")
        plan.run(rel, off_buf, R, dirs, windows, out=images, use_graph=True)
        mark("a6_a8")
        idx, score = nat.index_orientations(ctx, images, lib, 16)
        mark("a9")
        top_q = lib_q_d[idx[:, 0].long()].contiguous()
        dis = nat.ar_disorientation_cubic(top_q, truth_q)
        mark("a10")
        q = top_q.float().contiguous()
        nat.ar_refine_orientations(ctx, rel, off_buf, q, phase, dirs, freqs, T, args.refine_steps, 0.01)
        dis_ref = nat.ar_disorientation_cubic(q.double().contiguous(), truth_q)
        mark("end")
        out.update(idx=idx, score=score, dis=dis, dis_ref=dis_ref, q=q)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps

    names = ["a1", "a2_a5", "a6_a8", "a9", "a10", "end"]
    stage_ms = {}
    for a, b in zip(names[:-1], names[1:]):
        stage_ms[a] = float(np.mean([x.elapsed_time(y) for x, y in zip(ev[a], ev[b])]))
    log("stage ms:", json.dumps({k: round(v, 3) for k, v in stage_ms.items()}))

    dis = out["dis"].cpu().numpy()
    dis_ref = out["dis_ref"].cpu().numpy()
    counts = torch.diff(off_buf).cpu().numpy()
    n_w_mean = float(counts.mean())

    # ------------------------------------------------------------ rooflines
    # a10 adjoint (dominant).  Unit: one (atom, evaluated direction,
    # frequency) term; antipodal mesh directions share one evaluation, so
    # n_eval = n_dir / 2 for the icosphere.  Algorithmic FP32 arithmetic per
    # term (FMA = 2 flops): phase 1 + C,S accumulation 2 + P,Q accumulation
    # 6 FMA = 12, plus the shared dot product 5/n_freq; the sine and cosine
    # (2 per term) run on the transcendental unit and are reported against
    # its measured rate, not counted as flops.  Bound: FP32 vector ALU, peak
    # 157.3 TFLOP/s.
    n_freq = len(F_AL)
    n_eval = evaluated_directions(s.directions)
    # The refinement makes refine_steps adjoint evaluations and a last,
    # score-only one (forward kernel: dot product, phase, sin/cos, C and S =
    # 5 + 5/n_freq per term); the stage time holds all of them.
    terms_eval = float(counts.sum()) * n_eval * n_freq
    evals = args.refine_steps + 1
    a10_s = stage_ms["a10"] / 1e3
    flop_per_term = sf_flop_per_term(n_freq, True)
    flop_per_term_score = sf_flop_per_term(n_freq, False)
    achieved_terms = terms_eval * evals / a10_s
    achieved_flops = terms_eval * (args.refine_steps * flop_per_term + flop_per_term_score) / a10_s
    roofline = {
        "kernel": "k_sf<1,4> (structure-factor adjoint, a10)",
        "bound": "alu",
        "achieved": achieved_flops / 1e12,
        "peak": PEAK_FP32_VECTOR / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved_flops / PEAK_FP32_VECTOR,
        "traffic": measured_traffic("k_sf_adjoint_single_grain_hbm_counters.md", "paper_2009_00735_amd/csrc/refine.hip"),
        "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-probe scaled)",
        "terms_per_s": achieved_terms,
        "evaluated_directions": n_eval,
        "flop_per_term": {"adjoint": flop_per_term, "score_only": flop_per_term_score},
        "frac_of_measured_fp32_fma": achieved_flops / peaks["fp32_fma_flop_per_s"],
        "transcendentals_per_s": 2.0 * achieved_terms,
        "frac_of_measured_sin": 2.0 * achieved_terms / peaks["sin_per_s"],
    }
    # signatures (a2-a5), unit = one ROI x direction, against the measured
    # peaks of the three units the kernel uses:
    #   FP32 flops: 7 N_w (Eq. (1)) + 2.5 N_b log2 N_b (real FFT, the paper's
    #     cost model).  The kernel forms the last FFT stage only for the window
    #     bins, so it executes fewer: 7 N_w + 5 N_c log2 NS + per window bin
    #     two (R-1)-term complex sums (8 flops each) + 20 for |X_k|;
    #   LDS atomics: N_w;
    #   LDS bytes: 12 N_w atom reads, 4 N_b zeroing, 4 N_b histogram read,
    #     (2P - 1) 4 N_b for the P passes before the last stage (writes and
    #     reads of N_b/2 complex), 16 R per window bin for the last stage.
    # frac = max over the units of achieved rate / measured peak.
    sig_s = stage_ms["a2_a5"] / 1e3
    units = float(n_roi * n_dir)
    nc = nb // 2
    ns_last = 1
    while nc // ns_last > 8:
        ns_last *= 8
    r_last = nc // ns_last
    passes = int(round(math.log(ns_last, 8)))
    n_bins_win = int(windows[:, 1].max() - windows[:, 0].min() + 1)
    flop_full = 7.0 * n_w_mean + 2.5 * nb * math.log2(nb)
    flop_pruned = 7.0 * n_w_mean + 5.0 * nc * math.log2(ns_last) + n_bins_win * (16.0 * (r_last - 1) + 20.0)
    lds_bytes = 12.0 * n_w_mean + 8.0 * nb + (2 * passes - 1) * 4.0 * nb + 16.0 * r_last * n_bins_win
    fr = {
        "fp32_flops_full_fft": flop_full * units / sig_s / peaks["fp32_fma_flop_per_s"],
        "fp32_flops_executed": flop_pruned * units / sig_s / peaks["fp32_fma_flop_per_s"],
        "lds_atomics": n_w_mean * units / sig_s / peaks["lds_atomics_per_s"],
        "lds_bytes": lds_bytes * units / sig_s / peaks["lds_bytes_per_s"],
    }
    bound = max(fr, key=fr.get)
    roof_sig = {"kernel": "k_signatures_persistent<10,*> (a2-a5)", "bound": bound, "frac": fr[bound],
                "frac_by_unit": fr, "peaks": "measured (ar_measure_peaks)",
                "per_roi_direction": {"flop_full_fft": flop_full, "flop_executed": flop_pruned,
                                      "lds_atomics": n_w_mean, "lds_bytes": lds_bytes},
                "achieved_tflops_full_fft": flop_full * units / sig_s / 1e12,
                "frac_of_published_fp32": flop_full * units / sig_s / PEAK_FP32_VECTOR,
                "hbm_gbps": (16.0 * counts.sum() + 4.0 * n_roi * n_win * n_dir) / sig_s / 1e9}
    Kp = lib.n_win * lib.n_dir
    Kp = (Kp + 63) // 64 * 64
    gemm_flops = 2.0 * ((n_roi + 127) // 128 * 128) * ((n_lib + 127) // 128 * 128) * Kp
    roof_idx = {"kernel": "index_orientations (a6-a8, BF16 MFMA correlation + rescore)", "bound": "mfma",
                "achieved": gemm_flops / (stage_ms["a6_a8"] / 1e3) / 1e12, "peak": PEAK_BF16_DENSE / 1e12,
                "unit": "TFLOP/s", "frac": gemm_flops / (stage_ms["a6_a8"] / 1e3) / PEAK_BF16_DENSE,
                "frac_of_measured_mfma": gemm_flops / (stage_ms["a6_a8"] / 1e3) / peaks["bf16_mfma_flop_per_s"]}

    rec = {
        "metric": "ROI·direction signatures/s + indexed ROIs/s at fixed top-1 disorientation",
        "value": n_roi * n_dir / (ms_step / 1e3),
        "unit": "ROI·direction/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single-grain fcc Al box 20x20x40 nm, 30 atoms/nm^3, sigma 0.05 nm; "
                               "2000 ROIs R=2 nm; 10242 directions; 1024 bins; 4 windows; "
                               "20000-orientation library; 50-step refinement",
                   "n_roi": n_roi, "n_dir": n_dir, "nbins": nb, "n_win": n_win, "n_lib": n_lib,
                   "mean_atoms_per_roi": n_w_mean, "refine_steps": args.refine_steps,
                   "signature_plan": dict(zip(["dirs_per_item", "atoms_per_stage", "blocks_per_cu", "min_waves"],
                                             plan.config()))},
        "indexed_rois_per_s": n_roi / (ms_step / 1e3),
        "stage_ms": stage_ms,
        "stage_rates": {
            "signatures_roi_dir_per_s": n_roi * n_dir / (stage_ms["a1"] / 1e3 + sig_s),
            "indexing_rois_per_s": n_roi / (stage_ms["a6_a8"] / 1e3),
            "refine_roi_steps_per_s": n_roi * args.refine_steps / a10_s,
        },
        "accuracy": {
            "top1_disorientation_deg": {"median": float(np.median(dis)), "p95": float(np.percentile(dis, 95))},
            "refined_disorientation_deg": {"median": float(np.median(dis_ref)),
                                           "p95": float(np.percentile(dis_ref, 95))},
        },
        "roofline": roofline,
        "roofline_signatures": roof_sig,
        "measured_peaks": peaks,
        "roofline_indexing": roof_idx,
    }

    # ------------------------------------------------------------ CPU oracle baseline
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(s, windows.numpy(), L, lib_q, ref, T, args, n_lib)
    if not args.no_config_legs:
        del plan, images, rel_buf, L, lib
        torch.cuda.empty_cache()
        rec["config_legs"] = config_legs(nat, synth, torch, dev, ctx, peaks, args)
    print(json.dumps(rec), flush=True)


def evaluated_directions(directions) -> int:
    """Directions the structure-factor kernels evaluate: an exact antipodal
    pair shares one evaluation (|F(-u)| = |F(u)|)."""
    key = {tuple(v): i for i, v in enumerate(directions.tolist())}
    n = 0
    for i, v in enumerate(directions.tolist()):
        m = key.get(tuple(-x for x in v), -1)
        n += 1 if (m < 0 or m > i) else 0
    return n


def sf_flop_per_term(n_freq: int, adjoint: bool) -> float:
    """FP32 arithmetic per (atom, evaluated direction, frequency) term of the
    structure-factor kernels (FMA = 2): phase 1, C and S 2, the shared dot
    product 5 / n_freq, and with the adjoint the P and Q sums 6 FMA."""
    return 1.0 + 2.0 + 5.0 / n_freq + (12.0 if adjoint else 0.0)


def signature_flops(n_w: float, nb: int) -> float:
    """FP32 flops per ROI x direction in the paper's cost model: 7 N_w for
    Eq. (1) and 2.5 N_b log2 N_b for the real FFT."""
    return 7.0 * n_w + 2.5 * nb * math.log2(nb)


def event_ms(torch, fn, reps: int):
    """Mean milliseconds of fn() over reps, HIP events on the current stream
    (one untimed call first)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def config_legs(nat, synth, torch, dev, ctx, peaks, args):
    """The other benchmark workloads at full size, each timed with HIP events
    over `leg_reps` repetitions after one untimed call, with its roofline and
    the oracle timed beside it on a bounded sample:
      batched_polycrystal  8000 surface-clipped ROIs (100..1500 atoms) of the
                           fcc Al / bcc Fe cone, 10242 directions, 1024 bins:
                           the autotuned persistent plan replayed as a graph;
      two_phase_indexing   20000 polycrystal ROI images x 2 phases x 50000
                           rotated references (K = 4 x 10242), BF16 MFMA +
                           top-16 + FP32 rescore; accuracy against the
                           synthetic truth and the top-1 against the FP64
                           oracle over the whole library on sampled ROIs;
      refinement_4096      4096 polycrystal ROIs of 800..1200 atoms, 50
                           structure-factor steps from the two-phase top-1."""
    from oracle import oracle as orc
    threads = orc.default_threads()
    reps = args.leg_reps
    legs = {}
    R, NB = 2.0, 1024
    freqs = torch.tensor([F_AL, F_FE], dtype=torch.float32, device=dev)

    # ---------------------------------------------------------- batched polycrystal
    t_set = time.perf_counter()
    s3 = synth.polycrystal_cone()
    pos = torch.from_numpy(s3.positions).to(dev)
    dirs = torch.from_numpy(s3.directions).to(dev)
    w = nat.windows_for(R, NB, s3.spacings)
    n_win, n_dir = w.shape[0], dirs.shape[0]
    off3, rel3 = nat.ar_roi_gather(ctx, pos, torch.from_numpy(s3.centres).to(dev), R)
    rel3 = rel3.contiguous()
    plan = nat.SignaturePlan(ctx, len(s3.centres), rel3.shape[0], n_dir, NB, n_win)
    img3 = plan.tune(rel3, off3, R, dirs, w)
    torch.cuda.synchronize()
    log(f"leg batched_polycrystal: setup {time.perf_counter() - t_set:.1f} s, plan {plan.config()}")
    ms = event_ms(torch, lambda: plan.run(rel3, off3, R, dirs, w, out=img3, use_graph=True), reps)
    counts3 = torch.diff(off3).cpu().numpy()
    units = len(s3.centres) * n_dir
    flop = signature_flops(float(counts3.mean()), NB)
    t0 = time.perf_counter()
    sel = np.linspace(0, len(s3.centres) - 1, 4).astype(int)
    orc.signatures(s3.positions, s3.centres[sel], R, s3.directions, NB, w.numpy(), threads)
    t_o = time.perf_counter() - t0
    legs["batched_polycrystal"] = {
        "workload": "20-grain fcc Al / bcc Fe truncated cone (60 nm, top radius 15 nm), 8000 surface-clipped ROIs "
                    "R = 2 nm, 10242 directions, 1024 bins, persistent plan replayed as a HIP graph",
        "value": units / (ms / 1e3), "unit": "ROI·direction/s", "ms": ms,
        "atoms_min": int(counts3.min()), "atoms_max": int(counts3.max()), "atoms_mean": float(counts3.mean()),
        "plan": dict(zip(["dirs_per_item", "atoms_per_stage", "blocks_per_cu", "min_waves"], plan.config())),
        "roofline": {"bound": "fp32_flops_full_fft", "achieved": flop * units / (ms / 1e3) / 1e12,
                     "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                     "frac": flop * units / (ms / 1e3) / PEAK_FP32_VECTOR,
                     "frac_of_measured_fp32_fma": flop * units / (ms / 1e3) / peaks["fp32_fma_flop_per_s"],
                     "flop_per_roi_direction": flop},
        "cpu_baseline": {"value": len(sel) * n_dir / t_o, "unit": "ROI·direction/s", "cores": threads,
                         "kind": "oracle", "sample": f"{len(sel)} of 8000 ROIs, all 10242 directions, {t_o:.1f} s"}}
    del plan, img3, rel3, off3
    log("leg batched_polycrystal done")

    # ---------------------------------------------------------- two-phase indexing
    t_set = time.perf_counter()
    centres, dom, share, _ = synth.polycrystal_rois(20000)
    S = nat.araullo_signatures(ctx, pos, torch.from_numpy(centres).to(dev), R, dirs, NB, w, counts=False)
    refs = []
    for ph in (0, 1):
        rpos, roffs = synth.reference_rois(ph, 16, R=R, cfg=4)
        refs.append(nat.araullo_signatures(ctx, torch.from_numpy(rpos).to(dev), torch.from_numpy(roffs).to(dev), R,
                                           dirs, NB, w, counts=False).mean(0))
    ref = torch.stack(refs).contiguous()
    n_per = 50000
    libq = synth.library_orientations(2 * n_per, 4)
    libph = np.repeat(np.arange(2, dtype=np.int32), n_per)
    libq_d, libph_d = torch.from_numpy(libq).to(dev), torch.from_numpy(libph).to(dev)
    L = nat.ar_rotate_reference(ctx, ref, dirs, libq_d, libph_d)
    lib = nat.Library(ctx, L, libq_d, libph_d)
    torch.cuda.synchronize()
    log(f"leg two_phase_indexing: setup {time.perf_counter() - t_set:.1f} s")
    res = {}

    def index():
        res["idx"], res["score"] = nat.index_orientations(ctx, S, lib, 16)
    ms = event_ms(torch, index, reps)
    top = res["idx"][:, 0].contiguous()
    tq, tph = lib.lookup(top)
    dis = nat.ar_disorientation_cubic(tq, torch.from_numpy(s3.grain_q[dom]).to(dev)).cpu().numpy()
    tph = tph.cpu().numpy()
    good = share >= 0.9
    phase_ok = tph == s3.grain_phase[dom]
    m = good & phase_ok
    # CPU baseline of this leg: the FP64 oracle over the whole library for
    # sampled ROIs (host copies excluded from its time); its result also
    # tells whether the GPU top-1 is the oracle's or a tie
    n_chk = 4
    chk = np.sort(np.random.default_rng(41).choice(len(centres), n_chk, replace=False))
    t_o = 0.0
    t0 = time.perf_counter()
    Sh = orc.normalise(S[torch.as_tensor(chk, device=dev)].cpu().numpy())
    t_o += time.perf_counter() - t0
    best_i = np.zeros((n_chk, 0), np.int64)
    best_s = np.zeros((n_chk, 0))
    chunk = 10000
    for c0 in range(0, L.shape[0], chunk):
        Lc = L[c0:c0 + chunk].cpu().numpy()
        t0 = time.perf_counter()
        i, sc = orc.index_topk(Sh, orc.normalise(Lc), 1, threads)
        t_o += time.perf_counter() - t0
        best_i = np.concatenate([best_i, i.astype(np.int64) + c0], axis=1)
        best_s = np.concatenate([best_s, sc], axis=1)
    o = np.lexsort((best_i, best_s), axis=1)[:, 0]
    o_i, o_s = best_i[np.arange(n_chk), o], best_s[np.arange(n_chk), o]
    g_i = res["idx"][torch.as_tensor(chk, device=dev), 0].cpu().numpy()
    same = int(np.sum(g_i == o_i))
    ties = 0
    for a in range(n_chk):
        if g_i[a] != o_i[a]:
            d = orc.ssd_pairs(Sh[a:a + 1], orc.normalise(L[int(g_i[a])][None].cpu().numpy()), [0], [0])[0]
            ties += int(d - o_s[a] <= 1e-5 * o_s[a] + 1e-6)
    Kp = (n_win * n_dir + 63) // 64 * 64
    gemm = 2.0 * ((len(centres) + 255) // 256 * 256) * ((2 * n_per + 255) // 256 * 256) * Kp
    legs["two_phase_indexing"] = {
        "workload": "20000 polycrystal ROI images x 2 phases x 50000 Shoemake references, K = 4 x 10242, "
                    "BF16 MFMA correlation, top-16, FP32 rescore",
        "value": len(centres) / (ms / 1e3), "unit": "indexed ROIs/s", "ms": ms,
        "accuracy": {"rois_share_ge_0.9": int(good.sum()), "phase_correct": float(phase_ok[good].mean()),
                     "top1_disorientation_deg": {"median": float(np.median(dis[m])),
                                                 "p95": float(np.percentile(dis[m], 95))}},
        "fp64_oracle_check": {"rois": n_chk, "references": int(L.shape[0]), "top1_identical": same,
                              "top1_ties": ties, "top1_other": n_chk - same - ties},
        "roofline": {"bound": "mfma", "achieved": gemm / (ms / 1e3) / 1e12, "peak": PEAK_BF16_DENSE / 1e12,
                     "unit": "TFLOP/s", "frac": gemm / (ms / 1e3) / PEAK_BF16_DENSE,
                     "frac_of_measured_mfma": gemm / (ms / 1e3) / peaks["bf16_mfma_flop_per_s"],
                     "gemm_flop": gemm},
        "cpu_baseline": {"value": n_chk / t_o, "unit": "indexed ROIs/s", "cores": threads, "kind": "oracle",
                         "sample": f"{n_chk} ROIs, FP64 normalise + Eq. S1 against all 100000 references, "
                                   f"{t_o:.1f} s (device-to-host copies excluded)"}}
    log("leg two_phase_indexing done")

    # ---------------------------------------------------------- refinement
    t_set = time.perf_counter()
    rc, rqt, rpht, _ = synth.refinement_rois(4096)
    offr, relr = nat.ar_roi_gather(ctx, pos, torch.from_numpy(rc).to(dev), R)
    relr = relr.contiguous()
    Sr = nat.araullo_signatures_csr(ctx, relr, offr, R, dirs, NB, w)
    ridx, _ = nat.index_orientations(ctx, Sr, lib, 1)
    q0, ph0 = lib.lookup(ridx[:, 0].contiguous())
    q0 = q0.float().contiguous()
    T = []
    ident = torch.tensor([[1.0, 0, 0, 0]], device=dev).repeat(16, 1).contiguous()
    for ph in (0, 1):
        rpos, roffs = synth.reference_rois(ph, 16, R=R, cfg=4)
        ro, rr = nat.ar_roi_gather(ctx, torch.from_numpy(rpos).to(dev), torch.from_numpy(roffs).to(dev), R)
        zf = torch.full((16,), ph, dtype=torch.int32, device=dev)
        T.append(nat.ar_sf_amplitudes(ctx, rr.contiguous(), ro, ident, zf, dirs, freqs).mean(0))
    T = torch.stack(T).contiguous()
    del S, L, lib
    torch.cuda.empty_cache()
    q = q0.clone()
    torch.cuda.synchronize()
    log(f"leg refinement_4096: setup {time.perf_counter() - t_set:.1f} s")

    def refine():
        q.copy_(q0)
        nat.ar_refine_orientations(ctx, relr, offr, q, ph0, dirs, freqs, T, args.refine_steps, 0.01)
    ms = event_ms(torch, refine, max(1, reps - 1))
    countsr = torch.diff(offr).cpu().numpy()
    terms = float(countsr.sum()) * evaluated_directions(s3.directions) * len(F_AL)
    flop = terms * (args.refine_steps * sf_flop_per_term(4, True) + sf_flop_per_term(4, False))
    ok = ph0.cpu().numpy() == rpht
    rqt_d = torch.from_numpy(rqt).to(dev)
    d0 = nat.ar_disorientation_cubic(q0.double().contiguous(), rqt_d).cpu().numpy()[ok]
    d1 = nat.ar_disorientation_cubic(q.double().contiguous(), rqt_d).cpu().numpy()[ok]
    # oracle: FP64 finite-difference refinement, one iteration per ROI, one ROI per thread
    import concurrent.futures as cf
    n_o = threads
    sub = np.linspace(0, len(rc) - 1, n_o).astype(int)
    rels = [orc.roi_gather(s3.positions, rc[i], R) for i in sub]
    qs = q0.double().cpu().numpy()[sub]
    phs = ph0.cpu().numpy()[sub]
    Tn = T.double().cpu().numpy()
    fr = np.array([F_AL, F_FE])
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda a: orc.sf_refine(rels[a], qs[a], s3.directions, fr[phs[a]], Tn[phs[a]], steps=1),
                    range(n_o)))
    t_o = time.perf_counter() - t0
    legs["refinement_4096"] = {
        "workload": "4096 polycrystal ROIs of 800..1200 atoms (dominant-grain share >= 0.9), structure-factor "
                    "score at 4 frequencies per phase x 10242 directions, 50 steps from the two-phase top-1",
        "value": len(rc) * args.refine_steps / (ms / 1e3), "unit": "ROI-steps/s", "ms": ms,
        "accuracy": {"phase_correct": float(ok.mean()),
                     "top1_disorientation_deg": {"median": float(np.median(d0)), "p95": float(np.percentile(d0, 95))},
                     "refined_disorientation_deg": {"median": float(np.median(d1)),
                                                    "p95": float(np.percentile(d1, 95))}},
        "roofline": {"bound": "alu", "achieved": flop / (ms / 1e3) / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": flop / (ms / 1e3) / PEAK_FP32_VECTOR,
                     "frac_of_measured_fp32_fma": flop / (ms / 1e3) / peaks["fp32_fma_flop_per_s"],
                     "transcendentals_per_s": 2.0 * terms * (args.refine_steps + 1) / (ms / 1e3),
                     "frac_of_measured_sin": 2.0 * terms * (args.refine_steps + 1) / (ms / 1e3) / peaks["sin_per_s"]},
        "cpu_baseline": {"value": n_o / t_o, "unit": "ROI-steps/s", "cores": threads, "kind": "oracle",
                         "sample": f"{n_o} ROIs x 1 FP64 finite-difference step (one ROI per thread), {t_o:.1f} s"}}
    log("leg refinement_4096 done")
    return legs


def compare(nat, synth, torch, dev):
    """The batched and BF16 forms against the plain method on the same GPU.
    Signatures: the plain per-launch kernel (one workgroup per ROI and
    256-direction tile) against the autotuned persistent plan replayed as a
    graph, on the single-grain box (even ROIs) and the polycrystal cone (uneven,
    surface-clipped);
    the images must be bit-identical.  Indexing: the BF16 MFMA correlation
    with fused top-16 and FP32 rescore against a plain FP32 evaluation of the
    same dense score (library GEMM in FP32 through torch, then top-16) on the
    single-grain images and 20000-reference library; reported: times and top-1
    agreement."""
    def best_ms(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    ctx = nat.Context(0)
    rec = {"compare": "plain vs batched signatures; BF16 MFMA + FP32 rescore vs plain FP32 indexing"}
    for name, s in (("single_grain", synth.single_grain_box()), ("polycrystal", synth.polycrystal_cone())):
        w = nat.windows_for(s.radius, s.nbins, s.spacings)
        pos = torch.from_numpy(s.positions).to(dev)
        cen = torch.from_numpy(s.centres).to(dev)
        dirs = torch.from_numpy(s.directions).to(dev)
        off, rel = nat.ar_roi_gather(ctx, pos, cen, s.radius)
        plain = nat.araullo_signatures_csr(ctx, rel, off, s.radius, dirs, s.nbins, w)
        t_plain = best_ms(lambda: nat.araullo_signatures_csr(ctx, rel, off, s.radius, dirs, s.nbins, w, out=plain))
        plan = nat.SignaturePlan(ctx, len(s.centres), rel.shape[0], len(s.directions), s.nbins, len(w))
        out = plan.tune(rel, off, s.radius, dirs, w)
        t_plan = best_ms(lambda: plan.run(rel, off, s.radius, dirs, w, out=out, use_graph=True))
        units = len(s.centres) * len(s.directions)
        counts = torch.diff(off).cpu().numpy()
        rec[f"signatures_{name}"] = {
            "rois": len(s.centres), "atoms_min": int(counts.min()), "atoms_max": int(counts.max()),
            "plain_ms": t_plain, "batched_ms": t_plan, "speedup": t_plain / t_plan,
            "batched_roi_dir_per_s": units / (t_plan / 1e3), "identical": bool(torch.equal(out, plain)),
            "plan": dict(zip(["dirs_per_item", "atoms_per_stage", "blocks_per_cu", "min_waves"], plan.config()))}
        if name == "single_grain":
            images = out.clone()
            rpos, roffs = synth.reference_rois(0, 16, R=s.radius, cfg=4)
            ref = nat.araullo_signatures(ctx, torch.from_numpy(rpos).to(dev), torch.from_numpy(roffs).to(dev),
                                         s.radius, dirs, s.nbins, w, counts=False).mean(0, keepdim=True)
            lib_q = torch.from_numpy(synth.library_orientations(20000, 2)).to(dev)
            L = nat.ar_rotate_reference(ctx, ref.contiguous(), dirs, lib_q,
                                        torch.zeros(20000, dtype=torch.int32, device=dev))
        del plain, out, plan
    log("compare: signatures done")
    lib = nat.Library(ctx, L)
    t_bf16 = best_ms(lambda: nat.index_orientations(ctx, images, lib, 16))
    idx_bf16, _ = nat.index_orientations(ctx, images, lib, 16)

    def plain_fp32():
        Sh = (images / images.amax(dim=2, keepdim=True).clamp_min(1e-30)).reshape(len(images), -1)
        Lh = (L / L.amax(dim=2, keepdim=True).clamp_min(1e-30)).reshape(len(L), -1)
        d = (Lh * Lh).sum(1)[None, :] - 2.0 * (Sh @ Lh.T)
        return torch.topk(d, 16, dim=1, largest=False).indices
    t_fp32 = best_ms(plain_fp32)
    idx_fp32 = plain_fp32()
    agree = float((idx_fp32[:, 0] == idx_bf16[:, 0].long()).float().mean())
    rec["indexing_single_grain"] = {
        "rois": int(images.shape[0]), "references": int(L.shape[0]), "k": 16,
        "bf16_mfma_rescored_ms": t_bf16, "plain_fp32_ms": t_fp32, "speedup": t_fp32 / t_bf16,
        "top1_agreement": agree,
        "plain_fp32": "normalise, FP32 GEMM S L^T (torch / hipBLASLt), |L|^2 - 2 S.L, torch.topk"}
    # the paper's sparse form of Eq. S1 (strongest reference entries through a
    # look-up table) against the dense score, same images and orientations
    truth = torch.from_numpy(synth.single_grain_box().truth_q).to(dev)
    n_rot = lib_q.shape[0]
    dis_dense = nat.ar_disorientation_cubic(lib_q[idx_bf16[:, 0].long()].contiguous(), truth).cpu().numpy()
    sparse = {"rois": int(images.shape[0]), "orientations": n_rot, "k": 16,
              "dense_ms": t_bf16, "dense_top1_disorientation_median_deg": float(np.median(dis_dense))}
    peaks = nat.ar_measure_peaks(ctx)
    sparse["measured_lds_gather8_per_s"] = peaks["lds_gather8_per_s"]
    for n_hat in (250, 1000, 4000):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lut = nat.SparseLUT(ctx, ref.contiguous(), dirs, lib_q, [n_rot], n_hat)
        torch.cuda.synchronize()
        t_lut = (time.perf_counter() - t0) * 1e3
        rb = lut.screen
        sparse["screen_rois_per_lds_read"] = rb
        t_sp = best_ms(lambda: nat.index_orientations_sparse(ctx, images, lut, 16))
        idx_sp, _ = nat.index_orientations_sparse(ctx, images, lut, 16)
        dis_sp = nat.ar_disorientation_cubic(lib_q[idx_sp[:, 0].long()].contiguous(), truth).cpu().numpy()
        log(f"compare: sparse indexing N^ = {n_hat}")
        sparse[f"n_hat_{n_hat}"] = {
            "lut_build_ms": t_lut, "index_ms": t_sp, "speedup_vs_dense": t_bf16 / t_sp,
            "terms_per_s": images.shape[0] * n_rot * n_hat / (t_sp / 1e3),
            # whole call (screen + rescore + normalise) against random LDS reads:
            # one 8-byte read serves rb ROI terms
            "lds_gather_frac": images.shape[0] * n_rot * n_hat / rb / (t_sp / 1e3) / peaks["lds_gather8_per_s"],
            "top1_same_as_dense": float((idx_sp[:, 0] == idx_bf16[:, 0]).float().mean()),
            "top1_disorientation_median_deg": float(np.median(dis_sp)),
            "top1_disorientation_p95_deg": float(np.percentile(dis_sp, 95))}
        del lut
    # the oracle beside it, on a bounded sample: strongest entries and the
    # look-up rows of 400 orientations (N^ = 1000), then Eq. S1 for 16 ROIs
    # against those orientations; rates extrapolate per unit of work
    from oracle import oracle as orc
    threads = orc.default_threads()
    t0 = time.perf_counter()
    osi, osv = orc.sparse_strong(ref.cpu().numpy(), 1000)
    sub = np.linspace(0, n_rot - 1, 400).astype(int)
    qs = lib_q.cpu().numpy()[sub]
    olut = orc.sparse_lut(qs, np.zeros(len(sub), np.int32), osi, dirs.cpu().numpy(), threads)
    t_olut = time.perf_counter() - t0
    Sh16 = orc.normalise(images[:16].cpu().numpy())
    t0 = time.perf_counter()
    orc.sparse_index_topk(Sh16, osi, osv, np.zeros(len(sub), np.int32), olut, 16, threads)
    t_oidx = time.perf_counter() - t0
    sparse["cpu_oracle"] = {
        "kind": "oracle", "cores": threads,
        "sample": "N^ = 1000: strongest entries + look-up rows of 400 of the 20000 orientations; Eq. S1 (FP64) "
                  "for 16 ROIs against those 400",
        "lut_rows_per_s": len(sub) / t_olut, "terms_per_s": 16 * len(sub) * 1000 / t_oidx,
        "full_call_estimate_s": 2000 * n_rot * 1000 / (16 * len(sub) * 1000 / t_oidx)}
    rec["sparse_indexing_single_grain"] = sparse
    log("compare: indexing done")
    # sub-lattice signatures: an L1_2 Al3Sc crystal (eta 0.5, sigma 0.03 nm),
    # 2000 ROIs of R = 2 nm, 10242 directions, 1024 bins, the four windows plus
    # the superlattice window at d = a; channels: all atoms, Al, Sc
    pos, types, cen, _ = synth.l12_specimen(n_roi=2000, R=2.0, seed=1)
    a = synth.A_AL3SC
    w5 = nat.windows_for(2.0, 1024, [(0.9 * a, 1.1 * a)] + list(synth.window_spacings()))
    pos_d, types_d, cen_d = (torch.from_numpy(pos).to(dev), torch.from_numpy(types).to(dev),
                             torch.from_numpy(cen).to(dev))
    masks = [(1 << 64) - 1, 1 << synth.TYPE_AL, 1 << synth.TYPE_MINOR]
    t_typed = best_ms(lambda: nat.araullo_signatures_typed(ctx, pos_d, types_d, cen_d, 2.0, dirs, 1024, w5, masks,
                                                           counts=False))
    t_untyped = best_ms(lambda: nat.araullo_signatures(ctx, pos_d, cen_d, 2.0, dirs, 1024, w5, counts=False))
    _, cnt = nat.araullo_signatures_typed(ctx, pos_d, types_d, cen_d, 2.0, dirs, 1024, w5, masks)
    cnt = cnt.float().mean(0).cpu().numpy()
    rec["typed_signatures_l12"] = {
        "rois": len(cen), "directions": int(dirs.shape[0]), "nbins": 1024, "windows": int(w5.shape[0]),
        "channels": ["all", "Al", "Sc"], "mean_atoms_per_channel": [float(x) for x in cnt],
        "typed_ms": t_typed, "untyped_ms": t_untyped, "typed_over_untyped": t_typed / t_untyped,
        "roi_dir_channel_per_s": len(cen) * int(dirs.shape[0]) * 3 / (t_typed / 1e3),
        "note": "each channel = one typed ROI query + the plain signature kernel + a pitched copy"}
    t0 = time.perf_counter()
    orc.signatures_typed(pos, types, masks, cen[:2], 2.0, dirs.cpu().numpy(), 1024, w5.numpy(), threads)
    t_ot = time.perf_counter() - t0
    rec["typed_signatures_l12"]["cpu_oracle"] = {
        "kind": "oracle", "cores": threads, "sample": "2 ROIs x 3 channels, all 10242 directions",
        "roi_dir_channel_per_s": 2 * 3 * int(dirs.shape[0]) / t_ot}
    log("compare: typed signatures done")
    # reciprocal-space signatures on a cubic grid (Eq. (2)): the paper's
    # benchmark shape, 10^4 ROIs of R = 2 nm in full-density fcc Al, L = 64
    # (and fewer of them at L = 128, 256, 512); algorithmic work 8 N_w L^3 flop per ROI
    # (one complex multiply-add per atom and grid point)
    del pos_d, types_d, cen_d
    pos, cen, _ = synth.fsp_specimen(10000, 2.0)
    off, rel = nat.ar_roi_gather(ctx, torch.from_numpy(pos).to(dev), torch.from_numpy(cen).to(dev), 2.0)
    rel = rel.contiguous()
    n_atoms = int(off[-1])
    fsp = {"rois": len(cen), "mean_atoms": n_atoms / len(cen), "k_max_per_nm": 10.0,
           "measured_fp32_mfma_flop_per_s": peaks["fp32_mfma_flop_per_s"]}
    for L, n in ((64, len(cen)), (128, 2000), (256, 200), (512, 24)):
        o = off[:n + 1]
        out = torch.empty((n, L, L, L), dtype=torch.float32, device=dev)
        t = best_ms(lambda: nat.ar_fsp_amplitudes(ctx, rel, o, L, 10.0, out=out))
        flops = 8.0 * float(o[-1]) * L ** 3
        fsp[f"L{L}"] = {"rois": n, "ms": t, "tflop_per_s": flops / (t / 1e3) / 1e12,
                        "frac_of_datasheet_fp32_mfma": flops / (t / 1e3) / 157.3e12,
                        "frac_of_measured_fp32_mfma": flops / (t / 1e3) / peaks["fp32_mfma_flop_per_s"],
                        "output_gb": n * L ** 3 * 4 / 1e9}
        del out
    x0 = orc.roi_gather(pos, cen[0], 2.0)
    kk = orc.fsp_grid_k(64, 10.0)
    idx = np.random.default_rng(0).integers(0, 64, (2048, 3))
    t0 = time.perf_counter()
    orc.fsp_at(x0, kk[idx])
    t_of = time.perf_counter() - t0
    fsp["cpu_oracle"] = {
        "kind": "oracle", "cores": 1, "sample": f"1 ROI ({len(x0)} atoms) x 2048 grid points, FP64, one thread",
        "flop_per_s": 8.0 * len(x0) * 2048 / t_of,
        "L64_estimate_s": n_atoms * 64 ** 3 / (len(x0) * 2048 / t_of)}
    rec["fsp_cubic_grid"] = fsp
    log("compare: reciprocal-space grid done")
    del rel, off
    # adaptive ROI-grid refinement on the polycrystal cone: a coarse 2 nm grid over the
    # specimen's bounding box (ROIs with >= 100 atoms), batched signatures,
    # kappa = 0.75 on any window, 5^3 split, batched signatures of the refined
    # ROIs; a naive 5^3 refinement of every coarse ROI is priced at the
    # measured refined rate
    log("compare: adaptive grid on the polycrystal cone")
    s3 = synth.polycrystal_cone()
    pos3 = torch.from_numpy(s3.positions).to(dev)
    dirs3 = torch.from_numpy(s3.directions).to(dev)
    w3 = nat.windows_for(s3.radius, s3.nbins, s3.spacings)
    grid = synth.roi_grid(s3.positions.min(0), s3.positions.max(0), 2.0)
    off_all, _ = nat.ar_roi_gather(ctx, pos3, torch.from_numpy(grid).to(dev), s3.radius)
    keep = (torch.diff(off_all) >= 100).cpu().numpy()
    coarse = torch.from_numpy(grid[keep]).to(dev)

    def batch(centres, config=None):
        off, rel = nat.ar_roi_gather(ctx, pos3, centres, s3.radius)
        plan = nat.SignaturePlan(ctx, centres.shape[0], rel.shape[0], dirs3.shape[0], s3.nbins, w3.shape[0])
        if config is None:
            img = plan.tune(rel, off, s3.radius, dirs3, w3)
        else:
            plan.set_config(*config)
            img = plan.run(rel, off, s3.radius, dirs3, w3, use_graph=False)
        t = best_ms(lambda: plan.run(rel, off, s3.radius, dirs3, w3, out=img, use_graph=True), reps=2)
        return off, img, t, plan.config()

    log(f"adaptive grid: {len(coarse)} coarse ROIs")
    off_c, img_c, t_coarse, cfg_c = batch(coarse)
    counts_c = torch.diff(off_c).to(torch.int32).contiguous()
    t_refine = best_ms(lambda: nat.ar_refine_roi_grid(ctx, coarse, img_c, counts_c, 0xF, 0.75, 2.0, 5))
    refined, parent = nat.ar_refine_roi_grid(ctx, coarse, img_c, counts_c, 0xF, 0.75, 2.0, 5)
    del img_c
    log(f"adaptive grid: {refined.shape[0]} refined ROIs")
    off_r, img_r, t_refined, _ = batch(refined.contiguous(), cfg_c)
    n_c, n_r = int(coarse.shape[0]), int(refined.shape[0])
    rec["adaptive_grid_polycrystal"] = {
        "coarse_rois": n_c, "kept": n_r // 125, "refined_rois": n_r, "directions": int(dirs3.shape[0]),
        "coarse_signatures_ms": t_coarse, "selection_and_split_ms": t_refine, "refined_signatures_ms": t_refined,
        "total_ms": t_coarse + t_refine + t_refined,
        "naive_refined_rois": n_c * 125, "naive_estimate_ms": t_refined * n_c * 125 / max(n_r, 1),
        "refined_roi_dir_per_s": n_r * int(dirs3.shape[0]) / (t_refined / 1e3)}
    print(json.dumps(rec))


def cpu_baseline(s, windows, L, lib_q, ref, T, args, n_lib):
    """The oracle, as it stands, on a bounded sample of the same workload:
    signatures of `cpu_sample_rois` ROIs (all directions), their FP64 indexing
    against the full library, and the FP64 refinement of the same ROIs for 2
    iterations (finite-difference gradients), extrapolated per ROI to the
    step's 50 iterations."""
    from oracle import oracle as orc
    threads = orc.default_threads()
    n = args.cpu_sample_rois
    sel = np.linspace(0, len(s.centres) - 1, n).astype(int)
    Lh = None
    t0 = time.perf_counter()
    img, cnt = orc.signatures(s.positions, s.centres[sel], s.radius, s.directions, s.nbins, windows, threads)
    t_sig = time.perf_counter() - t0
    Lcpu = L.cpu().numpy()
    t0 = time.perf_counter()
    Lh = orc.normalise(Lcpu)
    Sh = orc.normalise(img.astype(np.float32))
    idx, sc = orc.index_topk(Sh, Lh, 16, threads)
    t_idx = time.perf_counter() - t0
    del Lh
    # refinement: 2 iterations on `threads` ROIs in parallel (one per thread)
    import concurrent.futures as cf
    Tn = T.cpu().numpy()[0].astype(np.float64)
    it = 2
    rels = [orc.roi_gather(s.positions, s.centres[r], s.radius) for r in sel[:threads]]
    qs = [lib_q[idx[i, 0]] for i in range(len(rels))]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda a: orc.sf_refine(a[0], a[1], s.directions, np.array(F_AL), Tn, steps=it),
                    zip(rels, qs)))
    t_ref = time.perf_counter() - t0
    per_roi = t_sig / n + t_idx / n + (t_ref / len(rels)) * (args.refine_steps / it)
    return {
        "value": len(s.directions) / per_roi,
        "unit": "ROI·direction/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_info(),
        "sample": (f"{n} of 2000 ROIs: oracle signatures (all 10242 directions) {t_sig:.1f} s and FP64 indexing "
                   f"against all {n_lib} references {t_idx:.1f} s; FP64 finite-difference refinement of "
                   f"{len(rels)} ROIs for {it} iterations {t_ref:.1f} s, scaled per ROI to "
                   f"{args.refine_steps} iterations; {threads} threads"),
        "seconds": {"signatures": t_sig, "indexing": t_idx, "refinement_sample": t_ref},
    }


if __name__ == "__main__":
    main()
