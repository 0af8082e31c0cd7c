#!/usr/bin/env python
"""Benchmark: milliseconds per 300-frame RCA ensemble on one MI355X.

One step = the whole path on one ensemble whose IQ channel data (5.66 GB,
300 frames x 2 orientations x 9 angles x 128 elements x 1024 samples, complex64)
is already resident in HBM: stage-1 DAS -> stage-2 projection -> clutter filter
-> localisation.  Two forms are timed on the same IQ:
  plain     FP64-accumulated Gram, FP64 eigen, FP64 removal; NCC localisation
            (`value` is this form's ms/ensemble)
  bf16_cnn  BF16 hi/lo split Gram and removal with FP32 accumulation, FP64
            eigen; the learned CNN localiser (BF16 activations) with the
            trained weights in paper_2511_21647_amd/weights/
  xdoppler  the plain path with XDoppler before the NCC: cross projections of
            the other orientation's volume, both stacks filtered, 3-frame
            cross-correlation of the filtered stacks
  slab_p8   the paper's sub-block projection: slabs of 8 slices (2 x 35
            planes), plain filter and NCC on every slab plane, then the
            XZ/YZ pairing into 3D localisations
The IQ comes from the library's forward simulator of a
synthetic medium shaped like the paper's pig-kidney acquisition (2000 MBs on
vessel splines, 20000 tissue scatterers 40 dB above the MBs, rigid 0.2 mm
1 Hz motion), generated on the GPU before timing.

Prints one JSON line.  `roofline` is for the dominant kernel (stage-1 DAS,
VALU-bound); `cpu_baseline` times the FP64 oracle on a bounded sample on the
host cores (rank 0, N=1 only).

Sub-commands used to produce the committed profiles:
  --profile-das       run the simulator, one stage-1 launch and a 1 GiB copy
                      (for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs)
  --summarize-pmc DIR write the counter summary from two rocprofv3 --pmc runs
  --stream N          streaming run: N consecutive ensembles (MB count ramping
                      1000 -> 10000, non-rigid tissue motion), both forms per
                      ensemble, p50/p99 ms and the density-map SSIM of the forms,
                      and the paper's whole per-ensemble order (motion, slabs of
                      one, separation, per-subset NCC and pairing)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12      # 128 B per clock per CU
# per channel-pixel-angle-frame evaluation: the complex interpolation as two
# FMAs on the staged (sample, forward difference) pair, and the complex
# multiply-accumulate by the phasor as four FMAs: 6 FMAs = 12 flop
DAS_FLOPS_PER_EVAL = 12
COUNTERS_FILE = os.path.join(ROOT, "profiles", "das_stage1_paper_counters.json")
DAS_SOURCE = os.path.join(ROOT, "paper_2511_21647_amd", "csrc", "das.hip")
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    return hashlib.sha256(open(DAS_SOURCE, "rb").read()).hexdigest()[:16]


def setup(precision: str, ensemble: int = 0):
    import numpy as np
    import torch
    import paper_2511_21647_amd as ulm
    from synth import cfg_paper, make_medium

    cfg = cfg_paper()
    prec = ulm.ULM_PREC_BF16X3 if precision == "bf16x3" else ulm.ULM_PREC_FP64GRAM
    t0 = time.time()
    med = make_medium(cfg, ensemble)
    ctx = ulm.Context(cfg, precision=prec)
    pos = torch.from_numpy(np.ascontiguousarray(med.pos)).cuda()
    amp = torch.from_numpy(med.amp).cuda()
    iq = ulm.ulm_sim_channel_data(ctx, pos, amp, med.noise_seed, med.noise_sigma)
    torch.cuda.synchronize()
    del pos, amp
    log(f"setup: medium + GPU simulation of {tuple(iq.shape)} IQ in {time.time() - t0:.1f} s")
    return cfg, ctx, iq


def das_evals(cfg) -> int:
    g = cfg.grid
    return 2 * cfg.n_angles * cfg.seq.n_frames * g.nz * g.nu * cfg.probe.n_elem


def das_staged_entries(cfg) -> int:
    """Staged (sample, difference) entries of one frame summed over every
    (transmit, 8 x 32 tile, receive element): each window is staged in 16-sample
    chunks from the first to the last sample the tile reads (the library's host
    rule, with its FP32 sum of receive and transmit delay)."""
    import numpy as np
    p, g, q = cfg.probe, cfg.grid, cfg.seq
    z = g.z0 + np.arange(g.nz) * g.dz
    u = g.u0 + np.arange(g.nu) * g.du
    ue = (np.arange(p.n_elem) - 0.5 * (p.n_elem - 1)) * p.pitch
    dx = u[None, None, :] - ue[:, None, None]
    zz = z[None, :, None]
    rxd = (dx * dx / (np.sqrt(dx * dx + zz * zz) + zz) * p.fs / p.c).astype(np.float32)
    L = (p.n_elem - 1) * p.pitch
    ntz, ntu = -(-g.nz // 8), -(-g.nu // 32)
    total = 0
    for th in np.deg2rad(np.asarray(q.angles_deg, dtype=np.float64)):
        ttx = (z * np.cos(th) + g.v_ref * np.sin(th) + 0.5 * L * abs(np.sin(th))) / p.c
        sfull = (ttx + z / p.c - q.t_start) * p.fs
        sti = np.floor(sfull)
        stx = (sfull - sti).astype(np.float32)
        idx = np.floor(rxd + stx[None, :, None]).astype(np.int64) + sti.astype(np.int64)[None, :, None]
        pad_hi = np.full((p.n_elem, ntz * 8, ntu * 32), np.iinfo(np.int64).min)
        pad_lo = np.full((p.n_elem, ntz * 8, ntu * 32), np.iinfo(np.int64).max)
        pad_hi[:, :g.nz, :g.nu] = idx
        pad_lo[:, :g.nz, :g.nu] = idx
        hi = pad_hi.reshape(p.n_elem, ntz, 8, ntu, 32).max(axis=(2, 4))
        lo = pad_lo.reshape(p.n_elem, ntz, 8, ntu, 32).min(axis=(2, 4))
        total += int((16 * -(-(hi - lo + 1) // 16)).sum())
    return 2 * total


WEIGHTS = os.path.join(ROOT, "paper_2511_21647_amd", "weights", "cnn_paper.npy")


def run_form(form, cfg, ctx, iq, args, cnn_params=None):
    """Times `args.steps` steps of one form; returns (ms/step, stage ms, detections)."""
    import torch
    import paper_2511_21647_amd as ulm

    cap = 4_000_000 if form != "slab_p8" else 1 << 25
    proj = torch.empty(ctx.proj_shape, dtype=torch.complex64, device="cuda")
    eig = torch.empty(ctx.proj_shape[:3], dtype=torch.float64, device="cuda")
    locs = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    cws = None
    if form == "bf16_cnn":
        cws = ulm.Workspace(ulm.ulm_cnn_localize_workspace_size(ctx, 64), "cuda")
    pair = form == "slab_p8"
    xd = form == "xdoppler"
    if xd:
        cross = torch.empty(ctx.proj_shape, dtype=torch.complex64, device="cuda")
    if pair:
        pair_cap = 1 << 24
        pairs = torch.empty((pair_cap, 8), dtype=torch.int32, device="cuda")
        pair_count = torch.zeros(1, dtype=torch.int32, device="cuda")
        pws = ulm.Workspace(ulm.ulm_pair_workspace_size(ctx, cap), "cuda")

    def step(ev=None):
        if ev: ev[0].record()
        ulm.rca_beamform_stage1(ctx, iq)
        if ev: ev[1].record()
        ulm.rca_beamform_stage2(ctx, proj)
        if xd:
            ulm.rca_beamform_cross(ctx, cross)
        if ev: ev[2].record()
        ulm.svd_clutter_filter(ctx, proj, eig)
        if xd:
            ulm.svd_clutter_filter(ctx, cross, eig)
            ulm.ulm_xdoppler(ctx, proj, cross, 3, out=proj)
        if ev: ev[3].record()
        if form == "bf16_cnn":
            ulm.ulm_cnn_localize(ctx, cnn_params, proj, cap, ulm.CNN_THRESHOLD, 64, ulm.ULM_CNN_BF16, locs,
                                 count, ws=cws)
        else:
            ulm.ncc_localize(ctx, proj, cap, locs, count)
        if ev: ev[4].record()
        if pair:
            ulm.ulm_pair_planes(ctx, locs, count, cap, pair_cap, pairs, pair_count, ws=pws)
            if ev: ev[5].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ulm.ulm_check_status(ctx, count, cap)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ulm.ulm_check_status(ctx, count, cap)
    ms_step = (t1 - t0) * 1e3 / args.steps
    names = ["das_stage1", "stage2_projection" + ("_and_cross" if xd else ""),
             "clutter_filter" + ("_both_and_xdoppler" if xd else ""),
             "cnn_localize" if form == "bf16_cnn" else "ncc_localize"] + (["pairing_3d"] if pair else [])
    stage = {n: sum(e[i].elapsed_time(e[i + 1]) for e in evs) / args.steps
             for i, n in enumerate(names)}
    n_det = int(count.item())
    if pair:
        ulm.ulm_check_status(ctx, pair_count, pair_cap)
        n_det = (n_det, int(pair_count.item()))
        del pairs, pws
    del proj, eig, locs, cws
    if xd:
        del cross
    torch.cuda.empty_cache()
    return ms_step, stage, n_det


def run_inflight(cfg, ctx, iq, args):
    """Throughput of the plain path with `args.inflight` ensembles in flight: each
    has its own context (tables and workspace) and HIP stream, and consecutive
    ensembles alternate between them, so one ensemble's latency-bound kernels
    (the eigensolver holds one XCD per plane) overlap the next one's DAS.
    Returns (ms per ensemble, detections of the last ensemble per context)."""
    import torch
    import paper_2511_21647_amd as ulm

    n = args.inflight
    cap = 4_000_000
    ctxs = [ctx] + [ulm.Context(cfg) for _ in range(n - 1)]
    streams = [torch.cuda.Stream() for _ in range(n)]
    bufs = [dict(proj=torch.empty(ctx.proj_shape, dtype=torch.complex64, device="cuda"),
                 eig=torch.empty(ctx.proj_shape[:3], dtype=torch.float64, device="cuda"),
                 locs=torch.empty((cap, 8), dtype=torch.int32, device="cuda"),
                 count=torch.zeros(1, dtype=torch.int32, device="cuda")) for _ in range(n)]
    torch.cuda.synchronize()

    def step(k):
        i = k % n
        c, b = ctxs[i], bufs[i]
        with torch.cuda.stream(streams[i]):
            ulm.rca_beamform_stage1(c, iq)
            ulm.rca_beamform_stage2(c, b["proj"])
            ulm.svd_clutter_filter(c, b["proj"], b["eig"])
            ulm.ncc_localize(c, b["proj"], cap, b["locs"], b["count"])

    for k in range(max(args.warmup, n)):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dets = []
    for c, b in zip(ctxs, bufs):
        ulm.ulm_check_status(c, b["count"], cap)
        dets.append(int(b["count"].item()))
    for c in ctxs[1:]:
        c.close()
    del bufs
    torch.cuda.empty_cache()
    return (t1 - t0) * 1e3 / args.steps, dets


MOTION_MAX_LAG = 8
FP32_MFMA_PEAK_TFLOPS = 157.3


def time_motion(cfg, ctx, args):
    """Rigid motion estimation on the stage-1 slices left in the workspace by
    the last timed step (lag window +-8 px, reference frame 0): ms per
    ensemble and the correlation contraction's rate against the FP32 MFMA
    peak (2 flop per pixel, lag, frame and slice)."""
    import torch
    import paper_2511_21647_amd as ulm

    S = ulm.ulm_stage1_slices(ctx)
    ws = ulm.Workspace(ulm.ulm_motion_workspace_size(ctx, MOTION_MAX_LAG), "cuda")
    F, K = cfg.seq.n_frames, cfg.n_angles
    disp = torch.empty((2, K, F, 2), dtype=torch.float32, device="cuda")
    mot = torch.empty((F, 3), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        ulm.ulm_motion_estimate(ctx, S, 0, MOTION_MAX_LAG, disp, mot, ws=ws)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        ulm.ulm_motion_estimate(ctx, S, 0, MOTION_MAX_LAG, disp, mot, ws=ws)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    nl = (2 * MOTION_MAX_LAG + 1) ** 2
    flops = 2.0 * 2 * K * F * nl * cfg.grid.nz * cfg.grid.nu
    tf = flops / (ms * 1e-3) / 1e12
    del ws
    return {"ms_per_ensemble": round(ms, 3), "max_lag": MOTION_MAX_LAG, "ref_frame": 0,
            "roofline": {"bound": "mfma", "kernel": "ulm_motion_estimate (its four kernels)",
                         "achieved": round(tf, 2), "peak": FP32_MFMA_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tf / FP32_MFMA_PEAK_TFLOPS, 4),
                         "algorithmic_flops": flops}}


SEPARATION_SPEEDS = 3


def time_separation(cfg, ctx, args):
    """MB separation of a 2 x 250 x 274 x 300 plane stack into up/down x 3 speed
    ranges (six subsets): ms per ensemble and the HBM rate of its algorithmic
    traffic (one read of the planes, one write per subset)."""
    import torch
    import paper_2511_21647_amd as ulm

    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    planes = torch.randn(ctx.proj_shape, dtype=torch.complex64, device="cuda", generator=g)
    subs = torch.empty((2 * SEPARATION_SPEEDS,) + tuple(ctx.proj_shape), dtype=torch.complex64,
                       device="cuda")
    for _ in range(args.warmup):
        ulm.ulm_separate(ctx, planes, SEPARATION_SPEEDS, subs)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        ulm.ulm_separate(ctx, planes, SEPARATION_SPEEDS, subs)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.steps
    nbytes = planes.numel() * 8 * (1 + 2 * SEPARATION_SPEEDS)
    gbs = nbytes / (ms * 1e-3) / 1e9
    del planes, subs
    torch.cuda.empty_cache()
    return {"ms_per_ensemble": round(ms, 3), "subsets": 2 * SEPARATION_SPEEDS,
            "roofline": {"bound": "hbm", "kernel": "sep_kernel", "achieved": round(gbs, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes": nbytes}}


def run_gpu(args):
    import numpy as np
    import torch
    import paper_2511_21647_amd as ulm

    cfg, ctx, iq = setup("fp64gram")
    forms = {}
    ms, stage, n = run_form("plain", cfg, ctx, iq, args)
    forms["plain"] = {"ms_per_ensemble": round(ms, 3), "stages_ms": {k: round(v, 3) for k, v in
                                                                       stage.items()},
                      "detections": n}
    log(f"plain: {ms:.2f} ms/ensemble {stage}")
    if args.inflight > 1:
        ms_i, dets = run_inflight(cfg, ctx, iq, args)
        if any(d != n for d in dets):
            raise SystemExit(f"in-flight run found {dets} detections, the single run {n}")
        forms["plain"]["inflight"] = {"ensembles_in_flight": args.inflight,
                                      "ms_per_ensemble": round(ms_i, 3)}
        log(f"plain, {args.inflight} ensembles in flight: {ms_i:.2f} ms/ensemble")
    forms["plain"]["motion_estimation"] = time_motion(cfg, ctx, args)
    log(f"motion estimation: {forms['plain']['motion_estimation']}")
    forms["plain"]["mb_separation"] = time_separation(cfg, ctx, args)
    log(f"MB separation: {forms['plain']['mb_separation']}")
    if args.form == "both":
        # XDoppler: the other orientation's volume projected onto every plane,
        # both stacks filtered, 3-frame cross-correlation, NCC on its image
        ms_x, stage_x, n_x = run_form("xdoppler", cfg, ctx, iq, args)
        forms["xdoppler"] = {"ms_per_ensemble": round(ms_x, 3),
                             "stages_ms": {k: round(v, 3) for k, v in stage_x.items()},
                             "detections": n_x, "window": 3}
        log(f"xdoppler: {ms_x:.2f} ms/ensemble {stage_x}")
    if args.form == "both" and os.path.exists(WEIGHTS):
        ctx_b = ulm.Context(cfg, precision=ulm.ULM_PREC_BF16X3)
        params = torch.from_numpy(np.load(WEIGHTS).astype(np.float32)).cuda()
        ms_b, stage_b, n_b = run_form("bf16_cnn", cfg, ctx_b, iq, args, params)
        forms["bf16_cnn"] = {"ms_per_ensemble": round(ms_b, 3),
                             "stages_ms": {k: round(v, 3) for k, v in stage_b.items()},
                             "detections": n_b}
        log(f"bf16_cnn: {ms_b:.2f} ms/ensemble {stage_b}")
        ctx_b.close()
    elif args.form == "both":
        forms["bf16_cnn"] = {"skipped": f"no trained weights at {WEIGHTS}"}
    if args.form == "both":
        # the paper's sub-block form: slabs of 8 slices, 2 x 35 planes, 3D pairing
        from synth import with_blocks
        cfg_s = with_blocks(cfg, -(-cfg.grid.nv // 8))
        ctx_s = ulm.Context(cfg_s)
        ms_s, stage_s, (n_s, n_pairs) = run_form("slab_p8", cfg_s, ctx_s, iq, args)
        forms["slab_p8"] = {"ms_per_ensemble": round(ms_s, 3),
                            "planes": [2 * cfg_s.grid.n_blocks, cfg_s.grid.nz, cfg_s.grid.nu],
                            "stages_ms": {k: round(v, 3) for k, v in stage_s.items()},
                            "detections": n_s, "pairs_3d": n_pairs}
        log(f"slab_p8: {ms_s:.2f} ms/ensemble {stage_s}")
        ctx_s.close()
    torch.cuda.synchronize()
    ctx.close()
    del iq
    torch.cuda.empty_cache()
    return cfg, ms, stage, n, forms


def run_stream(args):
    import numpy as np
    import torch
    import paper_2511_21647_amd as ulm
    from paper_2511_21647_amd.train_cnn import ssim
    from synth import cfg_stream, make_medium, plane_positions

    N = args.stream
    cfg0 = cfg_stream(1000)
    ctx_p = ulm.Context(cfg0)
    ctx_b = ulm.Context(cfg0, precision=ulm.ULM_PREC_BF16X3)
    params = torch.from_numpy(np.load(WEIGHTS).astype(np.float32)).cuda()
    iq = torch.empty(ctx_p.iq_shape, dtype=torch.complex64, device="cuda")
    proj = torch.empty(ctx_p.proj_shape, dtype=torch.complex64, device="cuda")
    cap = 4_000_000
    locs = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    cws = ulm.Workspace(ulm.ulm_cnn_localize_workspace_size(ctx_b, 64), "cuda")
    g = cfg0.grid
    dens = {f: torch.zeros((2, 2 * g.nz, 2 * g.nu), dtype=torch.int32, device="cuda")
            for f in ("plain", "bf16_cnn")}
    ms = {"plain": [], "bf16_cnn": [], "paper_order": []}
    dets = {"plain": 0, "bf16_cnn": 0, "paper_order": 0}
    # the paper's whole per-ensemble order on the plain path: stage 1, motion
    # estimation on the slices, stage 2, filter, separation (Up3Down3), NCC of
    # every subset, XZ/YZ pairing of every subset
    S = SEPARATION_SPEEDS
    subs = torch.empty((2 * S,) + tuple(ctx_p.proj_shape), dtype=torch.complex64, device="cuda")
    mws = ulm.Workspace(ulm.ulm_motion_workspace_size(ctx_p, MOTION_MAX_LAG), "cuda")
    disp = torch.empty((2, cfg0.n_angles, cfg0.seq.n_frames, 2), dtype=torch.float32, device="cuda")
    mot = torch.empty((cfg0.seq.n_frames, 3), dtype=torch.float32, device="cuda")
    pair_cap = 1 << 21
    pairs = torch.empty((pair_cap, 8), dtype=torch.int32, device="cuda")
    pcount = torch.zeros(1, dtype=torch.int32, device="cuda")
    pws = ulm.Workspace(ulm.ulm_pair_workspace_size(ctx_p, cap), "cuda")
    n_pairs = 0
    axial_err = []
    # true MB density on the same 2x grid (fine bin floor((x + 1/2) 2))
    truth = np.zeros((2, 2 * g.nz, 2 * g.nu))
    for e in range(N):
        n_mb = int(round(1000 + 9000 * e / max(N - 1, 1)))
        cfg = cfg_stream(n_mb)
        med = make_medium(cfg, e)
        for o, per_frame in enumerate(plane_positions(cfg, med)):
            for zu in per_frame:
                bz = np.floor((zu[:, 0] + 0.5) * 2).astype(int)
                bu = np.floor((zu[:, 1] + 0.5) * 2).astype(int)
                ok = (bz >= 0) & (bz < 2 * g.nz) & (bu >= 0) & (bu < 2 * g.nu)
                np.add.at(truth[o], (bz[ok], bu[ok]), 1.0)
        pos = torch.from_numpy(med.pos).cuda()
        amp = torch.from_numpy(med.amp).cuda()
        ulm.ulm_sim_channel_data(ctx_p, pos, amp, med.noise_seed, med.noise_sigma, iq=iq)
        del pos, amp
        for form, ctx in (("plain", ctx_p), ("bf16_cnn", ctx_b)):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            torch.cuda.synchronize()
            ev[0].record()
            ulm.rca_beamform_proj(ctx, iq, proj)
            ulm.svd_clutter_filter(ctx, proj)
            if form == "plain":
                ulm.ncc_localize(ctx, proj, cap, locs, count)
            else:
                ulm.ulm_cnn_localize(ctx, params, proj, cap, ulm.CNN_THRESHOLD, 64, ulm.ULM_CNN_BF16, locs,
                                     count, ws=cws)
            ev[1].record()
            torch.cuda.synchronize()
            ulm.ulm_check_status(ctx, count, cap)
            ulm.ulm_density_accumulate(ctx, locs, count, cap, dens[form], upsample=2)
            ms[form].append(ev[0].elapsed_time(ev[1]))
            dets[form] += int(count.item())
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        ulm.rca_beamform_stage1(ctx_p, iq)
        ulm.ulm_motion_estimate(ctx_p, ulm.ulm_stage1_slices(ctx_p), 0, MOTION_MAX_LAG, disp, mot,
                                ws=mws)
        ulm.rca_beamform_stage2(ctx_p, proj)
        ulm.svd_clutter_filter(ctx_p, proj)
        ulm.ulm_separate(ctx_p, proj, S, subs)
        pair_total = []
        for i in range(2 * S):
            ulm.ncc_localize(ctx_p, subs[i], cap, locs, count)
            ulm.ulm_pair_planes(ctx_p, locs, count, cap, pair_cap, pairs, pcount, ws=pws)
            pair_total.append(pcount.clone())
        ev[1].record()
        torch.cuda.synchronize()
        ms["paper_order"].append(ev[0].elapsed_time(ev[1]))
        n_pairs += int(sum(int(c.item()) for c in pair_total))
        # the stream's tissue motion is non-rigid: compare the estimated axial
        # motion with the medium's displacement averaged over its tissue
        t_disp = med.pos[:, ~med.is_mb, 2] - med.pos[:1, ~med.is_mb, 2]
        axial_err.append(float(np.abs(mot[:, 2].cpu().numpy() - t_disp.mean(axis=1) / g.dz).max()))
        log(f"stream ensemble {e} ({n_mb} MBs): plain {ms['plain'][-1]:.2f} ms, "
            f"bf16_cnn {ms['bf16_cnn'][-1]:.2f} ms, paper order {ms['paper_order'][-1]:.2f} ms")
    dp = dens["plain"].cpu().numpy()
    db = dens["bf16_cnn"].cpu().numpy()
    nrm_ = lambda m: m / max(float(m.sum()), 1.0)
    out = {"metric": "streaming ms per 300-frame ensemble (p50/p99) and density-map SSIM",
           "ensembles": N, "acquisition_ms": 750.0,
           "mb_per_ensemble": [1000, 10000], "motion": "non-rigid, 0.3 mm, 0.5-2 Hz"}
    for f in ms:
        a = np.array(ms[f])
        out[f] = {"p50_ms": round(float(np.percentile(a, 50)), 3),
                  "p99_ms": round(float(np.percentile(a, 99)), 3),
                  "max_ms": round(float(a.max()), 3), "detections": dets[f]}
    out["density_ssim_bf16_cnn_vs_plain"] = [round(ssim(nrm_(db[o]), nrm_(dp[o])), 4) for o in range(2)]
    # each map as a distribution (divided by its total), so the SSIM compares structure
    nrm = lambda m: m / max(float(m.sum()), 1.0)
    out["density_ssim_vs_true_mbs"] = {
        "plain": [round(ssim(nrm(dp[o]), nrm(truth[o])), 4) for o in range(2)],
        "bf16_cnn": [round(ssim(nrm(db[o]), nrm(truth[o])), 4) for o in range(2)]}
    out["paper_order"]["steps"] = ("stage 1, motion estimation (L = 8), stage 2, filter, "
                                   f"separation into {2 * S} subsets, NCC and XZ/YZ pairing per subset")
    out["paper_order"]["pairs_3d"] = n_pairs
    out["paper_order"]["max_axial_motion_error_px"] = round(max(axial_err), 3)
    torch.cuda.synchronize()
    ctx_p.close()
    ctx_b.close()
    print(json.dumps(out), flush=True)


def roofline(cfg, das_ms):
    flops = DAS_FLOPS_PER_EVAL * das_evals(cfg)
    achieved = flops / (das_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(COUNTERS_FILE):
        rec = json.load(open(COUNTERS_FILE))
        if rec.get("source_sha") == source_hash():
            traffic = rec["hbm_bytes_per_launch"]
    # the kernel's LDS traffic: 16 B of (sample, difference) read per evaluation,
    # and per work-group (8 x 32 pixel tile, 16 frames, one transmit) and
    # receive element the window's staged entries of 16 B written for 16 frames
    frame_blocks = -(-cfg.seq.n_frames // 16)
    lds_bytes = 16 * das_evals(cfg) + das_staged_entries(cfg) * 16 * 16 * frame_blocks
    lds_tbs = lds_bytes / (das_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "das_stage1_kernel", "achieved": round(achieved, 2),
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic,
            "algorithmic_flops": flops, "launch_ms": round(das_ms, 3),
            "lds": {"bytes": lds_bytes, "achieved": round(lds_tbs, 2), "peak": LDS_PEAK_TBS,
                    "unit": "TB/s", "frac": round(lds_tbs / LDS_PEAK_TBS, 4)}}


def cpu_baseline(cfg):
    """The FP64 oracle on the host cores, scaled to one ensemble.  The clutter
    filter is timed whole (both 68,500 px x 300 frame planes of synthetic
    tissue, noise and MB echoes); the NCC localisation on 30 frames of each
    filtered plane, scaled by 10; stage-1 DAS and the stage-2 projection, about
    3 minutes per ensemble, on two of the 300 frames, scaled by 150."""
    import numpy as np
    from synth import arrays, with_frames
    from oracle import beamform, clutter, localize

    F = cfg.seq.n_frames
    g = cfg.grid
    nf = 2
    one = with_frames(cfg, nf)
    iq = arrays.complex_normal(one.iq_shape, seed=77, dtype=np.complex128)
    t = time.perf_counter()
    S = beamform.stage1_slices(iq, one)
    t_s1 = time.perf_counter() - t
    t = time.perf_counter()
    beamform.stage2_project(S, one)
    t_s2 = time.perf_counter() - t
    del iq, S
    # the filter and localiser input: a rank-20 tissue stack with weak white
    # "blood", plus about as many point-like MB echoes per image as the
    # simulated ensemble yields detections (370 per image, PSF of the NCC
    # template's width)
    planes = np.stack([(arrays.clutter_stack(g.nz * g.nu, F, rank=20, seed=78 + o).reshape(F, g.nz, g.nu)
                        + arrays.spot_frames(F, g.nz, g.nu, 370, cfg.loc.sigma_z, cfg.loc.sigma_u,
                                             seed=80 + o))
                       for o in range(2)])[:, None].astype(np.complex128)
    t = time.perf_counter()
    filt, _ = clutter.filter_planes(planes, cfg.svd_cutoff)
    t_f = time.perf_counter() - t
    del planes
    nl = 30                                      # frames of each plane localised
    t = time.perf_counter()
    recs, _, _ = localize.localize(filt[:, :, :nl], cfg)
    t_n = (time.perf_counter() - t) * F / nl
    total_s = (t_s1 + t_s2) * F / nf + t_f + t_n
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    return {"value": round(total_s * 1e3, 1), "unit": "ms/ensemble",
            "cores": min(threads, os.cpu_count()), "kind": "oracle",
            "sample": (f"clutter filter of both full planes of synthetic tissue, noise and MB "
                       f"echoes timed whole ({t_f:.2f} s); NCC localisation of {2 * nl} of the "
                       f"{2 * F} filtered images ({len(recs)} detections) scaled by {F // nl}; "
                       f"stage-1 DAS + stage-2 projection of {nf} of {F} frames "
                       f"({t_s1:.2f} + {t_s2:.2f} s) scaled by {F // nf}"),
            "stages_s": {"das_stage1": round(t_s1 * F / nf, 2), "stage2": round(t_s2 * F / nf, 2),
                         "clutter_filter": round(t_f, 2), "ncc_localize": round(t_n, 2)}}


def profile_das(args):
    import torch
    import paper_2511_21647_amd as ulm
    cfg, ctx, iq = setup("fp64gram")
    ulm.rca_beamform_stage1(ctx, iq)
    torch.cuda.synchronize()
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    log("profile run done: one das_stage1_kernel launch and one 1 GiB copy")


def profile_kernels(args):
    """One launch each of the clutter filter's Gram in both precision forms and
    of the CNN localiser on the paper-scale ensemble (for rocprofv3 --pmc runs
    of the matrix-core counters)."""
    import numpy as np
    import torch
    import paper_2511_21647_amd as ulm
    cfg, ctx, iq = setup("fp64gram")
    proj = ulm.rca_beamform_proj(ctx, iq)
    del iq
    ctx_b = ulm.Context(cfg, precision=ulm.ULM_PREC_BF16X3)
    d = proj.clone()
    ulm.svd_clutter_filter(ctx, proj)
    ulm.svd_clutter_filter(ctx_b, d)
    params = torch.from_numpy(np.load(WEIGHTS).astype(np.float32)).cuda()
    cws = ulm.Workspace(ulm.ulm_cnn_localize_workspace_size(ctx_b, 64), "cuda")
    cap = 4_000_000
    locs = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    ulm.ulm_cnn_localize(ctx_b, params, d, cap, ulm.CNN_THRESHOLD, 64, ulm.ULM_CNN_BF16, locs, count,
                         ws=cws)
    torch.cuda.synchronize()
    ctx_b.close()
    ctx.close()
    log("profile run done: both Gram forms, the CNN localiser")


MFMA_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_BF16",
                 "SQ_INSTS_VALU_MFMA_MOPS_F64", "MfmaUtil")


def summarize_mfma(d, out_md, cmd):
    """Matrix-core counters per kernel (summed over its dispatches) from a
    rocprofv3 --pmc run of --profile-kernels: MfmaUtil (rocprofiler's derived
    counter: MFMA-busy cycles over GUI-active cycles x SIMDs) and the issued
    MFMA flop (MOPS x 512)."""
    per = {}
    for r in _read_counter_rows(d):
        name = r.get("Kernel_Name", "")
        if not name or "ulm" not in name:
            continue
        key = (r.get("Dispatch_Id"), name)
        per.setdefault(key, {})[r["Counter_Name"]] = per.get(key, {}).get(r["Counter_Name"], 0.0) \
            + float(r["Counter_Value"])
    agg = {}
    for (_, name), vals in per.items():
        short = readable(name).split("(")[0].replace("void ", "")
        a = agg.setdefault(short, {"dispatches": 0, "util": []})
        a["dispatches"] += 1
        for k, v in vals.items():
            if k == "MfmaUtil":
                a["util"].append(v)
            else:
                a[k] = a.get(k, 0.0) + v
    lines = ["| Kernel | Dispatches | MfmaUtil (%) per dispatch, mean | MFMA-busy cycles (sum) | "
             "BF16 MFMA flop issued | FP64 MFMA flop issued |", "|---|---|---|---|---|---|"]
    for short, a in sorted(agg.items(), key=lambda kv: -kv[1].get("SQ_VALU_MFMA_BUSY_CYCLES", 0)):
        if a.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) <= 0:
            continue
        util = sum(a["util"]) / len(a["util"]) if a["util"] else float("nan")
        lines.append(f"| `{short}` | {a['dispatches']} | {util:.1f} | "
                     f"{a.get('SQ_VALU_MFMA_BUSY_CYCLES', 0):.3g} | "
                     f"{512 * a.get('SQ_INSTS_VALU_MFMA_MOPS_BF16', 0):.3g} | "
                     f"{512 * a.get('SQ_INSTS_VALU_MFMA_MOPS_F64', 0):.3g} |")
    text = (f"Command (run from the repository root on one MI355X):\n\n```\n{cmd}\n```\n\n"
            + "\n".join(lines) + "\n")
    with open(out_md, "w") as fh:
        fh.write(text)
    print(text)


def _read_counter_rows(d):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_pmc(d_fetch, d_write):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the DAS kernel, scaled by the
    same counter's reading for the 1 GiB device copy of the same run (the copy
    reads and writes COPY_BYTES)."""
    def dispatches(d, counter):
        out = {}
        for r in _read_counter_rows(d):
            if r.get("Counter_Name") != counter:
                continue
            key = (r.get("Dispatch_Id"), r.get("Kernel_Name", ""))
            out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
        return out

    def pick(vals, counter):
        das = [v for (_, n), v in vals.items() if "das_stage1" in n]
        copy = [v for (_, n), v in vals.items() if "copyBuffer" in n]
        if len(das) != 1 or not copy:
            raise SystemExit(f"{counter}: expected one das_stage1 dispatch and a copy, got "
                             f"{sorted(set(n for (_, n) in vals))[:8]}")
        return das[0], max(copy)

    f_das, f_cp = pick(dispatches(d_fetch, "FETCH_SIZE"), "FETCH_SIZE")
    w_das, w_cp = pick(dispatches(d_write, "WRITE_SIZE"), "WRITE_SIZE")
    f_scale = COPY_BYTES / (f_cp * 1024.0)
    w_scale = COPY_BYTES / (w_cp * 1024.0)
    rec = {"kernel": "das_stage1_kernel", "copy_kernel": "__amd_rocclr_copyBuffer (1 GiB)",
           "fetch_kib": f_das, "write_kib": w_das, "copy_fetch_kib": f_cp,
           "copy_write_kib": w_cp, "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_bytes": f_das * 1024.0 * f_scale, "write_bytes": w_das * 1024.0 * w_scale,
           "hbm_bytes_per_launch": f_das * 1024.0 * f_scale + w_das * 1024.0 * w_scale,
           "source_sha": source_hash()}
    os.makedirs(os.path.dirname(COUNTERS_FILE), exist_ok=True)
    with open(COUNTERS_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


# Algorithmic work per launch for the kernel-trace summary, on the paper-scale
# workload (F frames, NPIX pixels per plane, K transmits per orientation, NC
# elements).  `planes` / `images` are read off the launch grid.
F_P, NPIX_P, K_P, NC_P, C_P = 300, 250 * 274, 9, 128, 20
GRAM_WGS_PER_PLANE = 15 * 34           # 64x64 block pairs x 2048-pixel chunks
BF16_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6


def _kernel_work(name, wgs, gy, gz):
    """(bound, work per launch, unit of work, peak, note) or None."""
    plane_bytes = F_P * NPIX_P * 8
    short = name.split("(")[0].replace("void ", "")
    if "das_stage1_kernel" in short:
        return ("alu", DAS_FLOPS_PER_EVAL * 2 * K_P * F_P * NPIX_P * NC_P, "flop",
                FP32_VECTOR_PEAK_TFLOPS, "12 flop per channel-pixel-transmit-frame evaluation")
    if "gram_f64_kernel" in short or "gram_bf16x3_kernel" in short:
        planes = max(1, round(wgs / GRAM_WGS_PER_PLANE))
        flops = planes * 4.0 * F_P * F_P * NPIX_P        # Hermitian half, 8 flop per complex MAC
        if "f64" in short:
            return ("mfma", flops, "flop", FP64_PEAK_TFLOPS, f"{planes} planes, FP64 MFMA")
        return ("mfma", flops, "flop", BF16_PEAK_TFLOPS,
                f"{planes} planes; the split form issues 6 BF16 products per real product")
    if "removal_f64_kernel" in short:
        planes = gy
        return ("mfma", planes * 16.0 * F_P * C_P * NPIX_P, "flop", FP64_PEAK_TFLOPS,
                f"{planes} planes, two products of F x c complex MACs per pixel, FP64 MFMA")
    if "removal" in short and "tables" not in short:
        planes = gy
        return ("hbm", 2 * planes * plane_bytes, "byte", HBM_PEAK_GBS / 1e3,
                f"{planes} planes read and written once")
    if "stage2_fir_kernel" in short:
        planes = 2 * (35 if "<4>" in short else 1)
        return ("hbm", 2 * K_P * F_P * NPIX_P * 8 + planes * plane_bytes, "byte",
                HBM_PEAK_GBS / 1e3, f"slices read once, {planes} planes written")
    if "frame_max_kernel" in short or "ncc_band_kernel" in short:
        planes = gz if "ncc_band" in short else max(1, round(wgs / F_P))    # one work-group per image
        return ("hbm", planes * plane_bytes, "byte", HBM_PEAK_GBS / 1e3, f"{planes} planes read once")
    if "cnn_conv_kernel" in short:
        # the launch grid is the same for every batch; the median launch is a
        # full batch of 64 images (600 = 9 x 64 + 24)
        return ("mfma", 64 * NPIX_P * 32 * 288 * 2.0, "flop", BF16_PEAK_TFLOPS,
                "one 32 -> 32 conv3x3 layer on 64 images, BF16 MFMA")
    if "cross_profile_kernel" in short:
        return ("hbm", 2 * K_P * F_P * NPIX_P * 8, "byte", HBM_PEAK_GBS / 1e3, "slices read once")
    if "cross_project_kernel" in short:
        return ("hbm", 2 * plane_bytes, "byte", HBM_PEAK_GBS / 1e3, "2 planes written")
    if "xdoppler_kernel" in short:
        return ("hbm", 3 * 2 * plane_bytes, "byte", HBM_PEAK_GBS / 1e3, "2 x 2 planes read, 2 written")
    if "sep_kernel" in short:
        return ("hbm", 7 * 2 * plane_bytes, "byte", HBM_PEAK_GBS / 1e3, "2 planes read, 6 x 2 written")
    if "mot_corr_kernel" in short:
        return ("mfma", 2.0 * 2 * K_P * F_P * 289 * NPIX_P, "flop", FP32_MFMA_PEAK_TFLOPS,
                "2 flop per pixel, lag, frame, slice (289 lags)")
    if "cnn_head_decode_kernel" in short:
        images = gy
        return ("hbm", images * NPIX_P * 32 * 2, "byte", HBM_PEAK_GBS / 1e3,
                f"{images} images of BF16 activations read once")
    if "cnn_localize_fused_kernel" in short:
        # every image of the ensemble: conv0 (32 x 9), five 32 -> 32 conv3x3
        # (32 x 288 each) and the head (64 x 32) MACs per pixel; the strips'
        # halo rows are not counted
        images = 2 * F_P
        per_px = 2.0 * (32 * 9 + 5 * 32 * 288 + 64 * 32)
        return ("mfma", images * NPIX_P * per_px, "flop", BF16_PEAK_TFLOPS,
                f"{images} images, the whole network per pixel, BF16 MFMA")
    return None


def readable(name):
    """Kernel name as printed, the mangled names of the templated CNN kernels
    shown as ulm::<name><element type>."""
    import re
    m = re.match(r"_ZN3ulm(\d+)(\w+)", name)
    if not m:
        return name
    base = m.group(2)[:int(m.group(1))]
    return f"ulm::{base}<{'bf16' if 'DF16b' in name else 'float'}>"


def summarize_trace(src, out_md, cmd):
    """Per-kernel launch statistics of a rocprofv3 kernel trace (a rocpd SQLite
    database or a kernel_trace.csv), grouped by kernel and launch grid, with the
    roofline fraction of every kernel whose algorithmic work is known."""
    import statistics
    groups = {}
    if src.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(src)
        q = ("select name, grid_x / workgroup_x, grid_y, grid_z, duration from kernels")
        for name, wgs, gy, gz, dur in con.execute(q):
            groups.setdefault((name, int(wgs), int(gy), int(gz)), []).append(dur / 1e3)
    else:
        with open(src) as fh:
            for r in csv.DictReader(fh):
                wgs = int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])
                key = (r["Kernel_Name"], wgs, int(r["Grid_Size_Y"]), int(r["Grid_Size_Z"]))
                groups.setdefault(key, []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    rows = [((readable(k[0]),) + k[1:], d) for k, d in rows]
    lines = ["| Kernel | Work-groups | Calls | Mean (us) | Median (us) | Min (us) | Roofline |",
             "|---|---|---|---|---|---|---|"]
    for (name, wgs, gy, gz), d in rows:
        if sum(d) < 50.0:
            continue
        short = name.split("(")[0].replace("void ", "")
        mean, med = statistics.mean(d), statistics.median(d)
        work = _kernel_work(name, wgs, gy, gz)
        roof = ""
        if work:
            bound, w, unit, peak, note = work
            rate = w / (med * 1e-6) / 1e12            # T(flop|byte)/s at the median launch
            roof = (f"{bound}: {w:.3g} {unit} / launch, {rate:.3g} T{unit}/s of {peak:g}, "
                    f"**{rate / peak:.1%}** ({note})")
        lines.append(f"| `{short}` | {wgs * gy * gz} | {len(d)} | {mean:.1f} | {med:.1f} | "
                     f"{min(d):.1f} | {roof} |")
    text = (f"Command (run from the repository root on one MI355X):\n\n```\n{cmd}\n```\n\n"
            + "\n".join(lines) + "\n")
    with open(out_md, "w") as fh:
        fh.write(text)
    print(text)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", choices=["plain", "both"], default="both",
                    help="time the plain path only, or also the BF16 + CNN and slab forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-das", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="one launch each of both Gram forms and the CNN localiser "
                         "(for rocprofv3 --pmc matrix-core counters)")
    ap.add_argument("--summarize-mfma", nargs=3, metavar=("PMC_DIR", "OUT_MD", "COMMAND"))
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE", "OUT_MD", "COMMAND"),
                    help="write a per-kernel summary (with rooflines) of a rocprofv3 kernel "
                         "trace (rocpd .db or kernel_trace.csv)")
    ap.add_argument("--stream", type=int, default=0, metavar="N")
    ap.add_argument("--inflight", type=int, default=1, metavar="N",
                    help="also time the plain path with N > 1 ensembles in flight on N streams "
                         "(off by default, so every stage-1 launch of the run executes alone "
                         "and a kernel trace of the run averages the same launches)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this path runs on one GPU; multi-GPU runs are not supported "
                                   "(ensembles shard across GPUs with no communication)"}))
        sys.exit(2)
    if args.profile_das:
        profile_das(args)
        return
    if args.profile_kernels:
        profile_kernels(args)
        return
    if args.stream:
        run_stream(args)
        return
    cfg, ms_step, stage, n_det, forms = run_gpu(args)
    g = cfg.grid
    out = {
        "metric": "ms per 300-frame RCA ensemble (plain FP32 vs BF16+CNN), HBM/MFMA roofline %",
        "value": round(ms_step, 3), "unit": "ms/ensemble", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale RCA ensemble: 128+128 elements, 9 angles/orientation, "
                               "300 frames, 1024 samples, two 250x274 planes, SVD cutoff 20, "
                               "9x9 NCC",
                   "form": "plain (FP64-accumulated Gram, FP64 eigen, NCC)",
                   "frames": cfg.seq.n_frames,
                   "planes": [2 * g.n_blocks, g.nz, g.nu]},
        "stages_ms": {k: round(v, 3) for k, v in stage.items()},
        "ensembles_per_s": round(1e3 / ms_step, 2),
        "realtime_ratio_vs_750ms": round(ms_step / 750.0, 4),
        "detections": n_det,
        "forms": forms,
        "roofline": roofline(cfg, stage["das_stage1"]),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on host cores) ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
