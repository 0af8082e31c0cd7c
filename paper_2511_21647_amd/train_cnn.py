"""Training and evaluation of the learned MB localiser on simulated ensembles.

Data: for each ensemble the library's forward simulator generates paper-scale
IQ channel data of a seeded medium whose MB count is drawn per ensemble
(uniform in [500, 8000]); the library beamforms and clutter-filters it
(BF16 hi/lo Gram form) and ulm_cnn_images forms the network inputs.  Labels
are the true MB positions in plane pixels.  Training runs the library's
forward / backward kernels and Adam (ulm_cnn_train_step); nothing here
computes a step of the method.

    python -m paper_2511_21647_amd.train_cnn --ensembles 48 --out weights.npy
    python -m paper_2511_21647_amd.train_cnn --evaluate weights.npy --ensembles 4

Evaluation matches detections to the truth (and CNN detections to NCC
detections) one-to-one within 0.5 px, nearest pairs first, per image.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_SEED0 = 0          # training ensembles 0, 1, ...
HELDOUT_SEED0 = 10000    # held-out ensembles 10000, 10001, ... (disjoint)
MB_RANGE = (500, 8000)


def log(*a):
    print(*a, flush=True)


def n_mb_for(ensemble: int) -> int:
    g = np.random.Generator(np.random.PCG64(900_000 + ensemble))
    return int(g.integers(MB_RANGE[0], MB_RANGE[1] + 1))


def init_flat(seed: int) -> np.ndarray:
    """He-normal convolution weights, zero biases, a small head (outputs start near 0)."""
    import paper_2511_21647_amd as ulm
    g = np.random.Generator(np.random.PCG64(seed))
    p, cin = {}, 1
    for l in range(6):
        p[f"w{l}"] = g.standard_normal((32, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin))
        p[f"b{l}"] = np.zeros(32)
        cin = 32
    p["wh"] = g.standard_normal((64, 32)) * 0.01
    p["bh"] = np.zeros(64)
    return ulm.cnn_pack(p)


class Simulator:
    """Paper-scale ensemble -> filtered planes, CNN images and labels on the GPU."""

    def __init__(self, precision=None, blocks=1):
        import torch
        import paper_2511_21647_amd as ulm
        from synth import cfg_cnn, with_blocks
        self.torch, self.ulm = torch, ulm
        self.blocks = blocks
        self.cfg = with_blocks(cfg_cnn(2000), blocks)
        prec = ulm.ULM_PREC_BF16X3 if precision is None else precision
        self.ctx = ulm.Context(self.cfg, precision=prec)
        self.iq = torch.empty(self.ctx.iq_shape, dtype=torch.complex64, device="cuda")
        self.proj = torch.empty(self.ctx.proj_shape, dtype=torch.complex64, device="cuda")

    def ensemble(self, e: int):
        from synth import cfg_cnn, make_medium, plane_positions, with_blocks
        torch, ulm = self.torch, self.ulm
        cfg = with_blocks(cfg_cnn(n_mb_for(e)), self.blocks)
        med = make_medium(cfg, e)
        pos = torch.from_numpy(med.pos).cuda()
        amp = torch.from_numpy(med.amp).cuda()
        ulm.ulm_sim_channel_data(self.ctx, pos, amp, med.noise_seed, med.noise_sigma, iq=self.iq)
        del pos, amp
        ulm.rca_beamform_proj(self.ctx, self.iq, self.proj)
        ulm.svd_clutter_filter(self.ctx, self.proj)
        images = ulm.ulm_cnn_images(self.ctx, self.proj)
        labels = plane_positions(cfg, med)          # [plane][frame] -> [n][2]
        return images, labels, cfg.medium.n_mb


def batch_labels(torch, labels, idx, F):
    """(mb_zu [n][2] f32, mb_img [n] i32) on the GPU for the images `idx`."""
    zu, im = [], []
    for b, n in enumerate(idx):
        p = labels[n // F][n % F]
        zu.append(p.astype(np.float32))
        im.append(np.full(p.shape[0], b, np.int32))
    zu = np.concatenate(zu) if zu else np.zeros((0, 2), np.float32)
    im = np.concatenate(im) if im else np.zeros(0, np.int32)
    if zu.shape[0] == 0:
        return None, None
    return (torch.from_numpy(np.ascontiguousarray(zu)).cuda(),
            torch.from_numpy(np.ascontiguousarray(im)).cuda())


def train(args):
    """Trains on ensembles first .. first + ensembles - 1.  With --state the
    parameters, Adam moments, step count and the next ensemble are kept in an
    .npz file, so a run stopped by --max-seconds continues where it stopped
    (the learning-rate schedule runs over the whole planned number of steps)."""
    import torch
    import paper_2511_21647_amd as ulm
    sim = Simulator()
    cfg = sim.cfg
    F, nz, nu = cfg.seq.n_frames, cfg.grid.nz, cfg.grid.nu
    init = np.load(args.init).astype(np.float32) if args.init else init_flat(args.seed)
    params = torch.from_numpy(init).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    step, hist, start = 0, [], 0
    if args.state and os.path.exists(args.state):
        st = np.load(args.state)
        params = torch.from_numpy(st["params"]).cuda()
        m = torch.from_numpy(st["m"]).cuda()
        v = torch.from_numpy(st["v"]).cuda()
        step, start = int(st["step"]), int(st["next"])
        hist = json.loads(str(st["history"]))
        log(f"continuing from {args.state}: ensemble {args.first + start}, step {step}")
    prec = ulm.ULM_CNN_BF16
    B = args.batch
    ws = ulm.Workspace(ulm.ulm_cnn_workspace_size(B, nz, nu, prec, True), "cuda")
    rng = np.random.Generator(np.random.PCG64(args.seed + start))
    total_steps = args.ensembles * args.passes * (2 * F // B)
    t0 = time.time()
    done = True
    for i in range(start, args.ensembles):
        if args.max_seconds and time.time() - t0 > args.max_seconds:
            start, done = i, False
            break
        e = args.first + i
        images, labels, n_mb = sim.ensemble(e)
        losses = []
        for _ in range(args.passes):
            order = rng.permutation(2 * F)
            for s in range(0, 2 * F - B + 1, B):
                idx = order[s:s + B]
                x = images[torch.from_numpy(idx).cuda()].contiguous()
                zu, im = batch_labels(torch, labels, idx, F)
                step += 1
                frac = step / max(total_steps, 1)
                lr = args.lr * (0.5 * (1 + np.cos(np.pi * min(frac, 1.0)))) if args.cosine else args.lr
                loss = ulm.ulm_cnn_train_step(params, m, v, step, lr, x, zu, im, prec, ws=ws)
                losses.append(loss)
        ls = torch.cat(losses).cpu().numpy()
        hist.append({"ensemble": e, "n_mb": n_mb, "loss_first": float(ls[0]),
                     "loss_last": float(ls[-1]), "loss_mean": float(ls.mean())})
        log(f"ensemble {e} ({n_mb} MBs): loss {ls[0]:.4e} -> {ls[-1]:.4e} "
            f"(mean {ls.mean():.4e}), step {step}, {time.time() - t0:.0f} s")
    if args.state:
        np.savez(args.state, params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
                 step=step, next=start if not done else args.ensembles, history=json.dumps(hist))
    if not done:
        log(f"stopped after {time.time() - t0:.0f} s at ensemble {args.first + start}; state in "
            f"{args.state}")
        return
    out = params.cpu().numpy()
    np.save(args.out, out)
    with open(os.path.splitext(args.out)[0] + "_train.json", "w") as fh:
        json.dump({"ensembles": args.ensembles, "passes": args.passes, "batch": B, "lr": args.lr,
                   "cosine": args.cosine, "steps": step, "seconds": time.time() - t0,
                   "history": hist}, fh, indent=1)
    log(f"saved {args.out}")


def match(det, ref, radius=0.5):
    """One-to-one matches of det [n][2] to ref [m][2] within `radius`, nearest
    pairs first.  Returns (pairs det_i, ref_j).

    Greedy over the candidate pairs sorted by distance, in rounds: a pair that
    is the nearest remaining one of both its detection and its reference is
    one the greedy pass accepts, so each round accepts all such pairs and drops
    every pair that shares an end with them."""
    det = np.asarray(det, np.float64).reshape(-1, 2)
    ref = np.asarray(ref, np.float64).reshape(-1, 2)
    if len(det) == 0 or len(ref) == 0:
        return np.zeros(0, int), np.zeros(0, int)
    from scipy.spatial import cKDTree
    sdm = cKDTree(det).sparse_distance_matrix(cKDTree(ref), radius, output_type="ndarray")
    # ties broken by (det, ref) index so the result does not depend on the tree
    o = np.lexsort((sdm["j"], sdm["i"], sdm["v"]))
    ci, cj = sdm["i"][o].astype(np.int64), sdm["j"][o].astype(np.int64)
    used_d = np.zeros(len(det), bool)
    used_r = np.zeros(len(ref), bool)
    di, rj = [np.zeros(0, np.int64)], [np.zeros(0, np.int64)]
    while ci.size:
        first_i = np.zeros(ci.size, bool)
        first_i[np.unique(ci, return_index=True)[1]] = True
        first_j = np.zeros(cj.size, bool)
        first_j[np.unique(cj, return_index=True)[1]] = True
        acc = first_i & first_j
        di.append(ci[acc])
        rj.append(cj[acc])
        used_d[ci[acc]] = True
        used_r[cj[acc]] = True
        keep = ~(used_d[ci] | used_r[cj])
        ci, cj = ci[keep], cj[keep]
    return np.concatenate(di), np.concatenate(rj)


def per_image(recs, n_img, F):
    """Detections as one (z, u) array per image, image = plane * F + frame."""
    img = recs["plane"].astype(np.int64) * F + recs["frame"].astype(np.int64)
    o = np.argsort(img, kind="stable")
    zu = np.stack([recs["z"][o], recs["u"][o]], axis=1).astype(np.float64)
    cuts = np.searchsorted(img[o], np.arange(1, n_img))
    return np.split(zu, cuts)


def _stack(images):
    """All images' points in one array, image n moved by 4096 n px along z (no
    image is that tall, so points of different images are never within the
    match radius of each other)."""
    pts = [np.asarray(p, np.float64).reshape(-1, 2) + [4096.0 * n, 0.0] for n, p in enumerate(images)]
    return np.concatenate(pts) if pts else np.zeros((0, 2))


def score(dets, truth, radius=0.5):
    d, t = _stack(dets), _stack(truth)
    i, j = match(d, t, radius)
    sq = np.sum((d[i] - t[j]) ** 2, axis=1)
    return {"recall": len(i) / max(len(t), 1), "precision": len(i) / max(len(d), 1),
            "rms_px": float(np.sqrt(sq.mean())) if sq.size else float("nan"),
            "n_det": len(d), "n_ref": len(t), "n_match": len(i)}


def _score_ensemble(e, n_mb, ncc, truth, cnn_by_thr):
    """Scores of one ensemble (CPU only): NCC against the truth; the CNN at each
    threshold against the truth, against all NCC detections and against NCC's
    true detections (those matched one-to-one to a true MB within 0.5 px)."""
    d, t = _stack(ncc), _stack(truth)
    i, _ = match(d, t)
    ncc_true = np.zeros(len(d), bool)
    ncc_true[i] = True
    counts = np.cumsum([0] + [len(x) for x in ncc])
    ncc_t = [x[ncc_true[counts[k]:counts[k + 1]]] for k, x in enumerate(ncc)]
    r = {"ensemble": e, "n_mb": n_mb, "ncc_vs_truth": score(ncc, truth), "cnn": {}}
    for thr, cnn in cnn_by_thr.items():
        if cnn is None:
            r["cnn"][thr] = {"overflow": True}
            continue
        r["cnn"][thr] = {"vs_truth": score(cnn, truth), "vs_ncc": score(cnn, ncc),
                         "vs_ncc_true": score(cnn, ncc_t)}
    return r


def evaluate(weights, ensembles, thresholds=(0.5,), seed0=HELDOUT_SEED0, log_fn=log, workers=4,
             blocks=1):
    """NCC and CNN on held-out ensembles: each against the truth, and the CNN
    against NCC as the reference (all NCC detections, and NCC's true detections),
    for every CNN decode threshold given.  With `blocks` > 1 the planes are the
    slab projections of the sub-block form (Section II-A4): each image sums
    `ceil(Nv / blocks)` slices, so it holds that fraction of the MBs, and the
    truth of a slab image is the MBs whose v lies in its slab.  The matching runs
    in `workers` CPU processes, forked before the GPU is touched, while the GPU
    localises the next ensembles."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    pool = ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) if workers > 0 else None
    if pool is not None:
        list(pool.map(abs, range(workers)))      # start the workers now
    import torch
    import paper_2511_21647_amd as ulm
    sim = Simulator(blocks=blocks)
    cfg = sim.cfg
    F = cfg.seq.n_frames
    n_img = 2 * blocks * F
    params = torch.from_numpy(np.asarray(weights, np.float32)).cuda()
    cap = 4_000_000 if blocks == 1 else 1 << 25
    locs = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    cws = ulm.Workspace(ulm.ulm_cnn_localize_workspace_size(sim.ctx, 64), "cuda")
    jobs = []
    for i in range(ensembles):
        e = seed0 + i
        _, labels, n_mb = sim.ensemble(e)
        truth = [labels[n // F][n % F] for n in range(n_img)]
        ulm.ncc_localize(sim.ctx, sim.proj, cap, locs, count)
        ulm.ulm_check_status(sim.ctx, count, cap)
        ncc = per_image(ulm.locs_to_numpy(locs, count), n_img, F)
        by_thr = {}
        for thr in thresholds:
            ulm.ulm_cnn_localize(sim.ctx, params, sim.proj, cap, thr, 64, ulm.ULM_CNN_BF16,
                                 locs, count, ws=cws)
            try:
                ulm.ulm_check_status(sim.ctx, count, cap)
            except ulm.ULMError as err:
                # more peaks than an image row's staging slot or the capacity: the
                # threshold is recorded as overflowing instead of scored
                if err.code != ulm.ULM_ERR_OVERFLOW:
                    raise
                by_thr[str(thr)] = None
                log_fn(f"ensemble {e}: CNN threshold {thr} overflows ({int(count.item())} peaks)")
                continue
            by_thr[str(thr)] = per_image(ulm.locs_to_numpy(locs, count), n_img, F)
        args = (e, n_mb, ncc, truth, by_thr)
        jobs.append(pool.submit(_score_ensemble, *args) if pool else args)
        log_fn(f"ensemble {e}: {n_mb} MBs localised")
    results = []
    for j in jobs:
        r = j.result() if pool else _score_ensemble(*j)
        results.append(r)
        log_fn(json.dumps(r))
    if pool is not None:
        pool.shutdown()
    return results


def ssim(a, b, sigma=1.5):
    """Mean structural similarity (Wang et al. 2004) of two maps, Gaussian window
    (scipy.ndimage), dynamic range of the two maps."""
    from scipy.ndimage import gaussian_filter
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    L = max(a.max() - a.min(), b.max() - b.min(), 1e-12)
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    g = lambda x: gaussian_filter(x, sigma, mode="reflect", truncate=3.5)
    ma, mb = g(a), g(b)
    va, vb, cab = g(a * a) - ma * ma, g(b * b) - mb * mb, g(a * b) - ma * mb
    return float((((2 * ma * mb + c1) * (2 * cab + c2)) /
                  ((ma * ma + mb * mb + c1) * (va + vb + c2))).mean())


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--ensembles", type=int, default=48)
    ap.add_argument("--passes", type=int, default=1, help="passes over each ensemble's images")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--cosine", action="store_true", help="cosine learning-rate decay")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default="cnn_weights.npy")
    ap.add_argument("--init", default=None, help="weights (.npy) to continue training from")
    ap.add_argument("--state", default=None,
                    help=".npz holding parameters, Adam moments and progress (read if present, "
                         "written at the end or when --max-seconds stops the run)")
    ap.add_argument("--max-seconds", type=float, default=0.0,
                    help="stop before the next ensemble once this much time has passed")
    ap.add_argument("--first", type=int, default=TRAIN_SEED0, help="first training ensemble")
    ap.add_argument("--evaluate", default=None, help="weights (.npy) to evaluate instead")
    ap.add_argument("--thresholds", default="0.5",
                    help="comma-separated CNN decode thresholds to evaluate")
    ap.add_argument("--workers", type=int, default=4, help="CPU processes for the matching")
    ap.add_argument("--blocks", type=int, default=1,
                    help="slabs per orientation for --evaluate (35: the P = 8 sub-block planes)")
    args = ap.parse_args()
    if args.evaluate:
        thr = tuple(float(x) for x in args.thresholds.split(","))
        res = evaluate(np.load(args.evaluate), args.ensembles, thr, workers=args.workers,
                       blocks=args.blocks)
        suffix = "_eval.json" if args.blocks == 1 else "_eval_slabs.json"
        with open(os.path.splitext(args.evaluate)[0] + suffix, "w") as fh:
            json.dump(res, fh, indent=1)
    else:
        train(args)


if __name__ == "__main__":
    main()
