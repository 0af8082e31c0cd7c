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

    def __init__(self, precision=None):
        import torch
        import paper_2511_21647_amd as ulm
        from synth import cfg_cnn
        self.torch, self.ulm = torch, ulm
        self.cfg = cfg_cnn(2000)
        prec = ulm.ULM_PREC_BF16X3 if precision is None else precision
        self.ctx = ulm.Context(self.cfg, precision=prec)
        self.iq = torch.empty(self.ctx.iq_shape, dtype=torch.complex64, device="cuda")
        self.proj = torch.empty(self.ctx.proj_shape, dtype=torch.complex64, device="cuda")

    def ensemble(self, e: int):
        from synth import cfg_cnn, make_medium, plane_positions
        torch, ulm = self.torch, self.ulm
        cfg = cfg_cnn(n_mb_for(e))
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
    pairs first.  Returns (pairs det_i, ref_j)."""
    if len(det) == 0 or len(ref) == 0:
        return np.zeros(0, int), np.zeros(0, int)
    from scipy.spatial import cKDTree
    tree = cKDTree(ref)
    pairs = tree.query_ball_point(det, r=radius)
    cand = [(np.hypot(*(det[i] - ref[j])), i, j) for i, js in enumerate(pairs) for j in js]
    cand.sort()
    used_d, used_r, di, rj = set(), set(), [], []
    for _, i, j in cand:
        if i in used_d or j in used_r:
            continue
        used_d.add(i)
        used_r.add(j)
        di.append(i)
        rj.append(j)
    return np.array(di, int), np.array(rj, int)


def per_image(recs, n_img, F):
    out = [[] for _ in range(n_img)]
    for r in recs:
        out[int(r["plane"]) * F + int(r["frame"])].append((float(r["z"]), float(r["u"])))
    return [np.array(o).reshape(-1, 2) for o in out]


def score(dets, truth, radius=0.5):
    n_det = n_ref = n_match = 0
    sq = []
    for d, t in zip(dets, truth):
        i, j = match(d, t, radius)
        n_det += len(d)
        n_ref += len(t)
        n_match += len(i)
        if len(i):
            sq.append(np.sum((d[i] - t[j]) ** 2, axis=1))
    sq = np.concatenate(sq) if sq else np.zeros(0)
    return {"recall": n_match / max(n_ref, 1), "precision": n_match / max(n_det, 1),
            "rms_px": float(np.sqrt(sq.mean())) if sq.size else float("nan"),
            "n_det": n_det, "n_ref": n_ref, "n_match": n_match}


def evaluate(weights, ensembles, thresholds=(0.5,), seed0=HELDOUT_SEED0, log_fn=log):
    """NCC and CNN on held-out ensembles: each against the truth, and the CNN
    against NCC as the judge, for every CNN decode threshold given."""
    import torch
    import paper_2511_21647_amd as ulm
    sim = Simulator()
    cfg = sim.cfg
    F = cfg.seq.n_frames
    n_img = 2 * F
    params = torch.from_numpy(np.asarray(weights, np.float32)).cuda()
    cap = 4_000_000
    locs = torch.empty((cap, 8), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    cws = ulm.Workspace(ulm.ulm_cnn_localize_workspace_size(sim.ctx, 64), "cuda")
    results = []
    for i in range(ensembles):
        e = seed0 + i
        _, labels, n_mb = sim.ensemble(e)
        truth = [labels[n // F][n % F] for n in range(n_img)]
        ulm.ncc_localize(sim.ctx, sim.proj, cap, locs, count)
        ulm.ulm_check_status(sim.ctx, count, cap)
        ncc = per_image(ulm.locs_to_numpy(locs, count), n_img, F)
        r = {"ensemble": e, "n_mb": n_mb, "ncc_vs_truth": score(ncc, truth), "cnn": {}}
        for thr in thresholds:
            ulm.ulm_cnn_localize(sim.ctx, params, sim.proj, cap, thr, 64, ulm.ULM_CNN_BF16,
                                 locs, count, ws=cws)
            ulm.ulm_check_status(sim.ctx, count, cap)
            cnn = per_image(ulm.locs_to_numpy(locs, count), n_img, F)
            r["cnn"][str(thr)] = {"vs_truth": score(cnn, truth), "vs_ncc": score(cnn, ncc)}
        results.append(r)
        log_fn(json.dumps(r))
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
    args = ap.parse_args()
    if args.evaluate:
        thr = tuple(float(x) for x in args.thresholds.split(","))
        res = evaluate(np.load(args.evaluate), args.ensembles, thr)
        with open(os.path.splitext(args.evaluate)[0] + "_eval.json", "w") as fh:
            json.dump(res, fh, indent=1)
    else:
        train(args)


if __name__ == "__main__":
    main()
