"""GPU parity of the learned localiser through the C ABI against the FP64 CNN
oracle: forward heatmaps, loss and every parameter gradient, the Adam update,
and the fused head + decode against the decode rule applied to the GPU's own
heatmap.  Image sizes are ragged in both tiled axes (21 x 37: 4-row and
32-column tiles)."""
import numpy as np
import pytest

from synth import arrays
from oracle import cnn
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu

# FP32 activations: accumulation-order rounding only.  BF16 activations and
# weights: 8-bit mantissas (relative rounding 2^-9 per stored value).
FWD_TOL = {"fp32": 1e-5, "bf16": 1e-2}
GRAD_TOL = {"fp32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ulm():
    import paper_2511_21647_amd as u
    return u


def _prec(ulm, name):
    return ulm.ULM_CNN_FP32 if name == "fp32" else ulm.ULM_CNN_BF16


def _params(seed):
    g = np.random.default_rng(seed)
    p = cnn.init_params(g)
    for k in p:
        if k.startswith("b"):
            p[k] = p[k] + 0.05 * g.standard_normal(p[k].shape)
    return p


def _images(B, H, W, seed):
    """Envelope-like inputs: isolated Gaussian spots plus a weak uniform floor,
    scaled to a maximum of 1; returns (images [B][H][W], labels [(n, z, u)])."""
    imgs, labels = [], []
    for n in range(B):
        im, centres = arrays.gaussian_spots(H, W, 4, 1.2, seed + n, spacing=5.0, margin=2)
        im = im + 0.05 * arrays.rng(seed + 100 + n).uniform(0, 1, im.shape)
        imgs.append(im / im.max())
        labels += [(n, c[0], c[1]) for c in centres]
    return np.stack(imgs), labels


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cnn_forward_parity(torch, ulm, prec):
    B, H, W = 3, 21, 37
    say(f"[cnn forward {prec}] B={B} H={H} W={W}")
    p = _params(1)
    x, _ = _images(B, H, W, 10)
    params = _dev(torch, ulm.cnn_pack(p), torch.float32)
    heat = ulm.ulm_cnn_forward(params, _dev(torch, x, torch.float32), _prec(ulm, prec))
    torch.cuda.synchronize()
    got = heat.cpu().numpy()
    for n in range(B):
        ref, _ = cnn.forward(p, x[n])
        e = rel_l2(got[n], ref)
        say(f"  image {n}: heat rel-L2 {e:.2e}")
        assert e <= FWD_TOL[prec]


@pytest.mark.parametrize("prec,case", [("fp32", "spots"), ("bf16", "spots"), ("fp32", "empty")])
def test_cnn_gradient_parity(torch, ulm, prec, case):
    B, H, W = 3, 21, 37
    say(f"[cnn gradients {prec} {case}] B={B} H={H} W={W}")
    p = _params(2)
    x, labels = _images(B, H, W, 20)
    if case == "empty":
        labels = []
    # oracle: mean over the batch of the per-image loss and gradients
    loss_ref, grads_ref = 0.0, {k: np.zeros_like(v) for k, v in p.items()}
    for n in range(B):
        pos = np.array([[z, u] for (m, z, u) in labels if m == n]).reshape(-1, 2)
        T = cnn.target_map(pos, H, W)
        l, g = cnn.loss_and_grad(p, x[n], T)
        loss_ref += l / B
        for k in g:
            grads_ref[k] += g[k] / B
    params = _dev(torch, ulm.cnn_pack(p), torch.float32)
    if labels:
        zu = _dev(torch, np.array([[z, u] for (_, z, u) in labels]), torch.float32)
        img = _dev(torch, np.array([n for (n, _, _) in labels]), torch.int32)
    else:
        zu = img = None
    loss, grad = ulm.ulm_cnn_gradients(params, _dev(torch, x, torch.float32), zu, img,
                                       _prec(ulm, prec))
    torch.cuda.synchronize()
    el = abs(float(loss.item()) - loss_ref) / loss_ref
    say(f"  loss {float(loss.item()):.6e} vs {loss_ref:.6e} (rel {el:.2e})")
    assert el <= FWD_TOL[prec]
    got = ulm.cnn_unpack(grad)
    worst = 0.0
    for k in grads_ref:
        e = rel_l2(got[k], grads_ref[k])
        worst = max(worst, e)
        say(f"  grad {k:3s} rel-L2 {e:.2e}")
    assert worst <= GRAD_TOL[prec]


def test_cnn_adam_matches_oracle(torch, ulm):
    """Two training steps: the parameters after each equal the oracle's Adam
    update applied to the gradients the library computed."""
    B, H, W = 2, 21, 37
    p = _params(3)
    x, labels = _images(B, H, W, 30)
    xs = _dev(torch, x, torch.float32)
    zu = _dev(torch, np.array([[z, u] for (_, z, u) in labels]), torch.float32)
    img = _dev(torch, np.array([n for (n, _, _) in labels]), torch.int32)
    prec = ulm.ULM_CNN_FP32
    params = _dev(torch, ulm.cnn_pack(p), torch.float32)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = ulm.Workspace(ulm.ulm_cnn_workspace_size(B, H, W, prec, True), "cuda")
    ref = {k: a.copy() for k, a in ulm.cnn_unpack(params).items()}
    state = {}
    lr = 1e-3
    for step in (1, 2):
        _, grad = ulm.ulm_cnn_gradients(params, xs, zu, img, prec, ws=ws)
        g = ulm.cnn_unpack(grad)
        ulm.ulm_cnn_train_step(params, m, v, step, lr, xs, zu, img, prec, ws=ws)
        torch.cuda.synchronize()
        cnn.adam_step(ref, g, state, lr=lr)
        got = ulm.cnn_unpack(params)
        err = max(float(np.abs(got[k] - ref[k]).max()) for k in ref)
        say(f"[cnn adam] step {step}: max |param - oracle| {err:.2e}")
        assert err <= 1e-6


def _filtered_tiny(torch, ulm, cfg, iq):
    ctx = ulm.Context(cfg)
    out = ulm.ulm_reconstruct_ensemble(ctx, _dev(torch, iq, torch.complex64), capacity=1 << 16)
    return ctx, out["proj"]


def _expected_records(heat, thr, F, W):
    """Decode rule on the GPU heatmaps, in the library's output order."""
    R = cnn.R
    rows = []
    for n in range(heat.shape[0]):
        for z, u in cnn.decode(heat[n].astype(np.float64), thr):
            qz, qu = int(round((z + 0.5) * R - 0.5)), int(round((u + 0.5) * R - 0.5))
            rows.append((n // F, n % F, qz // R, qu // R, qz, qu, z, u, heat[n][qz, qu]))
    rows.sort(key=lambda r: r[:6])
    return rows


def _row_threshold(heat, F, W):
    """The lowest of a few high quantiles of the heat whose peaks fit every
    row's staging slot (random weights give noisy heatmaps with many maxima)."""
    cap = max(16, (W + 1) // 2)
    for q in (0.998, 0.999, 0.9995, 0.9998, 0.9999):
        thr = float(np.float32(np.quantile(heat, q)))
        exp = _expected_records(heat, thr, F, W)
        rows = {}
        for x in exp:
            rows[x[:3]] = rows.get(x[:3], 0) + 1
        if exp and max(rows.values()) <= cap:
            return thr, exp
    raise AssertionError("no threshold keeps every row within its slot")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cnn_localize_matches_decode(torch, ulm, prec, tiny_cfg, tiny_iq):
    """ulm_cnn_localize (fused head + decode, 7 images per pass) equals the
    decode rule applied to ulm_cnn_forward's heatmaps, record for record."""
    cfg = tiny_cfg
    say(f"[cnn localize {prec}] tiny ensemble")
    ctx, filt = _filtered_tiny(torch, ulm, cfg, tiny_iq)
    images = ulm.ulm_cnn_images(ctx, filt)
    torch.cuda.synchronize()
    env = np.abs(filt.cpu().numpy()).reshape(images.shape)
    ref_img = env / env.reshape(env.shape[0], -1).max(axis=1)[:, None, None]
    e = float(np.abs(images.cpu().numpy() - ref_img).max())
    say(f"  images max abs err {e:.2e}")
    assert e <= 1e-6
    params = _dev(torch, ulm.cnn_pack(_params(4)), torch.float32)
    pr = _prec(ulm, prec)
    heat = ulm.ulm_cnn_forward(params, images, pr).cpu().numpy()
    F, W = cfg.seq.n_frames, cfg.grid.nu
    thr, exp = _row_threshold(heat, F, W)
    locs, count = ulm.ulm_cnn_localize(ctx, params, filt, capacity=1 << 16, threshold=thr, batch=7,
                                       precision=pr)
    ulm.ulm_check_status(ctx, count, 1 << 16)
    got = ulm.locs_to_numpy(locs, count)
    say(f"  threshold {thr:.4f}: {len(exp)} expected, {len(got)} found")
    assert len(got) == len(exp) > 0
    for r, x in zip(got, exp):
        assert (int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"])) == x[:4]
        assert float(r["z"]) == x[6] and float(r["u"]) == x[7]
        assert np.float32(r["ncc"]) == np.float32(x[8])
        pz = env[int(r["plane"]) * F + int(r["frame"]), int(r["iz"]), int(r["iu"])]
        assert abs(float(r["intensity"]) - pz) <= 1e-6 * max(pz, 1e-30)


@pytest.mark.parametrize("nz,nu", [(101, 45), (50, 1), (7, 130), (113, 2)])
def test_cnn_localize_fused_strips(torch, ulm, tiny_cfg, nz, nu):
    """The BF16 localiser runs every layer of a strip of rows in one work-group,
    column by column.  On random complex planes of ragged sizes (strips of 34,
    50, 7 and 38 rows; one, two, 45 and 130 columns) its records equal the
    decode rule applied to the layer-by-layer BF16 heatmaps, record for record,
    intensities and all."""
    from dataclasses import replace
    cfg = tiny_cfg
    g = cfg.grid
    cfg = cfg.with_(grid=replace(g, nz=nz, nu=nu, nv=max(nu, 2), n_blocks=2, v0=g.u0))
    cfg = cfg.with_(seq=replace(cfg.seq, n_frames=3))
    ctx = ulm.Context(cfg)
    rng = np.random.default_rng(nz * 1000 + nu)
    shape = ctx.proj_shape
    planes = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    planes[0, 0, 1] *= 0.0                       # an all-zero image: frame maximum 0
    filt = _dev(torch, planes, torch.complex64)
    images = ulm.ulm_cnn_images(ctx, filt)
    params = _dev(torch, ulm.cnn_pack(_params(6)), torch.float32)
    heat = ulm.ulm_cnn_forward(params, images, ulm.ULM_CNN_BF16).cpu().numpy()
    F = cfg.seq.n_frames
    thr, exp = _row_threshold(heat, F, nu)
    say(f"[cnn fused {nz}x{nu}] threshold {thr:.4f}, {len(exp)} expected")
    locs, count = ulm.ulm_cnn_localize(ctx, params, filt, capacity=1 << 16, threshold=thr,
                                       precision=ulm.ULM_CNN_BF16)
    ulm.ulm_check_status(ctx, count, 1 << 16)
    got = ulm.locs_to_numpy(locs, count)
    assert len(got) == len(exp) > 0
    env = np.abs(planes.reshape(-1, nz, nu))
    for r, x in zip(got, exp):
        assert (int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"])) == x[:4]
        assert float(r["z"]) == x[6] and float(r["u"]) == x[7]
        assert np.float32(r["ncc"]) == np.float32(x[8])
        pz = env[int(r["plane"]) * F + int(r["frame"]), int(r["iz"]), int(r["iu"])]
        assert abs(float(r["intensity"]) - pz) <= 1e-6 * max(pz, 1e-30)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cnn_whole_path_entry(torch, ulm, prec, tiny_cfg, tiny_iq):
    """ulm_reconstruct_ensemble_cnn equals beamforming, filtering and
    ulm_cnn_localize called one by one: the same filtered planes and the same
    records, bit for bit; its timing covers the three stages."""
    cfg = tiny_cfg
    ctx = ulm.Context(cfg)
    d = _dev(torch, tiny_iq, torch.complex64)
    params = _dev(torch, ulm.cnn_pack(_params(4)), torch.float32)
    pr = _prec(ulm, prec)
    proj = ulm.rca_beamform_proj(ctx, d)
    ulm.svd_clutter_filter(ctx, proj)
    heat = ulm.ulm_cnn_forward(params, ulm.ulm_cnn_images(ctx, proj), pr).cpu().numpy()
    thr, _ = _row_threshold(heat, cfg.seq.n_frames, cfg.grid.nu)
    out = ulm.ulm_reconstruct_ensemble_cnn(ctx, d, params, 1 << 16, threshold=thr, batch=7,
                                           precision=pr, timing=True)
    ulm.ulm_check_status(ctx, out["count"], 1 << 16)
    got = ulm.locs_to_numpy(out["locs"], out["count"]).copy()
    locs, count = ulm.ulm_cnn_localize(ctx, params, proj, 1 << 16, threshold=thr, batch=7, precision=pr)
    ulm.ulm_check_status(ctx, count, 1 << 16)
    ref = ulm.locs_to_numpy(locs, count)
    say(f"[cnn whole path {prec}] {len(got)} records, timing {out['timing']}")
    assert len(got) > 0
    assert torch.equal(out["proj"].view(torch.float32), proj.view(torch.float32))
    assert got.tobytes() == ref.tobytes()
    t = out["timing"]
    assert t["total"] >= t["beamform"] + t["filter"] + t["localize"] - 1e-3
    with pytest.raises(ulm.ULMError) as ei:
        ulm.ulm_reconstruct_ensemble_cnn(ctx, d, params, 1 << 16, threshold=float("inf"), precision=pr)
    assert ei.value.code == ulm.ULM_ERR_INVALID_ARG


def test_cnn_row_overflow_flag(torch, ulm, tiny_cfg, tiny_iq):
    """A threshold below every heat value floods the per-row staging: the call
    keeps the first peaks of each row and ulm_check_status reports OVERFLOW
    exactly when some row exceeds its slot."""
    cfg = tiny_cfg
    ctx, filt = _filtered_tiny(torch, ulm, cfg, tiny_iq)
    params = _dev(torch, ulm.cnn_pack(_params(5)), torch.float32)
    images = ulm.ulm_cnn_images(ctx, filt)
    heat = ulm.ulm_cnn_forward(params, images, ulm.ULM_CNN_BF16).cpu().numpy()
    F, W = cfg.seq.n_frames, cfg.grid.nu
    exp = _expected_records(heat, -1e29, F, W)
    per_row = {}
    for x in exp:
        per_row[(x[0], x[1], x[2])] = per_row.get((x[0], x[1], x[2]), 0) + 1
    cap = max(16, (W + 1) // 2)
    over = max(per_row.values()) > cap
    say(f"[cnn overflow] max peaks per row {max(per_row.values())}, slot {cap}")
    locs, count = ulm.ulm_cnn_localize(ctx, params, filt, capacity=1 << 18, threshold=-1e29)
    if over:
        with pytest.raises(ulm.ULMError) as ei:
            ulm.ulm_check_status(ctx, count, 1 << 18)
        assert ei.value.code == -3
    else:
        ulm.ulm_check_status(ctx, count, 1 << 18)
    kept = {}
    for x in exp:
        k = (x[0], x[1], x[2])
        kept[k] = kept.get(k, 0) + 1
    n_exp = sum(min(c, cap) for c in kept.values())
    assert int(count.item()) == n_exp
    # a later call whose rows all fit clears the flag
    thr, exp = _row_threshold(heat, F, W)
    ulm.ulm_cnn_localize(ctx, params, filt, capacity=1 << 18, threshold=thr, count=count)
    ulm.ulm_check_status(ctx, count, 1 << 18)
    assert int(count.item()) == len(exp)


def test_cnn_training_reduces_loss(torch, ulm):
    """60 BF16 Adam steps on spot images cut the batch loss at least fivefold."""
    B, H, W = 4, 32, 48
    p = _params(6)
    params = _dev(torch, ulm.cnn_pack(p), torch.float32)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    prec = ulm.ULM_CNN_BF16
    ws = ulm.Workspace(ulm.ulm_cnn_workspace_size(B, H, W, prec, True), "cuda")
    losses = []
    for step in range(1, 61):
        x, labels = _images(B, H, W, 1000 + 10 * step)
        zu = _dev(torch, np.array([[z, u] for (_, z, u) in labels]), torch.float32)
        img = _dev(torch, np.array([n for (n, _, _) in labels]), torch.int32)
        loss = ulm.ulm_cnn_train_step(params, m, v, step, 2e-3, _dev(torch, x, torch.float32), zu,
                                      img, prec, ws=ws)
        losses.append(float(loss.item()))
    say(f"[cnn training] loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.all(np.isfinite(losses))
    assert np.mean(losses[-5:]) <= losses[0] / 5
