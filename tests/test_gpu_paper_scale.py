"""Parity at the paper-scale workload, in the launch configuration bench.py
times (128 + 128 elements, 9 angles per orientation, 300 frames of 1024
samples, two 250 x 274 planes, cutoff 20, 9 x 9 NCC, CNN batches of 64).

The full arrays go through the library; the FP64 oracle checks sampled outputs
it can compute in seconds: whole frames of the beamformer, whole planes of the
clutter filter, whole images of the localisers.  Every input is seeded and
synthetic (never a library output)."""
import numpy as np
import pytest

from synth import arrays, cfg_paper, make_medium, with_frames
from oracle import beamform, clutter, cnn, localize
from gpu_util import compare_detections, rel_l2, say

pytestmark = pytest.mark.gpu

SAMPLE_FRAMES = (0, 157, 299)       # first, an interior and the last frame
BEAMFORM_TOL = 1e-4
FILTER_TOL = 2e-5
BF16X3_TOL = 1e-3
POS_TOL = 1e-3


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ulm():
    import paper_2511_21647_amd as u
    return u


@pytest.fixture(scope="module")
def cfg():
    return cfg_paper()


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_paper_beamform_sampled_frames(torch, ulm, cfg):
    """Seeded IQ in three frames of a 300-frame ensemble (zeros elsewhere): the
    projections of those frames against the oracle's two-stage beamformer, and
    exact zeros for a frame without data."""
    ctx = ulm.Context(cfg)
    iq = torch.zeros(ctx.iq_shape, dtype=torch.complex64, device="cuda")
    sub = arrays.complex_normal((len(SAMPLE_FRAMES),) + tuple(ctx.iq_shape[1:]), seed=31)
    for i, f in enumerate(SAMPLE_FRAMES):
        iq[f] = _dev(torch, sub[i], torch.complex64)
    say(f"[paper beamform] frames {SAMPLE_FRAMES} of {tuple(iq.shape)}")
    proj = ulm.rca_beamform_proj(ctx, iq)
    torch.cuda.synchronize()
    got = proj[:, :, list(SAMPLE_FRAMES)].cpu().numpy()
    ref = beamform.beamform_proj(sub.astype(np.complex128), with_frames(cfg, len(SAMPLE_FRAMES)))
    for o in range(2):
        for i, f in enumerate(SAMPLE_FRAMES):
            e = rel_l2(got[o, 0, i], ref[o, 0, i])
            say(f"  plane {o} frame {f}: rel-L2 {e:.2e}")
            assert e <= BEAMFORM_TOL
    assert float(proj[:, :, 1].abs().max().item()) == 0.0


def test_paper_filter_full_planes(torch, ulm, cfg):
    """Both full 68,500 x 300 Casorati planes: the plain filter and the BF16
    split form against the oracle's FP64 eigen route."""
    F, nz, nu, c = cfg.seq.n_frames, cfg.grid.nz, cfg.grid.nu, cfg.svd_cutoff
    x = np.stack([arrays.clutter_stack(nz * nu, F, rank=c, seed=40 + o, decay=0.85)
                  for o in range(2)]).reshape(2, 1, F, nz, nu)
    say(f"[paper filter] {x.shape}, cutoff {c}")
    ref, eig = clutter.filter_planes(x.astype(np.complex128), c)
    for name, prec, tol in (("plain", ulm.ULM_PREC_FP64GRAM, FILTER_TOL),
                            ("bf16x3", ulm.ULM_PREC_BF16X3, BF16X3_TOL)):
        ctx = ulm.Context(cfg, precision=prec)
        d = _dev(torch, x, torch.complex64)
        ev = ulm.svd_clutter_filter(ctx, d)
        ulm.ulm_check_status(ctx)
        got, gev = d.cpu().numpy(), ev.cpu().numpy()
        for o in range(2):
            e = rel_l2(got[o, 0], ref[o, 0])
            ee = np.max(np.abs(gev[o, 0] - eig[o, 0])) / eig[o, 0, 0]
            say(f"  {name} plane {o}: filtered rel-L2 {e:.2e}, eigenvalue err / lambda_1 {ee:.2e}")
            assert e <= tol
            if prec == ulm.ULM_PREC_FP64GRAM:
                assert ee <= 1e-10
        del ctx, d


def test_paper_two_streams_match_one(torch, ulm, cfg):
    """Two contexts on two HIP streams, consecutive paper-scale ensembles
    alternating between them (the eigensolver of one runs beside the other's
    DAS): every context's beamformed-and-filtered planes and eigenvalues equal,
    bit for bit, those of one context running alone."""
    gen = torch.Generator(device="cuda").manual_seed(77)
    ctx0 = ulm.Context(cfg)
    iq = torch.randn(ctx0.iq_shape, dtype=torch.complex64, device="cuda", generator=gen)
    shape = ctx0.proj_shape

    def run(ctx, proj, eig):
        ulm.rca_beamform_stage1(ctx, iq)
        ulm.rca_beamform_stage2(ctx, proj)
        ulm.svd_clutter_filter(ctx, proj, eig)

    ref = torch.empty(shape, dtype=torch.complex64, device="cuda")
    ref_eig = torch.empty(shape[:3], dtype=torch.float64, device="cuda")
    run(ctx0, ref, ref_eig)
    torch.cuda.synchronize()
    ulm.ulm_check_status(ctx0)
    ctxs = [ctx0, ulm.Context(cfg)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [(torch.empty_like(ref), torch.empty_like(ref_eig)) for _ in range(2)]
    for rnd in range(3):
        for k in range(6):
            i = k % 2
            with torch.cuda.stream(streams[i]):
                run(ctxs[i], *outs[i])
        torch.cuda.synchronize()
        for i in range(2):
            ulm.ulm_check_status(ctxs[i])
            same = bool(torch.equal(outs[i][0], ref)) and bool(torch.equal(outs[i][1], ref_eig))
            say(f"[two streams] round {rnd} context {i}: identical to the lone run: {same}")
            assert same


def _spot_frames(F, nz, nu, frames, seed):
    """Filtered-plane stand-ins: isolated Gaussian spots with random phase and a
    weak noise floor in the sampled frames, zeros elsewhere."""
    rng = np.random.default_rng(seed)
    out = np.zeros((2, 1, F, nz, nu), dtype=np.complex64)
    for o in range(2):
        for f in frames:
            img, _ = arrays.gaussian_spots(nz, nu, 60, 1.2, seed * 1000 + o * 500 + f,
                                           spacing=8.0, margin=3)
            amp = img * (0.5 + rng.uniform(0, 1)) + 0.05 * rng.standard_normal((nz, nu))
            out[o, 0, f] = np.abs(amp) * np.exp(1j * rng.uniform(0, 2 * np.pi, (nz, nu)))
    return out


def test_paper_ncc_sampled_frames(torch, ulm, cfg):
    """NCC localisation of the whole 600-image stack; the sampled images'
    detections against the oracle (identical decidable sets, positions within
    1e-3 px), and no detection in an all-zero image."""
    F, nz, nu = cfg.seq.n_frames, cfg.grid.nz, cfg.grid.nu
    x = _spot_frames(F, nz, nu, SAMPLE_FRAMES, seed=52)
    ctx = ulm.Context(cfg)
    cap = 1 << 20
    locs, cnt = ulm.ncc_localize(ctx, _dev(torch, x, torch.complex64), capacity=cap)
    ulm.ulm_check_status(ctx, cnt, cap)
    got = ulm.locs_to_numpy(locs, cnt)
    assert set(int(f) for f in got["frame"]) <= set(SAMPLE_FRAMES)
    sub = x[:, :, list(SAMPLE_FRAMES)]
    ora, N, I = localize.localize(sub.astype(np.complex128), with_frames(cfg, len(SAMPLE_FRAMES)))
    remap = {f: i for i, f in enumerate(SAMPLE_FRAMES)}
    got = got.copy()
    got["frame"] = [remap[int(f)] for f in got["frame"]]
    n, nund, err = compare_detections(got, ora, N, I, with_frames(cfg, len(SAMPLE_FRAMES)),
                                      delta=1e-4, pos_tol=POS_TOL)
    say(f"[paper ncc] matched {n}, undecidable {nund}, max pos err {err:.2e}")
    assert n >= 0.8 * 60 * 2 * len(SAMPLE_FRAMES)


def test_paper_cnn_forward_and_localize(torch, ulm, cfg):
    """The trained network on a full 250 x 274 image: heatmap against the
    oracle's forward pass (BF16 bound), and ulm_cnn_localize over the whole
    stack (64 images per pass) equal to the decode rule on the library's own
    heatmaps for the sampled images."""
    import os
    F, nz, nu = cfg.seq.n_frames, cfg.grid.nz, cfg.grid.nu
    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "paper_2511_21647_amd", "weights", "cnn_paper.npy")
    params = _dev(torch, np.load(wpath), torch.float32)
    x = _spot_frames(F, nz, nu, SAMPLE_FRAMES, seed=61)
    ctx = ulm.Context(cfg)
    filt = _dev(torch, x, torch.complex64)
    images = ulm.ulm_cnn_images(ctx, filt)
    f0 = SAMPLE_FRAMES[1]
    heat = ulm.ulm_cnn_forward(params, images[f0:f0 + 1].contiguous(), ulm.ULM_CNN_BF16)
    torch.cuda.synchronize()
    ref, _ = cnn.forward(ulm.cnn_unpack(params), images[f0].cpu().numpy().astype(np.float64))
    e = rel_l2(heat[0].cpu().numpy(), ref)
    say(f"[paper cnn] heatmap rel-L2 (BF16 vs FP64) {e:.2e}")
    assert e <= 1e-2
    heats = {}
    for o in range(2):
        n = o * F + f0
        heats[o] = ulm.ulm_cnn_forward(params, images[n:n + 1].contiguous(),
                                       ulm.ULM_CNN_BF16)[0].cpu().numpy()
    # a threshold with a few thousand peaks whatever the training state
    thr = float(np.float32(np.quantile(np.stack(list(heats.values())), 0.9995)))
    locs, cnt = ulm.ulm_cnn_localize(ctx, params, filt, capacity=1 << 22, threshold=thr, batch=64)
    ulm.ulm_check_status(ctx, cnt, 1 << 22)
    got = ulm.locs_to_numpy(locs, cnt)
    for o in range(2):
        dec = cnn.decode(heats[o].astype(np.float64), thr)
        mine = got[(got["plane"] == o) & (got["frame"] == f0)]
        want = sorted((int(round((z + 0.5) * cnn.R - 0.5)), int(round((u + 0.5) * cnn.R - 0.5)))
                      for z, u in dec)
        have = sorted((int(round((float(r["z"]) + 0.5) * cnn.R - 0.5)),
                       int(round((float(r["u"]) + 0.5) * cnn.R - 0.5))) for r in mine)
        say(f"  plane {o} frame {f0}: threshold {thr:.4f}, {len(have)} peaks, decode rule {len(want)}")
        assert have == want and len(want) > 0


def match_detections(a, b, radius=0.5):
    """One-to-one matching of two detection lists of one image (arrays of (z, u)),
    closest pairs first, within `radius` px.  Returns the matched distances."""
    if len(a) == 0 or len(b) == 0:
        return np.zeros(0)
    d = np.hypot(a[:, None, 0] - b[None, :, 0], a[:, None, 1] - b[None, :, 1])
    ia, ib = np.nonzero(d <= radius)
    order = np.argsort(d[ia, ib], kind="stable")
    used_a, used_b, out = set(), set(), []
    for t in order:
        i, j = int(ia[t]), int(ib[t])
        if i in used_a or j in used_b:
            continue
        used_a.add(i)
        used_b.add(j)
        out.append(d[i, j])
    return np.array(out)


def test_paper_whole_path_simulated(torch, ulm, cfg):
    """The paper-scale ensemble simulated by the library (2000 MBs on vessels,
    tissue 40 dB above them, rigid motion, noise), through the whole path in the
    launch configuration the bench times, against the oracle at every step:
      - beamformed projections of three sampled frames against the oracle's
        two-stage beamformer of those frames' channel data;
      - both full filtered planes against the oracle's filter of the library's
        own projections: plain form within 2e-5.  The split-precision form
        states its error; here the cutoff falls between two nearly equal
        eigenvalues (lambda_20 / lambda_21 about 1.02, with lambda_1 / lambda_20
        about 4e6), so the clutter subspace moves with any covariance error
        and even an exactly rounded FP32 covariance moves the filtered planes
        by about 1e-2; the split form must do at least as well as that;
      - NCC detections of three sampled frames of both planes against the
        oracle's localiser on the library's filtered planes: identical
        decidable sets, every decidable detection within 1e-3 px (the count
        of undecidable candidates is reported);
      - split-precision form: its NCC detections against the oracle's
        detections on the oracle's FP64-filtered planes, matched one to one
        within 0.5 px: recall >= 0.95 and RMS position error <= 0.1 px."""
    med = make_medium(cfg, 0)
    ctx = ulm.Context(cfg)
    pos = _dev(torch, med.pos, torch.float64)
    amp = torch.from_numpy(med.amp).cuda()
    iq = ulm.ulm_sim_channel_data(ctx, pos, amp, med.noise_seed, med.noise_sigma)
    del pos, amp
    proj = ulm.rca_beamform_proj(ctx, iq)
    torch.cuda.synchronize()
    sub = iq[list(SAMPLE_FRAMES)].cpu().numpy()
    del iq
    say(f"[paper whole path] simulated {med.pos.shape[1]} scatterers, frames {SAMPLE_FRAMES}")
    ref_p = beamform.beamform_proj(sub.astype(np.complex128), with_frames(cfg, len(SAMPLE_FRAMES)))
    p = proj.cpu().numpy()
    for o in range(2):
        e = rel_l2(p[o][:, list(SAMPLE_FRAMES)], ref_p[o])
        say(f"  beamformed plane {o}, sampled frames: rel-L2 {e:.2e}")
        assert e <= BEAMFORM_TOL
    ref_f, eig = clutter.filter_planes(p.astype(np.complex128), cfg.svd_cutoff)
    cut = cfg.svd_cutoff
    fp32_err = []
    for o in range(2):
        # the oracle's filter with its covariance rounded to FP32
        x = clutter.casorati(p[o, 0].astype(np.complex128))
        C32 = (x.conj().T @ x).astype(np.complex64).astype(np.complex128)
        _, V = clutter.clutter_subspace(C32, cut)
        f32 = (x - (x @ V) @ V.conj().T).T.reshape(p[o, 0].shape)
        fp32_err.append(rel_l2(f32, ref_f[o, 0]))
        say(f"  plane {o}: lambda_1/lambda_c {eig[o, 0, 0] / eig[o, 0, cut - 1]:.2e}, "
            f"lambda_c/lambda_c+1 {eig[o, 0, cut - 1] / eig[o, 0, cut]:.4f}; filter with an FP32-rounded "
            f"covariance: rel-L2 {fp32_err[-1]:.2e}")
    forms = {}
    for name, prec, tol in (("plain", ulm.ULM_PREC_FP64GRAM, [FILTER_TOL] * 2),
                            ("bf16x3", ulm.ULM_PREC_BF16X3, fp32_err)):
        c = ctx if prec == ulm.ULM_PREC_FP64GRAM else ulm.Context(cfg, precision=prec)
        d = proj.clone()
        ulm.svd_clutter_filter(c, d)
        ulm.ulm_check_status(c)
        locs, cnt = ulm.ncc_localize(c, d, capacity=4_000_000)
        ulm.ulm_check_status(c, cnt, 4_000_000)
        f = d.cpu().numpy()
        for o in range(2):
            e = rel_l2(f[o, 0], ref_f[o, 0])
            say(f"  {name} filtered plane {o}: rel-L2 {e:.2e} against the oracle's filter")
            assert e <= tol[o]
        forms[name] = (f, ulm.locs_to_numpy(locs, cnt))
        del d
    # plain NCC against the oracle on the library's filtered planes
    f, got = forms["plain"]
    fr = list(SAMPLE_FRAMES)
    ora, N, I = localize.localize(f[:, :, fr].astype(np.complex128), cfg)
    sel = got[np.isin(got["frame"], fr)].copy()
    sel["frame"] = np.searchsorted(np.array(fr), sel["frame"])
    n, nund, err = compare_detections(sel, ora, N, I, cfg, 1e-5, POS_TOL)
    say(f"  plain NCC, {len(fr)} frames x 2 planes: {n} decidable detections identical, "
        f"{nund} undecidable, max position error {err:.1e} px")
    # split-precision form against the oracle's FP64 chain
    ora64, _, _ = localize.localize(ref_f[:, :, fr], cfg)
    _, gotb = forms["bf16x3"]
    nm = no = ng = 0
    d2 = []
    for o in range(2):
        for i, fi in enumerate(fr):
            a = ora64[(ora64["plane"] == o) & (ora64["frame"] == i)]
            b = gotb[(gotb["plane"] == o) & (gotb["frame"] == fi)]
            m = match_detections(np.stack([a["z"], a["u"]], 1), np.stack([b["z"], b["u"]], 1))
            nm += len(m)
            no += len(a)
            ng += len(b)
            d2 += list(m ** 2)
    recall, precision = nm / max(no, 1), nm / max(ng, 1)
    rms = float(np.sqrt(np.mean(d2))) if d2 else 0.0
    say(f"  bf16x3 NCC vs the FP64 oracle chain: recall {recall:.4f}, precision {precision:.4f}, "
        f"RMS {rms:.2e} px over {nm} matched of {no} oracle detections")
    assert recall >= 0.95
    assert rms <= 0.1
