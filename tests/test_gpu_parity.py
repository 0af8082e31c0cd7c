"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same
seeded inputs (tiny and ragged sizes spanning several tiles)."""
from dataclasses import replace

import numpy as np
import pytest

from synth import arrays, cfg_tiny, make_medium, with_angles, with_blocks, with_frames
from oracle import beamform, clutter, localize, pipeline, sim
from gpu_util import compare_detections, rel_l2, say

pytestmark = pytest.mark.gpu

BEAMFORM_TOL = 1e-4        # relative L2 of projections (plain FP32 path)
FILTER_TOL = 2e-5          # relative L2 of filtered planes, shared FP32 input
POS_TOL = 1e-3             # pixel


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ulm():
    import paper_2511_21647_amd as u
    return u


def _to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _ragged_cfg():
    """Ragged in every tiled axis: 37 x 45 plane, 18 frames, 4 blocks, 5 angles incl. 0."""
    c = with_blocks(with_angles(with_frames(cfg_tiny(), 18), [-6, -2, 0, 3, 6]), 4)
    g = c.grid
    return c.with_(grid=replace(g, nu=45, nz=37, u0=-22 * g.du, nv=45, v0=-22 * g.dv))


@pytest.mark.parametrize("case", ["tiny", "ragged"])
def test_beamform_parity(torch, ulm, case, tiny_cfg, tiny_iq):
    if case == "tiny":
        cfg, iq = tiny_cfg, tiny_iq
    else:
        cfg = _ragged_cfg()
        iq = sim.simulate(cfg, make_medium(cfg, 3))
    say(f"[beamform {case}] iq {iq.shape}")
    ref = beamform.beamform_proj(iq, cfg)
    ctx = ulm.Context(cfg)
    proj = ulm.rca_beamform_proj(ctx, _to_dev(torch, iq, torch.complex64))
    torch.cuda.synchronize()
    got = proj.cpu().numpy()
    for o in range(2):
        for b in range(cfg.grid.n_blocks):
            e = rel_l2(got[o, b], ref[o, b])
            say(f"  plane o={o} b={b} rel-L2 {e:.2e}")
            assert e <= BEAMFORM_TOL


def test_beamform_record_edges(torch, ulm, tiny_cfg):
    """Receive windows that cross both ends of the record.  On the tiny geometry
    the echoes arrive 5.2-14.2 us after transmit (4-10 mm depth, 6.4 mm aperture);
    a record from 7 us to 13.7 us misses the shallowest and the deepest, so the
    staging of those windows must read zeros outside the record, as the oracle's
    interpolation does."""
    sq = tiny_cfg.seq
    cfg = tiny_cfg.with_(seq=replace(sq, t_start=7.0e-6, n_samp=160))
    iq = sim.simulate(cfg, make_medium(cfg, 5))
    say(f"[beamform record edges] iq {iq.shape}")
    ref = beamform.beamform_proj(iq, cfg)
    ctx = ulm.Context(cfg)
    proj = ulm.rca_beamform_proj(ctx, _to_dev(torch, iq, torch.complex64))
    torch.cuda.synchronize()
    got = proj.cpu().numpy()
    for o in range(2):
        e = rel_l2(got[o, 0], ref[o, 0])
        say(f"  plane o={o} rel-L2 {e:.2e}")
        assert e <= BEAMFORM_TOL


def test_beamform_wide_window(torch, ulm, tiny_cfg):
    """Sampled at 40 MHz, a tile of the tiny grid spans more than 64 and fewer than
    128 samples (the span grows by about 2.2 samples per MHz there; 60 MHz gives
    132 and is refused), so stage 1 stages 128-sample windows: two runs of four
    samples per thread instead of one."""
    pr, sq = tiny_cfg.probe, tiny_cfg.seq
    cfg = tiny_cfg.with_(probe=replace(pr, fs=40e6), seq=replace(sq, n_samp=432))
    iq = sim.simulate(cfg, make_medium(cfg, 6))
    say(f"[beamform 40 MHz] iq {iq.shape}")
    ref = beamform.beamform_proj(iq, cfg)
    ctx = ulm.Context(cfg)
    proj = ulm.rca_beamform_proj(ctx, _to_dev(torch, iq, torch.complex64))
    torch.cuda.synchronize()
    got = proj.cpu().numpy()
    for o in range(2):
        e = rel_l2(got[o, 0], ref[o, 0])
        say(f"  plane o={o} rel-L2 {e:.2e}")
        assert e <= BEAMFORM_TOL


def _filter_input(F, nz, nu, seed):
    st = np.stack([arrays.clutter_stack(nz * nu, F, rank=6, seed=seed + o) for o in range(2)])
    return st.reshape(2, 1, F, nz, nu)


# cutoffs 2, 3, 12 and 29 cover one to four 16-row tiles of the removal's 2c rows;
# frames and pixels ragged against its 8-frame and 32-pixel tiles
@pytest.mark.parametrize("F,nz,nu,c", [(20, 16, 20, 2), (70, 64, 70, 3), (130, 40, 37, 12),
                                       (45, 24, 27, 29)])
def test_filter_parity(torch, ulm, F, nz, nu, c):
    cfg = with_frames(cfg_tiny(), F)
    cfg = cfg.with_(svd_cutoff=c, grid=replace(cfg.grid, nz=nz, nu=nu, nv=nu))
    x = _filter_input(F, nz, nu, seed=100 + F)
    say(f"[filter F={F} {nz}x{nu} c={c}]")
    ref, eig = clutter.filter_planes(x.astype(np.complex128), c)
    ctx = ulm.Context(cfg)
    d = _to_dev(torch, x, torch.complex64)
    ev = ulm.svd_clutter_filter(ctx, d)
    ulm.ulm_check_status(ctx)
    got = d.cpu().numpy()
    gev = ev.cpu().numpy()
    for o in range(2):
        e = rel_l2(got[o, 0], ref[o, 0])
        ee = np.max(np.abs(gev[o, 0] - eig[o, 0])) / eig[o, 0, 0]
        say(f"  plane {o}: filtered rel-L2 {e:.2e}, eigenvalues max err / lambda_1 {ee:.2e}")
        assert e <= FILTER_TOL
        assert ee <= 1e-10


def test_filter_cutoff_zero_is_identity(torch, ulm):
    cfg = with_frames(cfg_tiny(), 12).with_(svd_cutoff=0)
    x = _filter_input(12, 64, 64, seed=5)
    ctx = ulm.Context(cfg)
    d = _to_dev(torch, x, torch.complex64)
    ulm.svd_clutter_filter(ctx, d)
    ulm.ulm_check_status(ctx)
    assert np.array_equal(d.cpu().numpy(), x)


def test_filter_store_modes_agree(torch, ulm, monkeypatch):
    """The eigensolver's two cross-work-group exchange modes (plain stores into
    the shared L2 of one XCD; agent-scope stores with release and acquire
    fences at every barrier) do the same arithmetic, so the filtered planes
    and eigenvalues agree bit for bit."""
    F, nz, nu, c = 130, 40, 37, 12
    cfg = with_frames(cfg_tiny(), F)
    cfg = cfg.with_(svd_cutoff=c, grid=replace(cfg.grid, nz=nz, nu=nu, nv=nu))
    x = _filter_input(F, nz, nu, seed=310)
    ctx = ulm.Context(cfg)
    out = []
    for fenced in (False, True):
        if fenced:
            monkeypatch.setenv("ULMPROJ_EIGEN_AGENT_SCOPE", "1")
        else:
            monkeypatch.delenv("ULMPROJ_EIGEN_AGENT_SCOPE", raising=False)
        d = _to_dev(torch, x, torch.complex64)
        ev = ulm.svd_clutter_filter(ctx, d)
        ulm.ulm_check_status(ctx)
        out.append((d.cpu().numpy(), ev.cpu().numpy()))
    say(f"[filter exchange modes] F={F}: planes equal {np.array_equal(out[0][0], out[1][0])}, "
        f"eigenvalues equal {np.array_equal(out[0][1], out[1][1])}")
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("F,nz,nu,c,rank", [(70, 64, 70, 3, 6), (37, 29, 33, 17, 17),
                                            (300, 16, 20, 20, 20)])
def test_filter_bf16x3_error(torch, ulm, F, nz, nu, c, rank):
    """Split-precision form (BF16 split Gram and removal on MFMA): states its
    error against the FP64 oracle.  Ragged in frames (not a multiple of 8 or
    32), pixels (not a multiple of 32) and cutoff (one or two 32-row tiles of
    the 2c real rows)."""
    cfg = with_frames(cfg_tiny(), F)
    cfg = cfg.with_(svd_cutoff=c, grid=replace(cfg.grid, nz=nz, nu=nu, nv=nu))
    # clutter modes decaying slowly enough that the cutoff mode stays well above
    # the blood part's singular values
    x = np.stack([arrays.clutter_stack(nz * nu, F, rank=rank, seed=300 + o, decay=0.85)
                  for o in range(2)]).reshape(2, 1, F, nz, nu)
    ref, eig = clutter.filter_planes(x.astype(np.complex128), c)
    ctx = ulm.Context(cfg, precision=ulm.ULM_PREC_BF16X3)
    d = _to_dev(torch, x, torch.complex64)
    ulm.svd_clutter_filter(ctx, d)
    ulm.ulm_check_status(ctx)
    got = d.cpu().numpy()
    for o in range(2):
        e = rel_l2(got[o, 0], ref[o, 0])
        say(f"  bf16x3 F={F} {nz}x{nu} c={c} plane {o}: filtered rel-L2 {e:.2e}")
        assert e <= 1e-3


def _spot_planes(F, nz, nu, seed, n_spots=12, noise=0.05):
    rng = np.random.default_rng(seed)
    out = np.zeros((2, 1, F, nz, nu), dtype=np.complex64)
    for o in range(2):
        for f in range(F):
            img, _ = arrays.gaussian_spots(nz, nu, n_spots, 1.2, seed * 1000 + o * 100 + f,
                                           spacing=6.0, margin=2)
            amp = img * (0.5 + rng.uniform(0, 1)) + noise * rng.standard_normal((nz, nu))
            out[o, 0, f] = (np.abs(amp) * np.exp(1j * rng.uniform(0, 2 * np.pi, (nz, nu))))
    return out


@pytest.mark.parametrize("F,nz,nu,size", [(3, 40, 50, 7), (4, 53, 61, 9), (2, 33, 29, 11)])
def test_ncc_parity(torch, ulm, F, nz, nu, size):
    cfg = with_frames(cfg_tiny(), F)
    cfg = cfg.with_(grid=replace(cfg.grid, nz=nz, nu=nu, nv=nu),
                    loc=replace(cfg.loc, ncc_size=size))
    x = _spot_planes(F, nz, nu, seed=F * 7 + size)
    ora, N, I = localize.localize(x.astype(np.complex128), cfg)
    ctx = ulm.Context(cfg)
    locs, cnt = ulm.ncc_localize(ctx, _to_dev(torch, x, torch.complex64), capacity=100000)
    ulm.ulm_check_status(ctx, cnt, 100000)
    got = ulm.locs_to_numpy(locs, cnt)
    n, nund, err = compare_detections(got, ora, N, I, cfg, delta=1e-4, pos_tol=POS_TOL)
    say(f"[ncc {nz}x{nu} size {size}] matched {n}, undecidable {nund}, max pos err {err:.2e}")
    assert n > 10 * F
    # NCC and intensity values agree for matched records
    g = {(int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"])): r for r in got}
    for r in ora:
        k = (int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"]))
        if k in g:
            assert abs(g[k]["ncc"] - r["ncc"]) < 1e-5
            assert abs(g[k]["intensity"] - r["intensity"]) <= 1e-6 * r["intensity"]


def test_ncc_parity_wide_plane(torch, ulm):
    """Planes wider than the register-column kernel's limit (input band plus
    halo over 512 columns) take the LDS band kernel: 512 columns with a 7x7
    template (520 input columns; the widest plane whose band fits the LDS is
    517 columns), ragged rows."""
    F, nz, nu, size = 2, 21, 512, 7
    cfg = with_frames(cfg_tiny(), F)
    cfg = cfg.with_(grid=replace(cfg.grid, nz=nz, nu=nu, nv=nu, u0=-(nu - 1) / 2 * cfg.grid.du,
                                 v0=-(nu - 1) / 2 * cfg.grid.du),
                    loc=replace(cfg.loc, ncc_size=size))
    x = _spot_planes(F, nz, nu, seed=501, n_spots=40)
    ora, N, I = localize.localize(x.astype(np.complex128), cfg)
    ctx = ulm.Context(cfg)
    locs, cnt = ulm.ncc_localize(ctx, _to_dev(torch, x, torch.complex64), capacity=100000)
    ulm.ulm_check_status(ctx, cnt, 100000)
    got = ulm.locs_to_numpy(locs, cnt)
    n, nund, err = compare_detections(got, ora, N, I, cfg, delta=1e-4, pos_tol=POS_TOL)
    say(f"[ncc wide {nz}x{nu} size {size}] matched {n}, undecidable {nund}, max pos err {err:.2e}")
    assert n > 10 * F


def test_filter_parity_many_frames(torch, ulm):
    """More than 512 frames take the single-work-group eigensolver: 520 frames
    of a 9 x 13 plane, cutoff 3."""
    F, nz, nu, c = 520, 9, 13, 3
    cfg = with_frames(cfg_tiny(), F)
    cfg = cfg.with_(svd_cutoff=c, grid=replace(cfg.grid, nz=nz, nu=nu, nv=nu,
                                                u0=-(nu - 1) / 2 * cfg.grid.du,
                                                v0=-(nu - 1) / 2 * cfg.grid.du))
    x = _filter_input(F, nz, nu, seed=520)
    ref, eig = clutter.filter_planes(x.astype(np.complex128), c)
    ctx = ulm.Context(cfg)
    d = _to_dev(torch, x, torch.complex64)
    ev = ulm.svd_clutter_filter(ctx, d)
    ulm.ulm_check_status(ctx)
    got, gev = d.cpu().numpy(), ev.cpu().numpy()
    for o in range(2):
        e = rel_l2(got[o, 0], ref[o, 0])
        ee = np.max(np.abs(gev[o, 0] - eig[o, 0])) / eig[o, 0, 0]
        say(f"[filter F={F} {nz}x{nu} c={c}] plane {o}: rel-L2 {e:.2e}, eigenvalue err / lambda_1 {ee:.2e}")
        assert e <= FILTER_TOL
        assert ee <= 1e-10


def _sensitivity():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "fp32_sensitivity_tiny.json")
    return json.load(open(path))


def test_end_to_end_tiny(torch, ulm, tiny_cfg, tiny_iq):
    """Whole path (IQ -> detections) on the tiny ensemble, in two comparisons.

    1. The library's filter and localiser against the oracle's, both run on the
       library's own FP32 projections (the projections themselves against the
       oracle's beamformer to 1e-4): identical decidable detection sets
       (margin 1e-5) and every decidable detection within 1e-3 px.
    2. The library's detections against the oracle's whole path from the same
       IQ.  The clutter filter amplifies the projections' FP32 error by the
       tissue-to-residual ratio, so this comparison can be no tighter than the
       oracle's own response to such an input error.  That response is
       measured by tests/golden/make_fp32_sensitivity.py (the oracle's filter and
       localiser on its projections with a relative error of 1e-6, rounded to
       FP32) and scales with the input error; the decidability margin and the
       position tolerance of every decidable detection are three times that
       response scaled to the measured projection error.  MB-scale peaks
       (envelope >= 0.2 x frame maximum) are held to 1e-3 px."""
    cfg = tiny_cfg
    say("[end-to-end tiny] oracle pipeline")
    ref = pipeline.reconstruct_ensemble(tiny_iq, cfg)
    ora, N, I = localize.localize(ref["filtered"], cfg)
    ctx = ulm.Context(cfg)
    d_iq = _to_dev(torch, tiny_iq, torch.complex64)
    proj_dev = ulm.rca_beamform_proj(ctx, d_iq)
    torch.cuda.synchronize()
    proj = proj_dev.cpu().numpy()
    out = ulm.ulm_reconstruct_ensemble(ctx, d_iq, capacity=100000, timing=True)
    ulm.ulm_check_status(ctx, out["count"], 100000)
    got = ulm.locs_to_numpy(out["locs"], out["count"])
    filt = out["proj"].cpu().numpy()
    eps = rel_l2(proj, ref["proj"])
    say(f"  projections rel-L2 {eps:.2e}")
    assert eps <= BEAMFORM_TOL
    # 1. shared FP32 projections
    ref32, _ = clutter.filter_planes(proj.astype(np.complex128), cfg.svd_cutoff)
    ora32, N32, I32 = localize.localize(ref32, cfg)
    for o in range(2):
        e = rel_l2(filt[o, 0], ref32[o, 0])
        say(f"  filtered plane {o} vs oracle on the same projections: rel-L2 {e:.2e}")
        assert e <= FILTER_TOL
    n1, und1, err1 = compare_detections(got, ora32, N32, I32, cfg, delta=1e-5, pos_tol=POS_TOL)
    say(f"  same projections: {n1} decidable detections identical, {und1} undecidable, "
        f"max position error {err1:.1e} px")
    # 2. against the oracle's whole path from IQ
    sens = _sensitivity()
    pert = sens["variants"]["fp32_perturbed"]
    scale = 3.0 * eps / sens["eps_perturb"]
    delta = max(1e-5, scale * max(pert["max_abs_dncc"], pert["max_rel_dintensity"]))
    pos_all = max(POS_TOL, scale * pert["max_dpos_decidable_px"])
    for o in range(2):
        say(f"  filtered plane {o} vs the oracle's whole path: rel-L2 "
            f"{rel_l2(filt[o, 0], ref['filtered'][o, 0]):.2e}")
    n, nund, err = compare_detections(got, ora, N, I, cfg, delta=delta, pos_tol=pos_all)
    strong = ora[ora["intensity"] >= 0.2 * np.array([I[r["plane"], r["block"], r["frame"]].max()
                                                      for r in ora])]
    g = {(int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"])): r for r in got}
    serr = 0.0
    for r in strong:
        k = (int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"]))
        assert k in g
        serr = max(serr, abs(g[k]["z"] - r["z"]), abs(g[k]["u"] - r["u"]))
    say(f"  whole path: margin {delta:.1e}, tolerance {pos_all:.1e} px: {n} decidable detections "
        f"identical, {nund} undecidable, max position error {err:.2e} px; {len(strong)} MB-scale "
        f"peaks, max position error {serr:.2e} px; timing {out['timing']}")
    assert serr <= POS_TOL


def test_sim_parity(torch, ulm, tiny_cfg, tiny_iq):
    cfg = tiny_cfg
    med = make_medium(cfg, 0)
    ctx = ulm.Context(cfg)
    iq = ulm.ulm_sim_channel_data(ctx, _to_dev(torch, med.pos, torch.float64),
                                  _to_dev(torch, med.amp, torch.complex128), med.noise_seed,
                                  med.noise_sigma)
    torch.cuda.synchronize()
    got = iq.cpu().numpy()
    e = rel_l2(got, tiny_iq)
    say(f"[sim] rel-L2 {e:.2e}")
    assert e <= 1e-5


def test_deterministic(torch, ulm, tiny_cfg, tiny_iq):
    ctx = ulm.Context(tiny_cfg)
    d = _to_dev(torch, tiny_iq, torch.complex64)
    a = ulm.ulm_reconstruct_ensemble(ctx, d, capacity=50000)
    pa = a["proj"].clone()
    la = ulm.locs_to_numpy(a["locs"], a["count"]).copy()
    b = ulm.ulm_reconstruct_ensemble(ctx, d, capacity=50000)
    torch.cuda.synchronize()
    assert torch.equal(pa.view(torch.float32), b["proj"].view(torch.float32))
    lb = ulm.locs_to_numpy(b["locs"], b["count"])
    assert la.tobytes() == lb.tobytes()


def test_capacity_overflow(torch, ulm, tiny_cfg, tiny_iq):
    ctx = ulm.Context(tiny_cfg)
    d = _to_dev(torch, tiny_iq, torch.complex64)
    full = ulm.ulm_reconstruct_ensemble(ctx, d, capacity=100000)
    n = int(full["count"].item())
    allrec = ulm.locs_to_numpy(full["locs"], full["count"]).copy()
    assert n > 20
    cap = n // 3
    part = ulm.ulm_reconstruct_ensemble(ctx, d, capacity=cap)
    assert int(part["count"].item()) == n
    with pytest.raises(ulm.ULMError) as ei:
        ulm.ulm_check_status(ctx, part["count"], cap)
    assert ei.value.code == -3
    got = ulm.locs_to_numpy(part["locs"], torch.tensor([cap]))
    assert got.tobytes() == allrec[:cap].tobytes()


def test_nan_input_flags_numeric(torch, ulm):
    cfg = with_frames(cfg_tiny(), 10).with_(svd_cutoff=2)
    x = _filter_input(10, 64, 64, seed=9)
    x[1, 0, 3, 10, 10] = np.nan
    ctx = ulm.Context(cfg)
    d = _to_dev(torch, x, torch.complex64)
    ulm.svd_clutter_filter(ctx, d)
    with pytest.raises(ulm.ULMError) as ei:
        ulm.ulm_check_status(ctx)
    assert ei.value.code == -4
    got = d.cpu().numpy()
    # plane 1 left unfiltered; plane 0 filtered normally
    fin = np.isfinite(x[1])
    diff = np.argwhere(fin & (got[1] != x[1]))
    say(f"  plane 1 changed finite entries: {len(diff)} e.g. {diff[:5].tolist()}")
    assert len(diff) == 0
    assert not np.isfinite(got[1][~fin]).any()
    assert not np.array_equal(got[0], x[0])


def test_density_accumulate(torch, ulm, tiny_cfg):
    """Synthetic records (seeded, host) binned on the GPU == the oracle's histogram."""
    g = tiny_cfg.grid
    rng = np.random.default_rng(17)
    n = 5000
    recs = np.zeros(n, dtype=ulm.LOC_DTYPE)
    recs["plane"] = rng.integers(0, 2, n)
    recs["frame"] = rng.integers(0, 20, n)
    recs["z"] = rng.uniform(-1.0, g.nz + 0.5, n).astype(np.float32)
    recs["u"] = rng.uniform(-1.0, g.nu + 0.5, n).astype(np.float32)
    recs["iz"] = np.rint(recs["z"]).astype(np.int32)
    recs["iu"] = np.rint(recs["u"]).astype(np.int32)
    ctx = ulm.Context(tiny_cfg)
    dev = torch.from_numpy(recs.view(np.int32).reshape(n, 8).copy()).cuda()
    cnt = torch.tensor([n], dtype=torch.int32, device="cuda")
    dens = torch.zeros((2, g.nz * 2, g.nu * 2), dtype=torch.int32, device="cuda")
    ulm.ulm_density_accumulate(ctx, dev, cnt, n, dens, upsample=2)
    ref = pipeline.density_map({"plane": recs["plane"], "z": recs["z"].astype(np.float64),
                                "u": recs["u"].astype(np.float64)}, 2, g.nz, g.nu)
    assert np.array_equal(dens.cpu().numpy().astype(np.uint32), ref)


def test_density_map_ssim(torch, ulm, tiny_cfg):
    """Density maps accumulated over four tiny ensembles (channel data from the
    oracle's forward model): the library's whole path and density kernel against
    the oracle's pipeline and histogram, SSIM per plane."""
    cfg = tiny_cfg
    g = cfg.grid
    ref = np.zeros((2, 2 * g.nz, 2 * g.nu), np.uint32)
    ctx = ulm.Context(cfg)
    dens = torch.zeros((2, 2 * g.nz, 2 * g.nu), dtype=torch.int32, device="cuda")
    n_total = 0
    for e in range(4):
        iq = sim.simulate(cfg, make_medium(cfg, e))
        r = pipeline.reconstruct_ensemble(iq, cfg)
        ref += pipeline.density_map(r["locs"], 2, g.nz, g.nu)
        out = ulm.ulm_reconstruct_ensemble(ctx, _to_dev(torch, iq, torch.complex64),
                                           capacity=100000)
        ulm.ulm_check_status(ctx, out["count"], 100000)
        ulm.ulm_density_accumulate(ctx, out["locs"], out["count"], 100000, dens, upsample=2)
        n_total += int(out["count"].item())
    got = dens.cpu().numpy().astype(np.uint32)
    for o in range(2):
        s = pipeline.ssim(got[o], ref[o])
        say(f"[density ssim] plane {o}: {got[o].sum()} vs {ref[o].sum()} localisations, SSIM {s:.5f}")
        assert s >= 0.99
    assert n_total > 0
