"""GPU parity of the XDoppler path (cross projections, windowed cross-correlation
of the filtered stacks, localisation on the XDoppler image) against the FP64
oracle, through the C ABI, on seeded inputs: tiny and ragged sizes with one and
several slabs (both profile paths: slabs of 64 or more columns and narrower
ones), and sampled frames of the paper-scale workload (one slab and the P = 8
slab form)."""
from dataclasses import replace

import numpy as np
import pytest

from synth import arrays, cfg_paper, cfg_tiny, make_medium, with_angles, with_blocks, with_frames
from oracle import beamform, localize, sim, xdoppler
from gpu_util import compare_detections, rel_l2, say

pytestmark = pytest.mark.gpu

BEAMFORM_TOL = 1e-4
XD_TOL = 1e-5
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


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _square(cfg, n, n_blocks):
    g = cfg.grid
    o = -(n - 1) / 2 * g.du
    return cfg.with_(grid=replace(g, nu=n, nv=n, u0=o, v0=o, n_blocks=n_blocks))


CASES = {
    # name: (config, medium seed); slab width 64 (wave sums), 12 and 5 (lane sums)
    "tiny": (lambda: cfg_tiny(), 0),
    "ragged_b4": (lambda: _square(with_angles(with_frames(cfg_tiny(), 18), [-6, -2, 0, 3, 6]),
                                  45, 4), 3),
    "slabs_b13": (lambda: with_blocks(with_frames(cfg_tiny(), 6), 13), 4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_cross_projection_parity(torch, ulm, case):
    make, seed = CASES[case]
    cfg = make()
    iq = sim.simulate(cfg, make_medium(cfg, seed))
    say(f"[cross {case}] iq {iq.shape}, B={cfg.grid.n_blocks}")
    ref = xdoppler.cross_project(beamform.stage1_slices(iq, cfg), cfg)
    ctx = ulm.Context(cfg)
    ulm.rca_beamform_stage1(ctx, _dev(torch, iq, torch.complex64))
    q = ulm.rca_beamform_cross(ctx)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    for o in range(2):
        for b in range(cfg.grid.n_blocks):
            e = rel_l2(got[o, b], ref[o, b])
            if b < 2 or b == cfg.grid.n_blocks - 1:
                say(f"  plane o={o} b={b} rel-L2 {e:.2e}")
            assert e <= BEAMFORM_TOL


@pytest.mark.parametrize("window", [1, 3, 5, 9])
def test_xdoppler_kernel_parity(torch, ulm, window):
    """Seeded native and cross stacks (ragged plane, 11 frames): the XDoppler
    image against the oracle, out of place and in place."""
    cfg = with_blocks(_square(with_frames(cfg_tiny(), 11), 37, 3), 3)
    shape = (2, 3, 11, cfg.grid.nz, 37)
    P = arrays.complex_normal(shape, seed=70)
    Q = arrays.complex_normal(shape, seed=71)
    ref = xdoppler.xdoppler(P.astype(np.complex128), Q.astype(np.complex128), window)
    ctx = ulm.Context(cfg)
    dP, dQ = _dev(torch, P, torch.complex64), _dev(torch, Q, torch.complex64)
    out = ulm.ulm_xdoppler(ctx, dP, dQ, window)
    ulm.ulm_xdoppler(ctx, dP, dQ, window, out=dP)
    torch.cuda.synchronize()
    got, inplace = out.cpu().numpy(), dP.cpu().numpy()
    e = rel_l2(got, ref)
    say(f"[xdoppler window {window}] rel-L2 {e:.2e}")
    assert e <= XD_TOL
    assert np.array_equal(got, inplace)
    assert np.all(got.imag == 0)


def test_xdoppler_argument_checks(torch, ulm):
    cfg = cfg_tiny()
    ctx = ulm.Context(cfg)
    P = torch.zeros(ctx.proj_shape, dtype=torch.complex64, device="cuda")
    Q = torch.zeros_like(P)
    for w in (0, 2, 11):
        with pytest.raises(ulm.ULMError):
            ulm.ulm_xdoppler(ctx, P, Q, w)
    with pytest.raises(ulm.ULMError):
        ulm.ulm_xdoppler(ctx, P, Q, 3, out=Q)
    rect = cfg.with_(grid=replace(cfg.grid, nv=60, v0=-29.5 * cfg.grid.dv))
    ctx_r = ulm.Context(rect)
    with pytest.raises(ulm.ULMError):
        ulm.rca_beamform_cross(ctx_r)


def test_xdoppler_path_tiny(torch, ulm, tiny_cfg, tiny_iq):
    """The whole XDoppler chain on the tiny ensemble: stage 1, native and cross
    projections, both filtered, XDoppler, NCC.  Each step against the oracle on
    the library's own input to that step (the filter amplifies FP32 rounding of
    its input, as in the plain path): the XDoppler image of the filtered stacks,
    then identical decidable detections within 1e-3 px."""
    cfg = tiny_cfg
    ctx = ulm.Context(cfg)
    ulm.rca_beamform_stage1(ctx, _dev(torch, tiny_iq, torch.complex64))
    P = ulm.rca_beamform_stage2(ctx)
    Q = ulm.rca_beamform_cross(ctx)
    ulm.svd_clutter_filter(ctx, P)
    ulm.svd_clutter_filter(ctx, Q)
    ulm.ulm_check_status(ctx)
    Pf, Qf = P.cpu().numpy(), Q.cpu().numpy()
    X = ulm.ulm_xdoppler(ctx, P, Q, 3)
    locs, cnt = ulm.ncc_localize(ctx, X, capacity=200000)
    ulm.ulm_check_status(ctx, cnt, 200000)
    got_x = X.cpu().numpy()
    ref_x = xdoppler.xdoppler(Pf.astype(np.complex128), Qf.astype(np.complex128), 3)
    e = rel_l2(got_x, ref_x)
    say(f"[xdoppler path tiny] XDoppler image rel-L2 {e:.2e}")
    assert e <= XD_TOL
    ora, N, I = localize.localize(got_x.astype(np.complex128), cfg)
    got = ulm.locs_to_numpy(locs, cnt)
    n, und, err = compare_detections(got, ora, N, I, cfg, 1e-5, POS_TOL)
    say(f"  {n} decidable detections identical, {und} undecidable, max position error {err:.1e} px")
    assert n > 0


SAMPLE_FRAMES = (0, 299)


@pytest.mark.parametrize("n_blocks", [1, 35])
def test_paper_cross_sampled_frames(torch, ulm, n_blocks):
    """Paper-scale workload in the launch configuration the bench times (one slab,
    and the P = 8 slab form with 35 slabs): seeded IQ in two frames of a
    300-frame ensemble, the cross projections of those frames against the oracle."""
    cfg = with_blocks(cfg_paper(), n_blocks)
    ctx = ulm.Context(cfg)
    iq = torch.zeros(ctx.iq_shape, dtype=torch.complex64, device="cuda")
    sub = arrays.complex_normal((len(SAMPLE_FRAMES),) + tuple(ctx.iq_shape[1:]), seed=33)
    for i, f in enumerate(SAMPLE_FRAMES):
        iq[f] = _dev(torch, sub[i], torch.complex64)
    say(f"[paper cross B={n_blocks}] frames {SAMPLE_FRAMES} of {tuple(iq.shape)}")
    ulm.rca_beamform_stage1(ctx, iq)
    q = ulm.rca_beamform_cross(ctx)
    torch.cuda.synchronize()
    got = q[:, :, list(SAMPLE_FRAMES)].cpu().numpy()
    del q, iq
    small = with_frames(cfg, len(SAMPLE_FRAMES))
    ref = xdoppler.cross_project(beamform.stage1_slices(sub.astype(np.complex128), small), small)
    e = rel_l2(got, ref)
    say(f"  rel-L2 over both frames and all {2 * n_blocks} planes {e:.2e}")
    assert e <= BEAMFORM_TOL
    for o in range(2):
        for b in (0, n_blocks - 1):
            assert rel_l2(got[o, b], ref[o, b]) <= BEAMFORM_TOL
