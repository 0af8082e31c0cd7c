"""GPU parity of the rigid motion estimation on stage-1 slices against the
oracle, through the C ABI.

Inputs are seeded speckle fields moved by known integer and sub-pixel shifts
per frame (each slice its own field and its own shifts), and at the paper
scale the library's own stage-1 slices of a simulated ensemble with rigid
axial motion (compared with the oracle on sampled frames, and with the
medium's true motion).  The displacement is a decision (the integer peak) plus
a fit: the peak must match wherever the oracle's best and second-best NCC
differ by more than the FP32 summation noise, and the fitted displacement
must agree to 1e-3 px."""
from dataclasses import replace

import numpy as np
import pytest

from synth import arrays, cfg_paper, cfg_tiny, make_medium, with_angles, with_frames
from oracle import motion
from gpu_util import say

pytestmark = pytest.mark.gpu

POS_TOL = 1e-3        # px
GAP = 1e-5            # NCC gap below which the integer peak is undecidable


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ulm():
    import paper_2511_21647_amd as u
    return u


def _ragged_cfg():
    c = with_angles(with_frames(cfg_tiny(), 37), [-6, -2, 0, 3, 6])
    g = c.grid
    return c.with_(grid=replace(g, nu=45, nz=37, u0=-22 * g.du, nv=45, v0=-22 * g.dv))


def _shifted_slices(cfg, seed, max_shift):
    """[2][K][F][Nz][Nu] complex64: per slice a speckle field moved per frame."""
    g = cfg.grid
    K, F = cfg.n_angles, cfg.seq.n_frames
    rng = np.random.default_rng(seed)
    S = np.zeros((2, K, F, g.nz, g.nu), np.complex64)
    for o in range(2):
        for k in range(K):
            base = arrays.speckle_field(g.nz, g.nu, seed * 100 + 10 * o + k)
            for f in range(F):
                d = (0.0, 0.0) if f == 0 else rng.uniform(-max_shift, max_shift, 2)
                S[o, k, f] = arrays.shift_field(base, d[0], d[1])
    return S


def _oracle_disp(S, ref, L, frames):
    """Oracle displacement and the NCC gap (best - second best, FP32) per
    (o, k, frame in `frames`)."""
    O, K = S.shape[:2]
    disp = np.zeros((O, K, len(frames), 2))
    gap = np.zeros((O, K, len(frames)))
    lz = np.arange(-L, L + 1)
    for o in range(O):
        for k in range(K):
            b = motion.envelope(S[o, k, ref].astype(np.complex128))
            for i, f in enumerate(frames):
                c = motion.ncc_surface(motion.envelope(S[o, k, f].astype(np.complex128)), b)
                disp[o, k, i] = motion.peak(c, L)
                w = np.sort(c[np.ix_(lz % c.shape[0], lz % c.shape[1])].astype(np.float32).ravel())
                gap[o, k, i] = w[-1] - w[-2]
    return disp, gap


def _compare(got, want, gap):
    dec = gap > GAP
    err = np.abs(got - want).max(axis=-1)
    say(f"  decidable {dec.sum()} of {dec.size}, max |d| error {err[dec].max():.2e} px")
    assert dec.mean() > 0.9
    assert err[dec].max() <= POS_TOL


@pytest.mark.parametrize("case,L", [("tiny", 8), ("tiny", 3), ("tiny", 10), ("ragged", 8)])
def test_motion_parity(torch, ulm, case, L):
    cfg = cfg_tiny() if case == "tiny" else _ragged_cfg()
    F = cfg.seq.n_frames
    S = _shifted_slices(cfg, 5 + L, max_shift=min(L, 4) + 0.5)
    ref = 0 if case == "tiny" else 7
    ctx = ulm.Context(cfg)
    d_S = torch.from_numpy(S).cuda()
    say(f"[motion {case} L={L}] slices {S.shape}, reference frame {ref}")
    disp, mot = ulm.ulm_motion_estimate(ctx, d_S, ref_frame=ref, max_lag=L)
    torch.cuda.synchronize()
    got = disp.cpu().numpy()
    want, gap = _oracle_disp(S, ref, L, list(range(F)))
    _compare(got, want, gap)
    # the 3D composition of the library's own per-slice displacements
    m = got.astype(np.float64).mean(axis=1)
    want3 = np.stack([m[0, :, 1], m[1, :, 1], 0.5 * (m[0, :, 0] + m[1, :, 0])], axis=1)
    assert np.allclose(mot.cpu().numpy(), want3, atol=1e-5)
    # the reference frame against itself: no motion
    assert np.abs(got[:, :, ref]).max() <= 1e-4


def test_motion_argument_checks(torch, ulm):
    cfg = cfg_tiny()
    ctx = ulm.Context(cfg)
    S = torch.zeros((2, cfg.n_angles, cfg.seq.n_frames, cfg.grid.nz, cfg.grid.nu),
                    dtype=torch.complex64, device="cuda")
    for kw in ({"max_lag": 0}, {"max_lag": 11}, {"ref_frame": cfg.seq.n_frames}, {"ref_frame": -1}):
        with pytest.raises(ulm.ULMError) as e:
            ulm.ulm_motion_estimate(ctx, S, **kw)
        assert e.value.code == ulm.ULM_ERR_INVALID_ARG


def test_motion_paper_scale(torch, ulm):
    """Stage-1 slices of a simulated paper-scale ensemble (rigid axial motion,
    0.2 mm at 1 Hz): the library's displacements of three sampled frames
    against the oracle, and the estimated axial motion of every frame against
    the medium's true motion."""
    cfg = cfg_paper()
    g = cfg.grid
    F = cfg.seq.n_frames
    med = make_medium(cfg, 3)
    ctx = ulm.Context(cfg)
    iq = ulm.ulm_sim_channel_data(ctx, torch.from_numpy(np.ascontiguousarray(med.pos)).cuda(),
                                  torch.from_numpy(med.amp).cuda(), med.noise_seed, med.noise_sigma)
    ulm.rca_beamform_stage1(ctx, iq)
    del iq
    S = ulm.ulm_stage1_slices(ctx)
    L = 8
    disp, mot = ulm.ulm_motion_estimate(ctx, S, ref_frame=0, max_lag=L)
    torch.cuda.synchronize()
    frames = [0, 97, 233]
    sub = S[:, :, frames].cpu().numpy()
    want, gap = _oracle_disp(sub, 0, L, [0, 1, 2])
    got = disp.cpu().numpy()[:, :, frames]
    say(f"[motion paper] slices {tuple(S.shape)}")
    _compare(got, want, gap)
    t = np.arange(F) / cfg.seq.frame_rate
    true_dz = cfg.medium.motion_amp * np.sin(2 * np.pi * cfg.medium.motion_freq[0] * t) / g.dz
    est = mot.cpu().numpy()
    err = np.abs(est[:, 2] - true_dz)
    say(f"  axial motion: true range [{true_dz.min():.2f}, {true_dz.max():.2f}] px, "
        f"max |error| {err.max():.3f} px, rms {np.sqrt(np.mean(err ** 2)):.3f} px; "
        f"lateral |dx|, |dy| max {np.abs(est[:, :2]).max():.3f} px")
    assert err.max() < 0.25
