"""Pins of the oracle's forward model and two-stage beamformer (CPU only).

Each test ties the oracle to something other than its own formulas: published
known-answer vectors, geometric constructions, closed forms, exact identities,
brute force, and the paper's error bound for two-stage beamforming.
"""
import os
from dataclasses import replace

import numpy as np
import pytest

from synth import cfg_tiny, point_medium, with_frames, with_angles
from oracle import beamform, sim
from oracle.philox import philox4x32_10, channel_noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Salmon et al., SC 2011)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [np.uint32(int(x, 16)) for x in r]
        out = philox4x32_10(v[0], v[1], v[2], v[3], v[4], v[5])
        assert [int(x) for x in out] == [int(x, 16) for x in r[6:10]]


def test_noise_moments():
    """Box-Muller noise: zero mean, E|n|^2 = sigma^2, independent re/im, Gaussian tails."""
    n = channel_noise(12345, 400000, seed=0xDEADBEEF12345, sigma=0.5)
    assert abs(n.mean()) < 0.005
    assert abs(np.mean(np.abs(n) ** 2) / 0.25 - 1) < 0.01
    assert abs(np.mean(n.real * n.imag)) < 0.002
    # P(|re| > 2 std) for a Gaussian is 0.0455
    frac = np.mean(np.abs(n.real) > 2 * 0.5 / np.sqrt(2))
    assert abs(frac - 0.0455) < 0.002


def _geometric_delays(cfg, p, o, k):
    """Time of flight by vector geometry: distance from the point to the plane
    wavefront through the first-firing array edge, plus distance to the receive
    line element (a line along v through the element centre)."""
    pr = cfg.probe
    th = cfg.seq.angles_rad[k]
    L = (pr.n_elem - 1) * pr.pitch
    x, y, z = p
    u, v = (x, y) if o == 0 else (y, x)
    edge = np.array([-L / 2 if th >= 0 else L / 2, 0.0])      # (v, z) of the first element to fire
    normal = np.array([np.sin(th), np.cos(th)])               # propagation direction in (v, z)
    d_tx = float(np.dot(np.array([v, z]) - edge, normal))
    out = []
    for e in range(pr.n_elem):
        ue = (e - (pr.n_elem - 1) / 2) * pr.pitch
        a = np.array([ue, 0.0, 0.0])                         # a point of the line, (u, v, z)
        d = np.array([0.0, 1.0, 0.0])                        # line direction
        w = np.array([u, v, z]) - a
        out.append(np.linalg.norm(np.cross(w, d)))
    return (d_tx + np.array(out)) / pr.c


def test_sim_single_scatterer_time_of_flight():
    """Echo peak time on every channel equals the geometric time of flight, and the
    demodulated phase there is -2 pi f0 tau."""
    cfg = with_frames(cfg_tiny(), 1)
    cfg = cfg.with_(probe=replace(cfg.probe, fs=480e6), seq=replace(cfg.seq, n_samp=256 * 20))
    p = (0.7e-3, -1.1e-3, 6.3e-3)
    iq = sim.simulate(cfg, point_medium(cfg, [p]), with_noise=False)
    t = cfg.seq.t_start + np.arange(cfg.seq.n_samp) / cfg.probe.fs
    for o in range(2):
        for k in range(cfg.n_angles):
            tof = _geometric_delays(cfg, p, o, k)
            env = np.abs(iq[0, o, k])
            pk = np.argmax(env, axis=1)
            assert np.all(np.abs(t[pk] - tof) <= 0.5 / cfg.probe.fs + 1e-12)
            ph = np.angle(iq[0, o, k, np.arange(cfg.probe.n_elem), pk])
            expect = np.angle(np.exp(-2j * np.pi * cfg.probe.f0 * tof))
            assert np.allclose(np.angle(np.exp(1j * (ph - expect))), 0, atol=1e-9)


def test_sim_pulse_bandwidth():
    """The echo's -6 dB amplitude spectrum width is 65% of f0 (Section II-C)."""
    cfg = with_frames(cfg_tiny(), 1)
    cfg = cfg.with_(probe=replace(cfg.probe, fs=480e6), seq=replace(cfg.seq, n_samp=8192))
    iq = sim.simulate(cfg, point_medium(cfg, [(0.0, 0.0, 6e-3)]), with_noise=False)
    x = iq[0, 0, 0, 16]
    spec = np.abs(np.fft.fftshift(np.fft.fft(x, 1 << 16)))
    freqs = np.fft.fftshift(np.fft.fftfreq(1 << 16, 1 / cfg.probe.fs))
    above = freqs[spec >= spec.max() / 2]
    width = above.max() - above.min()
    assert abs(width / cfg.probe.f0 - 0.65) < 0.005


def test_sim_mirror_symmetry():
    """Swapping x and y of the medium swaps the RC and CR channel data exactly."""
    cfg = with_frames(cfg_tiny(), 1)
    pts = np.array([[0.4e-3, -1.3e-3, 5.2e-3], [-2.0e-3, 0.9e-3, 8.1e-3]])
    a = sim.simulate(cfg, point_medium(cfg, pts), with_noise=False)
    b = sim.simulate(cfg, point_medium(cfg, pts[:, [1, 0, 2]]), with_noise=False)
    assert np.allclose(a[:, 0], b[:, 1], atol=1e-12, rtol=0)
    assert np.allclose(a[:, 1], b[:, 0], atol=1e-12, rtol=0)


def _pixel_centre_point(cfg, iu, iz, v=0.0):
    g = cfg.grid
    return (g.u0 + iu * g.du, v, g.z0 + iz * g.dz)


def test_stage1_single_scatterer_closed_form():
    """Noise-free scatterer at a pixel centre, theta = 0: the stage-1 value there is
    A e^{-i 4 pi f0 z / c} sum_e [(1 - fr_e) G(fr_e) + fr_e G(1 - fr_e)], G(x) the sampled
    Gaussian envelope x samples from its centre, and |S| peaks at that pixel."""
    cfg = with_angles(with_frames(cfg_tiny(), 1), [0.0])
    iu, iz = 21, 37
    p = _pixel_centre_point(cfg, iu, iz)
    iq = sim.simulate(cfg, point_medium(cfg, [p]), with_noise=False)
    S = beamform.stage1_slices(iq, cfg)
    plane = S[0, 0, 0]
    assert np.unravel_index(np.argmax(np.abs(plane)), plane.shape) == (iz, iu)
    tof = _geometric_delays(cfg, p, 0, 0)
    s = (tof - cfg.seq.t_start) * cfg.probe.fs
    fr = s - np.floor(s)
    sig = sim.pulse_sigma(cfg) * cfg.probe.fs
    G = lambda x: np.exp(-x * x / (2 * sig * sig))
    expect = np.exp(-4j * np.pi * cfg.probe.f0 * p[2] / cfg.probe.c) * \
        np.sum((1 - fr) * G(fr) + fr * G(1 - fr))
    assert abs(plane[iz, iu] - expect) <= 1e-9 * abs(expect)


def test_theta_zero_identity():
    """theta = 0: tau_tx has no v term, so brute-force 3D DAS summed over any slab
    equals (slab width) x the stage-1 slice, and stage 2 returns the same."""
    cfg = with_angles(with_frames(cfg_tiny(), 2), [0.0])
    rng = np.random.default_rng(3)
    pts = np.stack([rng.uniform(-3e-3, 3e-3, 8), rng.uniform(-3e-3, 3e-3, 8),
                    rng.uniform(4.5e-3, 9.5e-3, 8)], 1)
    iq = sim.simulate(cfg, point_medium(cfg, pts, noise_sigma=0.03, noise_seed=5))
    S = beamform.stage1_slices(iq, cfg)
    bf = beamform.das_3d_slab(iq, cfg, 10, 17)
    assert np.max(np.abs(bf - 7 * S)) <= 1e-12 * np.max(np.abs(S))
    P = beamform.stage2_project(S, cfg)
    assert np.max(np.abs(P[:, 0] - cfg.grid.nv * S[:, 0])) <= 1e-12 * np.max(np.abs(P))


def test_reference_slice_is_3d_slice():
    """At v = v_ref the extrapolated volume is the reference slice itself, and that
    slice equals the brute-force 3D DAS of slice v_ref, for every steering angle."""
    cfg = with_frames(cfg_tiny(), 1)
    g = cfg.grid
    cfg = cfg.with_(grid=replace(g, v_ref=g.v0 + 40 * g.dv))
    rng = np.random.default_rng(4)
    pts = np.stack([rng.uniform(-3e-3, 3e-3, 6), rng.uniform(-3e-3, 3e-3, 6),
                    rng.uniform(4.5e-3, 9.5e-3, 6)], 1)
    iq = sim.simulate(cfg, point_medium(cfg, pts), with_noise=False)
    S = beamform.stage1_slices(iq, cfg)
    bf = beamform.das_3d_slab(iq, cfg, 40, 41)
    ts = beamform.stage2_project_per_transmit(S, cfg, 40, 41)
    assert np.max(np.abs(bf - S)) <= 1e-12 * np.max(np.abs(S))
    assert np.max(np.abs(ts - S)) <= 1e-12 * np.max(np.abs(S))


def _fine_axial_case(t_scale=1.0):
    base = with_frames(cfg_tiny(), 1)
    dz = 12.5e-6
    cfg = base.with_(probe=replace(base.probe, n_elem=16, pitch=0.1e-3),
                     grid=replace(base.grid, nu=24, u0=-1.15e-3, nz=192, z0=7.8e-3, dz=dz),
                     seq=replace(base.seq, t_start=8e-6, n_samp=256))
    rng = np.random.default_rng(1)
    pts = np.stack([rng.uniform(-0.6e-3, 0.6e-3, 6), rng.uniform(-0.3e-3, 0.3e-3, 6),
                    rng.uniform(8.5e-3, 9.5e-3, 6)], 1)
    iq = sim.simulate(cfg, point_medium(cfg, pts), with_noise=False)
    return cfg, iq


def _two_stage_vs_3d(cfg, iq, m_lo, m_hi):
    S = beamform.stage1_slices(iq, cfg)
    bf = beamform.das_3d_slab(iq, cfg, m_lo, m_hi)
    ts = beamform.stage2_project_per_transmit(S, cfg, m_lo, m_hi)
    m = 32
    return [np.linalg.norm(bf[:, k, :, m:-m] - ts[:, k, :, m:-m]) /
            np.linalg.norm(bf[:, k, :, m:-m]) for k in range(cfg.n_angles)]


def test_two_stage_within_paper_bound():
    """Section III: two-stage beamforming is within 1% of 3D beamforming.  Holds
    per transmit on an 8-slice slab once the stage-1 slice resolves the axial
    pulse (dz = 12.5 um)."""
    cfg, iq = _fine_axial_case()
    err = _two_stage_vs_3d(cfg, iq, 28, 36)
    assert max(err) < 0.01, err


def test_two_stage_wrong_shift_law_fails(monkeypatch):
    """Planted mistakes in the oracle's stage 2 (shift law tan(theta) instead of
    tan(theta/2); dropped baseband phase) break the 1% agreement."""
    cfg, iq = _fine_axial_case()
    real_tan = np.tan
    monkeypatch.setattr(beamform.np, "tan", lambda x: real_tan(2 * x))
    assert max(_two_stage_vs_3d(cfg, iq, 28, 36)) > 0.05
    monkeypatch.setattr(beamform.np, "tan", real_tan)
    real_exp = np.exp
    monkeypatch.setattr(beamform.np, "exp", lambda x: real_exp(x.real) if np.iscomplexobj(x)
                        else real_exp(x))
    assert max(_two_stage_vs_3d(cfg, iq, 28, 36)) > 0.05


def test_beamform_linear_and_mirror():
    """Beamforming is linear in the channel data, and the mirrored medium gives the
    planes of the two orientations swapped."""
    cfg = with_frames(cfg_tiny(), 1)
    pts = np.array([[0.4e-3, -1.3e-3, 5.2e-3], [-2.0e-3, 0.9e-3, 8.1e-3]])
    a = sim.simulate(cfg, point_medium(cfg, pts), with_noise=False)
    b = sim.simulate(cfg, point_medium(cfg, pts[:, [1, 0, 2]]), with_noise=False)
    pa = beamform.beamform_proj(a, cfg)
    pb = beamform.beamform_proj(b, cfg)
    scale = np.max(np.abs(pa))
    assert np.max(np.abs(pa[0] - pb[1])) <= 1e-11 * scale
    assert np.max(np.abs(pa[1] - pb[0])) <= 1e-11 * scale
    pab = beamform.beamform_proj(a + 2.5j * b, cfg)
    assert np.max(np.abs(pab - (pa + 2.5j * pb))) <= 1e-11 * scale


STEERED_DEG = (-8.0, -6.0, -2.0, 2.0, 6.0, 8.0)


def _steered_closed_form_error(cfg, iu, iz):
    """|S - closed form| / |closed form| at the scatterer's pixel, and whether |S|
    peaks there, for one noise-free scatterer in the reference slice (v = v_ref).

    The expected value uses the geometric time of flight (wavefront through the
    first-firing array edge plus point-to-line distance), not the oracle's delay
    formula: A e^{-i 4 pi f0 z / c} sum_e [(1 - fr_e) G(fr_e) + fr_e G(1 - fr_e)],
    where fr_e is the fractional IQ sample index of that time of flight."""
    p = _pixel_centre_point(cfg, iu, iz, v=cfg.grid.v_ref)
    iq = sim.simulate(cfg, point_medium(cfg, [p]), with_noise=False)
    plane = beamform.stage1_slices(iq, cfg)[0, 0, 0]
    tof = _geometric_delays(cfg, p, 0, 0)
    s = (tof - cfg.seq.t_start) * cfg.probe.fs
    fr = s - np.floor(s)
    sig = sim.pulse_sigma(cfg) * cfg.probe.fs
    G = lambda x: np.exp(-x * x / (2 * sig * sig))
    expect = np.exp(-4j * np.pi * cfg.probe.f0 * p[2] / cfg.probe.c) * \
        np.sum((1 - fr) * G(fr) + fr * G(1 - fr))
    peak = np.unravel_index(np.argmax(np.abs(plane)), plane.shape) == (iz, iu)
    return abs(plane[iz, iu] - expect) / abs(expect), peak


@pytest.mark.parametrize("deg", STEERED_DEG)
def test_stage1_single_scatterer_closed_form_steered(deg):
    """Section II-A1, stage 1 with a steered plane wave: a scatterer at a pixel
    centre of the reference slice gives the closed-form value at that pixel (the
    steered transmit delay z cos(theta) + v sin(theta) + (L/2)|sin(theta)| enters
    only through the geometric time of flight), and |S| peaks at that pixel."""
    cfg = with_angles(with_frames(cfg_tiny(), 1), [deg])
    for iu, iz in ((21, 37), (45, 12)):
        err, peak = _steered_closed_form_error(cfg, iu, iz)
        assert err <= 1e-9, (deg, iu, iz, err)
        assert peak, (deg, iu, iz)


def _coherent_slab(cfg):
    """Four slices centred on the reference slice: a slab thin enough that a steered
    transmit's phase turns by well under a quarter cycle across it."""
    g = cfg.grid
    return cfg.with_(grid=replace(g, nv=4, v0=g.v_ref - 1.5 * g.dv, n_blocks=1))


POINT_TARGETS = ((16, 14), (44, 20), (24, 42), (48, 50), (32, 30))   # (iu, iz), 14+ px apart


def _point_target_errors(cfg):
    """Section II-A4 end to end on isolated point targets at pixel centres of the
    reference slice: simulate, beamform (both stages, coherent slab), filter with
    cutoff 0 (the identity), NCC-localise.  Returns the distance in pixels from
    each target to the nearest detection, for the x-z plane (targets at y = 0)
    and for the y-z plane (the mirrored medium)."""
    from oracle import clutter, localize
    g = cfg.grid
    pts = np.array([(g.u0 + iu * g.du, g.v_ref, g.z0 + iz * g.dz) for iu, iz in POINT_TARGETS])
    out = []
    for plane, pos in ((0, pts), (1, pts[:, [1, 0, 2]])):
        iq = sim.simulate(cfg, point_medium(cfg, pos), with_noise=False)
        P = beamform.beamform_proj(iq, cfg)
        Pf, _ = clutter.filter_planes(P, 0)
        assert np.array_equal(Pf, P)
        recs, _, _ = localize.localize(Pf, cfg)
        r = recs[recs["plane"] == plane]
        for iu, iz in POINT_TARGETS:
            out.append(float(np.min(np.hypot(r["u"] - iu, r["z"] - iz))))
    return np.array(out)


@pytest.mark.parametrize("deg", STEERED_DEG)
def test_point_targets_end_to_end(deg):
    """Isolated point targets through simulation -> two-stage beamforming ->
    identity filter -> NCC come back within 0.05 px of their known positions at
    every steering angle, one angle at a time.  The targets sit at pixel centres
    of the slab's middle, where the projected PSF is symmetric about the target,
    so any delay error shows as a displacement."""
    cfg = with_angles(_coherent_slab(with_frames(cfg_tiny(), 1)), [deg])
    err = _point_target_errors(cfg)
    assert err.max() <= 0.05, (deg, err)


def _planted_das(monkeypatch, tmp_path, old, new):
    """Load a copy of the oracle's DAS loops with one planted mistake."""
    from oracle import _clib
    src = open(os.path.join(os.path.dirname(beamform.__file__), "das.c")).read()
    assert src.count(old) == 1, old
    path = tmp_path / "das_planted.c"
    path.write_text(src.replace(old, new))
    h = _clib.load(_clib.compile_c(str(path), str(tmp_path / "libdas_planted.so")))
    monkeypatch.setattr(_clib, "_handle", h)


@pytest.mark.parametrize("old,new", [
    ("+ 0.5 * L * fabs(sin(theta))", ""),          # firing offset of a steered plane wave dropped
    ("z * cos(theta)", "z"),                         # wavefront depth term without cos(theta)
])
def test_steered_delay_planted_mistakes(monkeypatch, tmp_path, old, new):
    """Planted mistakes in the oracle's steered transmit delay break the steered
    closed form at every nonzero angle and the point-target pin at 6 and 8 deg."""
    _planted_das(monkeypatch, tmp_path, old, new)
    for deg in STEERED_DEG:
        cfg = with_angles(with_frames(cfg_tiny(), 1), [deg])
        err, _ = _steered_closed_form_error(cfg, 21, 37)
        assert err > 1e-3, (deg, err)
    for deg in (6.0, 8.0):
        cfg = with_angles(_coherent_slab(with_frames(cfg_tiny(), 1)), [deg])
        assert _point_target_errors(cfg).max() > 0.1, deg
