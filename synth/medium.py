"""Seeded synthetic media: microbubble (MB) and tissue scatterers per frame.

Inputs only: positions, complex amplitudes and the noise seed that both the
oracle and the HIP simulator consume.  No beamforming, filtering or
localisation arithmetic lives here.

Seeds: ensemble e of a configuration uses numpy PCG64(seed_base + e).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .configs import Config


@dataclass
class Medium:
    """Scatterer positions for every frame.

    pos:    [F][S][3] float64, (x, y, z) in metres, frame f at t = f / frame_rate
    amp:    [S] complex128 fixed complex amplitude of each scatterer
    is_mb:  [S] bool, True for microbubbles (the first n_mb entries)
    noise_seed: 64-bit key for the channel-noise counter-based generator
    noise_sigma: rms magnitude of the complex channel noise
    """
    pos: np.ndarray
    amp: np.ndarray
    is_mb: np.ndarray
    noise_seed: int
    noise_sigma: float

    @property
    def n_mb(self) -> int:
        return int(self.is_mb.sum())

    def mb_positions(self) -> np.ndarray:
        """[F][n_mb][3] MB positions."""
        return self.pos[:, self.is_mb, :]


def _rng(cfg: Config, ensemble: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(cfg.seed_base + ensemble))


def _uniform_box(rng, n, med):
    x = rng.uniform(*med.box_x, size=n)
    y = rng.uniform(*med.box_y, size=n)
    z = rng.uniform(*med.box_z, size=n)
    return np.stack([x, y, z], axis=-1)


def _straight_mbs(rng, cfg, t):
    med = cfg.medium
    p0 = _uniform_box(rng, med.n_mb, med)
    d = rng.standard_normal((med.n_mb, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    speed = rng.uniform(med.mb_speed[0], med.mb_speed[1], size=med.n_mb)
    return p0[None, :, :] + t[:, None, None] * (speed[:, None] * d)[None, :, :]


def _vessels(rng, med, n_pts=512):
    """Random smooth vessel centre lines: cubic Bezier curves inside the box."""
    ctrl = np.stack([_uniform_box(rng, 4, med) for _ in range(med.n_vessels)])  # [V][4][3]
    s = np.linspace(0.0, 1.0, n_pts)
    b = np.stack([(1 - s) ** 3, 3 * s * (1 - s) ** 2, 3 * s ** 2 * (1 - s), s ** 3], axis=1)
    pts = np.einsum("pk,vkd->vpd", b, ctrl)                 # [V][P][3]
    seg = np.linalg.norm(np.diff(pts, axis=1), axis=2)
    arc = np.concatenate([np.zeros((med.n_vessels, 1)), np.cumsum(seg, axis=1)], axis=1)
    return pts, arc


def _spline_mbs(rng, cfg, t):
    med = cfg.medium
    pts, arc = _vessels(rng, med)
    total = arc[:, -1]
    vessel = rng.integers(0, med.n_vessels, size=med.n_mb)
    s0 = rng.uniform(0.0, 1.0, size=med.n_mb) * total[vessel]
    median, sigma_ln = med.mb_speed
    speed = median * np.exp(sigma_ln * rng.standard_normal(med.n_mb))
    # travel along the centre line; an MB leaving the end re-enters at the start
    s = np.mod(s0[None, :] + t[:, None] * speed[None, :], total[vessel][None, :])
    out = np.empty((t.size, med.n_mb, 3))
    for v in range(med.n_vessels):
        sel = np.nonzero(vessel == v)[0]
        if sel.size == 0:
            continue
        for d in range(3):
            out[:, sel, d] = np.interp(s[:, sel], arc[v], pts[v, :, d])
    return out


def _motion(rng, cfg, t, base):
    """Displacement [F][S][3] applied to every scatterer (the organ moves)."""
    med = cfg.medium
    disp = np.zeros((t.size,) + base.shape)
    if med.motion == "static":
        return disp
    if med.motion == "rigid_axial":
        disp[:, :, 2] = med.motion_amp * np.sin(2 * np.pi * med.motion_freq[0] * t)[:, None]
        return disp
    if med.motion == "nonrigid":
        ext = np.array([med.box_x[1] - med.box_x[0], med.box_y[1] - med.box_y[0],
                        med.box_z[1] - med.box_z[0]])
        for _ in range(3):
            kvec = rng.standard_normal(3) * (2 * np.pi / ext) * 0.5
            psi = rng.uniform(0, 2 * np.pi)
            direction = rng.standard_normal(3)
            direction /= np.linalg.norm(direction)
            f = rng.uniform(*med.motion_freq)
            ph = rng.uniform(0, 2 * np.pi)
            spatial = np.cos(base @ kvec + psi)                      # [S]
            temporal = np.sin(2 * np.pi * f * t + ph)                # [F]
            disp += (med.motion_amp / 3.0) * temporal[:, None, None] * spatial[None, :, None] \
                * direction[None, None, :]
        return disp
    raise ValueError(f"unknown motion {med.motion}")


def make_medium(cfg: Config, ensemble: int = 0) -> Medium:
    """Seeded medium for ensemble `ensemble` of configuration `cfg`."""
    med = cfg.medium
    rng = _rng(cfg, ensemble)
    t = np.arange(cfg.seq.n_frames) / cfg.seq.frame_rate
    if med.mb_kind == "straight":
        mb = _straight_mbs(rng, cfg, t)
    elif med.mb_kind == "spline":
        mb = _spline_mbs(rng, cfg, t)
    else:
        raise ValueError(med.mb_kind)
    tissue0 = _uniform_box(rng, med.n_tissue, med)
    tissue = np.broadcast_to(tissue0, (t.size,) + tissue0.shape)
    pos = np.concatenate([mb, tissue], axis=1)
    pos = pos + _motion(rng, cfg, t, pos[0])
    mb_phase = rng.uniform(0, 2 * np.pi, size=med.n_mb)
    amp_mb = np.exp(1j * mb_phase)
    rms = 10.0 ** (med.tissue_db / 20.0)
    amp_t = (rng.standard_normal(med.n_tissue) + 1j * rng.standard_normal(med.n_tissue)) \
        * (rms / np.sqrt(2.0))
    amp = np.concatenate([amp_mb, amp_t])
    is_mb = np.zeros(amp.size, dtype=bool)
    is_mb[: med.n_mb] = True
    noise_seed = int(rng.integers(0, 2 ** 63 - 1))
    return Medium(pos=np.ascontiguousarray(pos), amp=amp, is_mb=is_mb, noise_seed=noise_seed,
                  noise_sigma=10.0 ** (med.noise_db / 20.0))


def point_medium(cfg: Config, points, amps=None, noise_sigma: float = 0.0,
                 noise_seed: int = 0) -> Medium:
    """Static point scatterers at given (x, y, z) positions (for pins and tests)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    a = np.ones(p.shape[0], dtype=np.complex128) if amps is None else np.asarray(amps, np.complex128)
    pos = np.broadcast_to(p, (cfg.seq.n_frames,) + p.shape).copy()
    return Medium(pos=pos, amp=a, is_mb=np.ones(p.shape[0], bool), noise_seed=noise_seed,
                  noise_sigma=noise_sigma)
