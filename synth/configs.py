"""Workload configurations: probe, transmit sequence, image grid, medium and
localisation constants.

This module holds inputs only (numbers that describe an acquisition and the
constants a run is configured with); it contains none of the method's
arithmetic.  Both the CPU oracle and the HIP path receive these values.

Conventions (the paper does not fix them; the readings are listed in the
design notes):
  * SI units throughout (m, s, Hz, rad).
  * Orientation 0 ("RC"): transmit on row elements (plane wave steered in the
    y-z plane), receive on column elements (focused in x).  Its image plane
    is x-z: u = x is the receive-focused axis, v = y the transmit-steered
    axis along which the volume is projected.
  * Orientation 1 ("CR") is the mirror image: u = y, v = x.
  * Element e of either array sits at (e - (N-1)/2) * pitch.
  * Grid pixel centres: u_i = u0 + i*du, z_l = z0 + l*dz, v_m = v0 + m*dv.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Tuple


@dataclass(frozen=True)
class Probe:
    n_elem: int          # elements per orientation (rows == columns)
    pitch: float         # m
    f0: float            # centre frequency of the transmit pulse, Hz
    fs: float            # IQ sampling rate, Hz
    c: float             # speed of sound, m/s
    bandwidth: float = 0.65  # fractional -6 dB amplitude bandwidth of the pulse


@dataclass(frozen=True)
class Sequence:
    angles_deg: Tuple[float, ...]   # plane-wave steering angles per orientation
    n_frames: int                   # frames (volumes) per ensemble
    frame_rate: float               # Hz
    t_start: float                  # time of IQ sample 0 after the firing, s
    n_samp: int                     # IQ samples per channel

    @property
    def angles_rad(self) -> Tuple[float, ...]:
        return tuple(math.radians(a) for a in self.angles_deg)


@dataclass(frozen=True)
class Grid:
    nu: int
    nz: int
    du: float
    dz: float
    u0: float
    z0: float
    nv: int
    dv: float
    v0: float
    n_blocks: int = 1    # slabs along v that are projected separately
    v_ref: float = 0.0   # position of the stage-1 reference slice on v


@dataclass(frozen=True)
class Localisation:
    ncc_size: int        # odd template width/height in pixels
    sigma_u: float       # Gaussian template sigma along u, pixels
    sigma_z: float       # Gaussian template sigma along z, pixels
    tau_ncc: float = 0.5     # NCC threshold for a detection
    alpha: float = 0.05      # intensity threshold relative to the frame maximum


@dataclass(frozen=True)
class Medium:
    n_mb: int
    mb_kind: str                 # "straight" or "spline"
    mb_speed: Tuple[float, ...]  # straight: (lo, hi) m/s uniform; spline: (median, sigma_ln)
    n_vessels: int
    n_tissue: int
    tissue_db: float             # tissue scatterer rms amplitude over a unit MB, dB
    noise_db: float              # rms of complex channel noise over one unit MB echo, dB
    motion: str                  # "static" | "rigid_axial" | "nonrigid"
    motion_amp: float            # m
    motion_freq: Tuple[float, ...]  # Hz (one value for rigid; (lo, hi) for non-rigid)
    box_x: Tuple[float, float]
    box_y: Tuple[float, float]
    box_z: Tuple[float, float]


@dataclass(frozen=True)
class Config:
    name: str
    probe: Probe
    seq: Sequence
    grid: Grid
    svd_cutoff: int
    loc: Localisation
    medium: Medium
    seed_base: int = 0

    @property
    def n_orient(self) -> int:
        return 2

    @property
    def n_angles(self) -> int:
        return len(self.seq.angles_deg)

    @property
    def iq_shape(self):
        """IQ channel data layout [F][O][K][Nc][Ns], complex."""
        return (self.seq.n_frames, 2, self.n_angles, self.probe.n_elem, self.seq.n_samp)

    @property
    def proj_shape(self):
        """Projection stack layout [O][B][F][Nz][Nu], complex."""
        g = self.grid
        return (2, g.n_blocks, self.seq.n_frames, g.nz, g.nu)

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


def _centred_origin(n: int, d: float) -> float:
    return -(n - 1) / 2.0 * d


def cfg_tiny() -> Config:
    """Tiny ensemble: 32+32 elements, 4 angles, 20 frames, 64x64 planes."""
    probe = Probe(n_elem=32, pitch=0.2e-3, f0=6e6, fs=24e6, c=1540.0)
    seq = Sequence(angles_deg=(-6.0, -2.0, 2.0, 6.0), n_frames=20, frame_rate=400.0,
                   t_start=4.5e-6, n_samp=256)
    nu = 64
    du = 0.1e-3
    grid = Grid(nu=nu, nz=64, du=du, dz=6e-3 / 64, u0=_centred_origin(nu, du), z0=4e-3,
                nv=nu, dv=du, v0=_centred_origin(nu, du))
    loc = Localisation(ncc_size=7, sigma_u=1.2, sigma_z=1.2)
    med = Medium(n_mb=5, mb_kind="straight", mb_speed=(5e-3, 20e-3), n_vessels=0,
                 n_tissue=200, tissue_db=40.0, noise_db=-30.0, motion="static",
                 motion_amp=0.0, motion_freq=(0.0,),
                 box_x=(-3.2e-3, 3.2e-3), box_y=(-3.2e-3, 3.2e-3), box_z=(4e-3, 10e-3))
    return Config("tiny", probe, seq, grid, svd_cutoff=2, loc=loc, medium=med, seed_base=1000)


def cfg_paper() -> Config:
    """Paper-scale ensemble: 128+128 elements, 9 angles, 300 frames, 250x274 planes."""
    probe = Probe(n_elem=128, pitch=0.214e-3, f0=6e6, fs=24e6, c=1540.0)
    seq = Sequence(angles_deg=tuple(float(a) for a in range(-8, 9, 2)), n_frames=300,
                   frame_rate=400.0, t_start=25.0e-6, n_samp=1024)
    nu = 274
    du = 0.1e-3
    grid = Grid(nu=nu, nz=250, du=du, dz=0.1e-3, u0=_centred_origin(nu, du), z0=20e-3,
                nv=nu, dv=du, v0=_centred_origin(nu, du))
    loc = Localisation(ncc_size=9, sigma_u=1.2, sigma_z=1.2)
    med = Medium(n_mb=2000, mb_kind="spline", mb_speed=(10e-3, 0.5), n_vessels=50,
                 n_tissue=20000, tissue_db=40.0, noise_db=-30.0, motion="rigid_axial",
                 motion_amp=0.2e-3, motion_freq=(1.0,),
                 box_x=(-13.7e-3, 13.7e-3), box_y=(-13.7e-3, 13.7e-3), box_z=(20e-3, 45e-3))
    return Config("paper", probe, seq, grid, svd_cutoff=20, loc=loc, medium=med, seed_base=2000)


def cfg_precision() -> Config:
    """Same acquisition as the paper-scale ensemble; the split-precision filter runs on it."""
    c = cfg_paper()
    return c.with_(name="paper_bf16x", seed_base=3000)


def cfg_cnn(n_mb: int = 2000) -> Config:
    """Paper-scale probe and grid with a chosen MB count (learned-localiser data)."""
    c = cfg_paper()
    return c.with_(name="cnn", medium=replace(c.medium, n_mb=n_mb), seed_base=4000)


def cfg_stream(n_mb: int = 1000) -> Config:
    """Streaming run: paper-scale probe and grid, non-rigid tissue motion."""
    c = cfg_paper()
    med = replace(c.medium, n_mb=n_mb, motion="nonrigid", motion_amp=0.3e-3,
                  motion_freq=(0.5, 2.0))
    return c.with_(name="stream", medium=med, seed_base=5000)


def with_frames(cfg: Config, n_frames: int) -> Config:
    return cfg.with_(seq=replace(cfg.seq, n_frames=n_frames))


def with_angles(cfg: Config, angles_deg) -> Config:
    return cfg.with_(seq=replace(cfg.seq, angles_deg=tuple(float(a) for a in angles_deg)))


def with_blocks(cfg: Config, n_blocks: int) -> Config:
    return cfg.with_(grid=replace(cfg.grid, n_blocks=n_blocks))


CONFIGS = {
    "tiny": cfg_tiny,
    "paper": cfg_paper,
    "paper_bf16x": cfg_precision,
    "cnn": cfg_cnn,
    "stream": cfg_stream,
}
