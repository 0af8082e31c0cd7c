"""Seeded synthetic arrays used as stage inputs by tests and the benchmark.

Every function returns plain numpy arrays drawn from numpy PCG64 with the given
seed.  None of them performs any step of the method.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def complex_normal(shape, seed: int, scale: float = 1.0, dtype=np.complex64) -> np.ndarray:
    """i.i.d. complex Gaussian with E|x|^2 = scale^2."""
    g = rng(seed)
    re = g.standard_normal(shape, dtype=np.float32 if dtype == np.complex64 else np.float64)
    im = g.standard_normal(shape, dtype=np.float32 if dtype == np.complex64 else np.float64)
    out = np.empty(shape, dtype=dtype)
    out.real = re * (scale / np.sqrt(2.0))
    out.imag = im * (scale / np.sqrt(2.0))
    return out


def clutter_stack(n_pix: int, n_frames: int, rank: int, seed: int, clutter_db: float = 40.0,
                  decay: float = 0.7) -> np.ndarray:
    """Casorati-shaped stack [F][n_pix] (complex64): a low-rank 'tissue' part with
    decaying mode energies, plus a weak i.i.d. 'blood' part of unit rms."""
    g = rng(seed)
    frames = np.arange(n_frames)
    out = np.zeros((n_frames, n_pix), dtype=np.complex128)
    amp = 10.0 ** (clutter_db / 20.0)
    for r in range(rank):
        spatial = (g.standard_normal(n_pix) + 1j * g.standard_normal(n_pix)) / np.sqrt(2)
        freq = g.uniform(-0.02, 0.02)
        temporal = np.exp(2j * np.pi * freq * frames) * (1.0 + 0.3 * g.standard_normal(n_frames))
        out += amp * (decay ** r) * temporal[:, None] * spatial[None, :]
    out += (g.standard_normal((n_frames, n_pix)) + 1j * g.standard_normal((n_frames, n_pix))) \
        / np.sqrt(2)
    return out.astype(np.complex64)


def gaussian_spots(nz: int, nu: int, n_spots: int, sigma: float, seed: int, spacing: float,
                   margin: int = 8):
    """A noise-free image made of isolated sampled 2D Gaussians.

    Returns (image [nz][nu] float64, centres [n][2] as (z, u) in pixel units).
    Centres are at least `spacing` pixels apart and `margin` pixels inside the
    border; sub-pixel offsets are uniform in [-0.5, 0.5).
    """
    g = rng(seed)
    centres = []
    tries = 0
    while len(centres) < n_spots and tries < 100000:
        tries += 1
        c = np.array([g.integers(margin, nz - margin), g.integers(margin, nu - margin)], float)
        c += g.uniform(-0.5, 0.5, size=2)
        if all(np.hypot(*(c - d)) >= spacing for d in centres):
            centres.append(c)
    centres = np.array(centres)
    zz, uu = np.meshgrid(np.arange(nz), np.arange(nu), indexing="ij")
    img = np.zeros((nz, nu))
    for cz, cu in centres:
        img += np.exp(-((zz - cz) ** 2 + (uu - cu) ** 2) / (2 * sigma ** 2))
    return img, centres


def spot_frames(n_frames: int, nz: int, nu: int, per_frame: int, sigma_z: float, sigma_u: float,
                seed: int, amplitude: float = 10.0, radius: int = 4) -> np.ndarray:
    """[F][nz][nu] complex64 frames of point-like echoes: per frame, `per_frame`
    sampled 2D Gaussians (sigmas in pixels) at uniform sub-pixel positions, each
    with a random phase, added over a (2 radius + 1)^2 patch."""
    g = rng(seed)
    out = np.zeros((n_frames, nz, nu), dtype=np.complex128)
    d = np.arange(-radius, radius + 1)
    for f in range(n_frames):
        cz = g.uniform(0, nz, per_frame)
        cu = g.uniform(0, nu, per_frame)
        ph = np.exp(2j * np.pi * g.uniform(0, 1, per_frame))
        iz = np.floor(cz).astype(int)[:, None] + d[None, :]          # [n][2r+1]
        iu = np.floor(cu).astype(int)[:, None] + d[None, :]
        wz = np.exp(-(iz - cz[:, None]) ** 2 / (2 * sigma_z ** 2))
        wu = np.exp(-(iu - cu[:, None]) ** 2 / (2 * sigma_u ** 2))
        val = amplitude * ph[:, None, None] * wz[:, :, None] * wu[:, None, :]
        zz = np.broadcast_to(iz[:, :, None], val.shape)
        uu = np.broadcast_to(iu[:, None, :], val.shape)
        ok = (zz >= 0) & (zz < nz) & (uu >= 0) & (uu < nu)
        np.add.at(out[f], (zz[ok], uu[ok]), val[ok])
    return out.astype(np.complex64)


def speckle_field(nz: int, nu: int, seed: int, smooth: float = 1.5) -> np.ndarray:
    """Band-limited complex Gaussian field [nz][nu] (complex128): a speckle
    pattern whose envelope has a correlation length of a few pixels."""
    g = rng(seed)
    x = g.standard_normal((nz, nu)) + 1j * g.standard_normal((nz, nu))
    kz = np.fft.fftfreq(nz)[:, None]
    ku = np.fft.fftfreq(nu)[None, :]
    return np.fft.ifft2(np.fft.fft2(x) * np.exp(-2 * (np.pi * smooth) ** 2 * (kz ** 2 + ku ** 2)))


def shift_field(field: np.ndarray, dz: float, du: float) -> np.ndarray:
    """`field` moved by (dz, du) pixels, circularly, by a Fourier phase ramp
    (exact for a band-limited field): out(p) = field(p - d)."""
    nz, nu = field.shape
    kz = np.fft.fftfreq(nz)[:, None]
    ku = np.fft.fftfreq(nu)[None, :]
    return np.fft.ifft2(np.fft.fft2(field) * np.exp(-2j * np.pi * (kz * dz + ku * du)))
