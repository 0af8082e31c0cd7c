"""Oracle: rigid motion estimation on the stage-1 reference slices (CPU).

TEST INFRASTRUCTURE ONLY.

The paper's motion estimation (Section II-A3, Fig. 1d) works on the 2K stage-1
slices instead of the volume: every frame of a slice is compared with a
reference frame by a Fourier-domain normalised cross-correlation (two forward
2D FFTs, a product, one inverse FFT); the displacement is the sub-pixel peak of
that correlation.  The K displacements of the RC slices (x-z plane) and of the
CR slices (y-z plane) are averaged per orientation, and the two in-plane
motions are combined into one 3D motion.

Readings (the cited method itself is not part of the paper):
  * the correlated images are the envelopes |S_k| of the slices; each is made
    zero-mean and the correlation is divided by the two norms, so the surface
    is the NCC of the frame with the reference circularly shifted by the lag;
  * no padding: the FFT correlation is circular over the Nz x Nu grid;
  * the peak is searched within |dz|, |du| <= max_lag (motion larger than the
    window is not representable); ties go to the first lag in raster order
    of (dz, du) from (-max_lag, -max_lag);
  * sub-pixel: the 3-point Gaussian fit per axis of the localiser (parabolic
    where a value is <= 0, zero for non-negative curvature, clamped to
    +-0.5), and zero along an axis whose integer peak lies on the window edge;
  * the peak choice and the fit are decided on FP32 NCC values (the kernel's
    precision): the FP64 surface is rounded to FP32 first;
  * 3D motion = (du of RC, du of CR, mean of the two dz): the two in-plane
    motions share the axial axis, so their axial parts are averaged rather
    than added.
Sign: a frame whose content moved by +d pixels (frame(p) = ref(p - d)) gives
displacement +d.
"""
from __future__ import annotations

import numpy as np

from .localize import subpixel


def envelope(S) -> np.ndarray:
    return np.abs(np.asarray(S))


def ncc_surface(a, b) -> np.ndarray:
    """Circular NCC of image a against reference b, indexed by lag mod (Nz, Nu):
    c[dz, du] = sum_p a0(p) b0(p - d) / (|a0| |b0|), a0, b0 the zero-mean images,
    computed in the Fourier domain as the paper describes."""
    a0 = np.asarray(a, np.float64) - np.mean(a)
    b0 = np.asarray(b, np.float64) - np.mean(b)
    den = np.linalg.norm(a0) * np.linalg.norm(b0)
    if den == 0.0:
        return np.zeros(a0.shape)
    A = np.fft.fft2(a0)
    B = np.fft.fft2(b0)
    return np.real(np.fft.ifft2(A * np.conj(B))) / den


def ncc_direct(a, b, lags) -> np.ndarray:
    """The same NCC by its plain definition at the listed lags (brute force)."""
    a0 = np.asarray(a, np.float64) - np.mean(a)
    b0 = np.asarray(b, np.float64) - np.mean(b)
    den = np.linalg.norm(a0) * np.linalg.norm(b0)
    out = []
    for dz, du in lags:
        out.append(np.sum(a0 * np.roll(b0, (dz, du), axis=(0, 1))) / den)
    return np.array(out)


def peak(c, max_lag: int):
    """Integer peak within the lag window and its sub-pixel refinement.
    Returns (dz, du) as floats."""
    L = max_lag
    nz, nu = c.shape
    c32 = c.astype(np.float32)
    lz = np.arange(-L, L + 1)
    win = c32[np.ix_(lz % nz, lz % nu)]
    k = int(np.argmax(win))                 # first maximum in raster order
    iz, iu = divmod(k, 2 * L + 1)
    dz, du = lz[iz], lz[iu]
    off = [0.0, 0.0]
    if abs(dz) < L:
        off[0] = float(subpixel(c32[(dz - 1) % nz, du % nu], c32[dz % nz, du % nu],
                                c32[(dz + 1) % nz, du % nu]))
    if abs(du) < L:
        off[1] = float(subpixel(c32[dz % nz, (du - 1) % nu], c32[dz % nz, du % nu],
                                c32[dz % nz, (du + 1) % nu]))
    return float(dz) + off[0], float(du) + off[1]


def estimate(S, ref_frame: int, max_lag: int):
    """S: stage-1 slices [2][K][F][Nz][Nu].  Returns (disp [2][K][F][2] = (dz, du)
    per slice and frame, motion [F][3] = (dx, dy, dz) in pixels)."""
    S = np.asarray(S)
    O, K, F = S.shape[:3]
    disp = np.zeros((O, K, F, 2))
    for o in range(O):
        for k in range(K):
            ref = envelope(S[o, k, ref_frame])
            for f in range(F):
                disp[o, k, f] = peak(ncc_surface(envelope(S[o, k, f]), ref), max_lag)
    mean = disp.mean(axis=1)                 # [2][F][2]
    motion = np.stack([mean[0, :, 1], mean[1, :, 1], 0.5 * (mean[0, :, 0] + mean[1, :, 0])], axis=1)
    return disp, motion
