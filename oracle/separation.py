"""Oracle: MB separation of the filtered planes into flow sub-populations (CPU).

TEST INFRASTRUCTURE ONLY.

The paper's MB separation (Section II-A5, Fig. 1c): at every pixel of every
projection plane, a temporal Fourier transform of the slow-time signal, several
band-pass filters that keep MBs of one flow direction and one speed range, and
an inverse Fourier transform per filter give the MB subsets (Up/Down x speed
ranges; the paper's results use three speed ranges per direction, six subsets).

Readings (the cited separation method is not part of the paper):
  * bins are those of the F-point DFT over the ensemble's frames, X[k] =
    sum_n x[n] exp(-2 pi i k n / F); with this library's baseband phase an
    MB moving towards the probe (decreasing depth) turns the pixel's phase
    forward in slow time, so "up" is the positive-frequency bins k = 1 ..
    H, H = (F - 1) // 2, and "down" the negative ones k = F - 1 .. F - H;
  * the S speed ranges split the H bins of each direction by |frequency| into
    S contiguous groups of as equal size as possible: range s holds
    |k| in [1 + floor(s H / S), 1 + floor((s + 1) H / S));
  * the filters are ideal (a 0/1 mask on the bins); the DC bin (no axial
    motion) and, for even F, the Nyquist bin (direction undefined) belong to
    no subset;
  * subset order: up range 0, ..., up range S-1, down range 0, ..., down
    range S-1 (range 0 is the slowest).
"""
from __future__ import annotations

import numpy as np


def band_bins(F: int, n_speed: int):
    """For each of the 2 S subsets, the list of DFT bins it keeps."""
    H = (F - 1) // 2
    out = []
    for direction in (+1, -1):
        for s in range(n_speed):
            lo = 1 + (s * H) // n_speed
            hi = 1 + ((s + 1) * H) // n_speed
            out.append([(direction * m) % F for m in range(lo, hi)])
    return out


def separate(planes, n_speed: int):
    """planes: [..., F, Nz, Nu] complex (frames on axis -3).  Returns the subsets
    [2 S][..., F, Nz, Nu]: inverse DFT of the masked temporal spectrum."""
    x = np.asarray(planes, dtype=np.complex128)
    F = x.shape[-3]
    X = np.fft.fft(x, axis=-3)
    out = np.zeros((2 * n_speed,) + x.shape, dtype=np.complex128)
    for i, bins in enumerate(band_bins(F, n_speed)):
        mask = np.zeros(F)
        mask[bins] = 1.0
        out[i] = np.fft.ifft(X * mask[:, None, None], axis=-3)
    return out
