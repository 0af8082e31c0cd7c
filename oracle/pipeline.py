"""Oracle: the whole per-ensemble path and the accumulated density map.

TEST INFRASTRUCTURE ONLY.

Channel data -> two-stage beamforming to projection planes (Section II-A1,
II-A4) -> eigen-based SVD clutter filter of each plane (Section II-A2) ->
NCC localisation with sub-pixel peaks (Section II-A4).  The density map
histograms the localisations on a grid twice as fine as the planes
(Section II-A6 accumulates tracks into a 50 um map; tracking is not part of
this path, so localisations are accumulated directly).
"""
from __future__ import annotations

import numpy as np

from .beamform import beamform_proj
from .clutter import filter_planes
from .localize import localize


def reconstruct_ensemble(iq, cfg):
    """Returns dict(proj, filtered, eig, locs)."""
    proj = beamform_proj(iq, cfg)
    filt, eig = filter_planes(proj, cfg.svd_cutoff)
    locs, _, _ = localize(filt, cfg)
    return {"proj": proj, "filtered": filt, "eig": eig, "locs": locs}


def density_map(locs, n_planes: int, nz: int, nu: int, upsample: int = 2) -> np.ndarray:
    """Histogram of localisations per plane on an `upsample`x finer grid.

    Pixel i covers [i - 0.5, i + 0.5); fine bin = floor((x + 0.5) * upsample).
    Returns uint32 [n_planes][nz*upsample][nu*upsample].
    """
    out = np.zeros((n_planes, nz * upsample, nu * upsample), dtype=np.uint32)
    if len(locs) == 0:
        return out
    plane = np.asarray(locs["plane"]).astype(np.int64)
    bz = np.floor((np.asarray(locs["z"]) + 0.5) * upsample).astype(np.int64)
    bu = np.floor((np.asarray(locs["u"]) + 0.5) * upsample).astype(np.int64)
    ok = (bz >= 0) & (bz < nz * upsample) & (bu >= 0) & (bu < nu * upsample)
    np.add.at(out, (plane[ok], bz[ok], bu[ok]), 1)
    return out


def ssim(a, b, data_range=None, sigma: float = 1.5, radius: int = 5) -> float:
    """Mean SSIM (Wang, Bovik, Sheikh, Simoncelli 2004) with a Gaussian window."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if data_range is None:
        data_range = max(a.max() - a.min(), b.max() - b.min(), 1e-12)
    x = np.arange(-radius, radius + 1)
    w = np.exp(-x * x / (2 * sigma * sigma))
    w /= w.sum()

    def filt(img):
        p = np.pad(img, radius, mode="reflect")
        t = sum(w[i] * p[:, i:i + img.shape[1]] for i in range(w.size))
        return sum(w[i] * t[i:i + img.shape[0], :] for i in range(w.size))

    C1 = (0.01 * data_range) ** 2
    C2 = (0.03 * data_range) ** 2
    mu_a, mu_b = filt(a), filt(b)
    saa = filt(a * a) - mu_a ** 2
    sbb = filt(b * b) - mu_b ** 2
    sab = filt(a * b) - mu_a * mu_b
    s = ((2 * mu_a * mu_b + C1) * (2 * sab + C2)) / ((mu_a ** 2 + mu_b ** 2 + C1) * (saa + sbb + C2))
    return float(s.mean())
