"""Oracle: NCC microbubble localisation on projection planes (FP64, CPU).

TEST INFRASTRUCTURE ONLY.

Section II-A4: each projection is normalised-cross-correlated with a
Gaussian-fitted PSF, and sub-pixel regional peaks of the correlation map are
the localisations; Section II-A4 (CUDA implementation) also thresholds on the
maximum intensity of each volume.  The paper leaves the details open; the
readings taken here:
  * image I = |filtered projection| (envelope magnitude);
  * template K(a, b) = g_z(a) g_u(b), g(a) = exp(-a^2 / (2 sigma^2)),
    a, b in [-h, h], h = (size - 1) / 2;
  * zero-mean NCC over the window W centred on the pixel, zero padding
    outside the image, |W| = size^2:
        NCC = (sum I K - Kbar sum I) / sqrt((sum I^2 - (sum I)^2/|W|) * sum (K - Kbar)^2)
    and NCC = 0 where the window variance is at most 1e-6 of sum I^2;
  * a detection is a pixel with NCC >= tau_ncc, I >= alpha * max_frame(I),
    and NCC strictly above the 3x3 neighbours that come before it in raster
    order and not below those after it (neighbours outside the image are
    ignored);
  * sub-pixel offset per axis from the three NCC values N-, N0, N+ by a
    3-point Gaussian fit, delta = (ln N- - ln N+) / (2 (ln N- - 2 ln N0 + ln N+)),
    the parabolic form where a value is <= 0, zero on an image border or for
    a non-negative curvature, clamped to [-0.5, 0.5].
Positions are in pixel units with pixel centres at integers.  Decisions
(thresholds, local maximum) are taken on the values rounded to float32, the
precision the GPU kernels compute in; the sub-pixel fit uses FP64 values.
"""
from __future__ import annotations

import numpy as np

VAR_EPS = 1e-6

LOC_DTYPE = np.dtype([("plane", np.int32), ("block", np.int32), ("frame", np.int32),
                      ("iz", np.int32), ("iu", np.int32), ("z", np.float64), ("u", np.float64),
                      ("ncc", np.float64), ("intensity", np.float64),
                      ("margin", np.float64)])


def gaussian_taps(size: int, sigma: float) -> np.ndarray:
    h = (size - 1) // 2
    a = np.arange(-h, h + 1, dtype=np.float64)
    return np.exp(-a * a / (2.0 * sigma * sigma))


def template(size: int, sigma_z: float, sigma_u: float) -> np.ndarray:
    return np.outer(gaussian_taps(size, sigma_z), gaussian_taps(size, sigma_u))


def envelope(filtered) -> np.ndarray:
    return np.abs(np.asarray(filtered, dtype=np.complex128))


def ncc_map(I, Kt) -> np.ndarray:
    """Direct (non-separable) zero-mean NCC of images [..][nz][nu] with template Kt."""
    I = np.asarray(I, dtype=np.float64)
    sz = Kt.shape[0]
    h = (sz - 1) // 2
    W = float(sz * sz)
    Kbar = Kt.sum() / W
    sK = ((Kt - Kbar) ** 2).sum()
    pad = [(0, 0)] * (I.ndim - 2) + [(h, h), (h, h)]
    Ip = np.pad(I, pad)
    nz, nu = I.shape[-2:]
    sIK = np.zeros_like(I)
    sI = np.zeros_like(I)
    sI2 = np.zeros_like(I)
    for a in range(sz):
        for b in range(sz):
            win = Ip[..., a:a + nz, b:b + nu]
            sIK += Kt[a, b] * win
            sI += win
            sI2 += win * win
    num = sIK - Kbar * sI
    var = sI2 - sI * sI / W
    ok = var > VAR_EPS * sI2
    out = np.zeros_like(I)
    out[ok] = num[ok] / np.sqrt(var[ok] * sK)
    return out


def ncc_map_separable(I, gz, gu) -> np.ndarray:
    """The same NCC from separable 1D correlations (two passes per sum)."""
    I = np.asarray(I, dtype=np.float64)
    sz = gz.size
    h = (sz - 1) // 2
    W = float(sz * sz)
    Kbar = gz.sum() * gu.sum() / W
    Kt = np.outer(gz, gu)
    sK = ((Kt - Kbar) ** 2).sum()

    def corr(x, taps, axis):
        xp = np.pad(x, [(h, h) if ax == (axis % x.ndim) else (0, 0) for ax in range(x.ndim)])
        n = x.shape[axis]
        out = np.zeros_like(x)
        for a in range(sz):
            out += taps[a] * np.take(xp, np.arange(a, a + n), axis=axis)
        return out

    ones = np.ones(sz)
    sIK = corr(corr(I, gu, -1), gz, -2)
    sI = corr(corr(I, ones, -1), ones, -2)
    sI2 = corr(corr(I * I, ones, -1), ones, -2)
    num = sIK - Kbar * sI
    var = sI2 - sI * sI / W
    ok = var > VAR_EPS * sI2
    out = np.zeros_like(I)
    out[ok] = num[ok] / np.sqrt(var[ok] * sK)
    return out


def subpixel(nm, n0, np_):
    """3-point Gaussian fit (parabolic where a value is <= 0), clamped to +-0.5."""
    nm, n0, np_ = (np.asarray(x, dtype=np.float64) for x in (nm, n0, np_))
    out = np.zeros(np.broadcast(nm, n0, np_).shape)
    pos = (nm > 0) & (n0 > 0) & (np_ > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        lm, l0, lp = np.log(np.where(pos, nm, 1)), np.log(np.where(pos, n0, 1)), \
            np.log(np.where(pos, np_, 1))
        den_g = 2.0 * (lm - 2.0 * l0 + lp)
        den_p = 2.0 * (nm - 2.0 * n0 + np_)
        d_g = np.where(den_g < 0, (lm - lp) / np.where(den_g < 0, den_g, 1), 0.0)
        d_p = np.where(den_p < 0, (nm - np_) / np.where(den_p < 0, den_p, 1), 0.0)
    out = np.where(pos, d_g, d_p)
    return np.clip(out, -0.5, 0.5)


def detect_frame(I, N, frame_max, tau_ncc, alpha, dec_dtype=np.float32):
    """Detections in one image.  Returns list of (iz, iu, dz, du, margin)."""
    nz, nu = N.shape
    Nd = N.astype(dec_dtype)
    Id = I.astype(dec_dtype)
    thr_i = dec_dtype(alpha) * dec_dtype(frame_max)
    cand = (Nd >= dec_dtype(tau_ncc)) & (Id >= thr_i)
    neg = np.full((nz + 2, nu + 2), -np.inf, dtype=dec_dtype)
    neg[1:-1, 1:-1] = Nd
    before = [(-1, -1), (-1, 0), (-1, 1), (0, -1)]
    after = [(0, 1), (1, -1), (1, 0), (1, 1)]
    gap = np.full((nz, nu), np.inf)
    for dz_, du_ in before:
        q = neg[1 + dz_:1 + dz_ + nz, 1 + du_:1 + du_ + nu]
        cand &= Nd > q
        gap = np.minimum(gap, N - np.where(np.isfinite(q), q.astype(np.float64), -np.inf))
    for dz_, du_ in after:
        q = neg[1 + dz_:1 + dz_ + nz, 1 + du_:1 + du_ + nu]
        cand &= Nd >= q
        gap = np.minimum(gap, N - np.where(np.isfinite(q), q.astype(np.float64), -np.inf))
    iz, iu = np.nonzero(cand)           # raster order
    res = []
    for z, u in zip(iz, iu):
        if 0 < z < nz - 1:
            dz = float(subpixel(N[z - 1, u], N[z, u], N[z + 1, u]))
        else:
            dz = 0.0
        if 0 < u < nu - 1:
            du = float(subpixel(N[z, u - 1], N[z, u], N[z, u + 1]))
        else:
            du = 0.0
        margin = min(abs(N[z, u] - tau_ncc), abs(I[z, u] / frame_max - alpha) if frame_max > 0
                     else np.inf, gap[z, u])
        res.append((int(z), int(u), dz, du, float(margin)))
    return res


def localize(filtered, cfg):
    """Detections for every plane/frame of filtered P[o][b][f][z][u].

    Returns (records sorted by (plane, block, frame, iz, iu), ncc maps, images).
    """
    P = np.asarray(filtered)
    loc = cfg.loc
    Kt = template(loc.ncc_size, loc.sigma_z, loc.sigma_u)
    I = envelope(P)
    N = ncc_map(I, Kt)
    recs = []
    O, B, F = P.shape[:3]
    for o in range(O):
        for b in range(B):
            for f in range(F):
                fmax = float(I[o, b, f].max())
                for (z, u, dz, du, m) in detect_frame(I[o, b, f], N[o, b, f], fmax,
                                                      loc.tau_ncc, loc.alpha):
                    recs.append((o, b, f, z, u, z + dz, u + du, N[o, b, f, z, u],
                                 I[o, b, f, z, u], m))
    return np.array(recs, dtype=LOC_DTYPE), N, I
