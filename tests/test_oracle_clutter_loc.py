"""Pins of the oracle's clutter filter and NCC localiser (CPU only)."""
import os

import numpy as np
import pytest

from synth import arrays
from oracle import clutter, localize, pipeline


# ---------------------------------------------------------------- clutter filter

def _stack(n_pix=300, F=40, rank=4, seed=7):
    return arrays.clutter_stack(n_pix, F, rank, seed).astype(np.complex128)


def test_eigen_route_equals_svd_route():
    """Eigen route of Section II-A2 == direct SVD truncation (LAPACK zgesvd)."""
    s = _stack()
    for c in (1, 3, 6):
        a, lam = clutter.clutter_filter(s, c)
        b, sv = clutter.clutter_filter_svd(s, c)
        assert lam[c - 1] / lam[c] > 1 + 1e-6
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(s)
        # eigenvalues of I^H I are the squared singular values
        assert np.allclose(lam, sv ** 2, rtol=1e-9, atol=1e-9 * lam[0])


def test_filter_invariants():
    """||I_f||_F^2 = sum_{i>c} sigma_i^2 and I_f V_c = 0."""
    s = _stack(seed=11)
    c = 3
    f, lam = clutter.clutter_filter(s, c)
    sv = np.linalg.svd(clutter.casorati(s), compute_uv=False)
    assert abs(np.linalg.norm(f) ** 2 - np.sum(sv[c:] ** 2)) <= 1e-9 * np.sum(sv ** 2)
    _, Vc = clutter.clutter_subspace(clutter.covariance(s), c)
    resid = clutter.casorati(f) @ Vc
    assert np.max(np.abs(resid)) <= 1e-9 * np.max(np.abs(s))


def test_cutoff_extremes():
    s = _stack(seed=12)
    f0, _ = clutter.clutter_filter(s, 0)
    assert np.array_equal(f0, s)
    fall, _ = clutter.clutter_filter(s, s.shape[0])
    assert np.max(np.abs(fall)) <= 1e-9 * np.max(np.abs(s))


def test_rank_c_clutter_recovered_exactly():
    """Rank-c clutter X T^T plus a signal Y R^T that is orthogonal to it in time
    (T^H R = 0) and in space (X^H Y = 0): the filter returns the signal exactly."""
    rng = np.random.default_rng(3)
    F, n, c = 30, 200, 3
    Q, _ = np.linalg.qr(rng.standard_normal((F, F)) + 1j * rng.standard_normal((F, F)))
    T, R = Q[:, :c], Q[:, c:]
    Qn, _ = np.linalg.qr(rng.standard_normal((n, F)) + 1j * rng.standard_normal((n, F)))
    X = Qn[:, :c] * np.array([1e3, 5e2, 2e2])
    Y = Qn[:, c:] @ (rng.standard_normal((F - c, F - c)) + 1j * rng.standard_normal((F - c, F - c)))
    signal = Y @ R.T
    stack = (X @ T.T + signal).T                         # [F][n]
    f, _ = clutter.clutter_filter(stack, c)
    assert np.max(np.abs(f - signal.T)) <= 1e-9 * np.max(np.abs(stack))


def test_static_tissue_removed():
    """Tissue constant over frames plus c = 1 removes it exactly (no blood)."""
    rng = np.random.default_rng(4)
    img = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    stack = np.broadcast_to(img, (25, 500)).copy()
    f, lam = clutter.clutter_filter(stack, 1)
    assert np.max(np.abs(f)) <= 1e-10 * np.max(np.abs(stack))
    assert np.allclose(lam[1:], 0, atol=1e-9 * lam[0])


def test_wrong_conjugation_fails():
    """A planted transposed/conjugated Gram (I^T I instead of I^H I) breaks the
    equality with the SVD route."""
    s = _stack(seed=13)
    I = clutter.casorati(s)
    lam, Vc = clutter.clutter_subspace(I.T @ I, 3)
    bad = (I - (I @ Vc) @ Vc.conj().T).T
    good, _ = clutter.clutter_filter_svd(s, 3)
    assert np.linalg.norm(bad - good) > 1e-3 * np.linalg.norm(s)


# ---------------------------------------------------------------- NCC localiser

def test_separable_equals_direct():
    """Section II-A4 / Fig. 1g: two 1D correlations reproduce the 2D NCC."""
    rng = np.random.default_rng(5)
    I = np.abs(rng.standard_normal((3, 41, 37)) + 1j * rng.standard_normal((3, 41, 37)))
    for size, sz, su in ((7, 1.2, 1.2), (9, 1.2, 1.5), (11, 2.0, 1.0)):
        gz = localize.gaussian_taps(size, sz)
        gu = localize.gaussian_taps(size, su)
        a = localize.ncc_map(I, np.outer(gz, gu))
        b = localize.ncc_map_separable(I, gz, gu)
        assert np.max(np.abs(a - b)) <= 1e-12


def test_ncc_template_is_one_and_affine_invariant():
    """The template itself correlates to exactly 1 at its centre; NCC is unchanged
    by I -> a I + b (a > 0) away from the zero-padded border."""
    Kt = localize.template(9, 1.2, 1.2)
    img = np.zeros((30, 30))
    img[10:19, 12:21] = Kt
    N = localize.ncc_map(img, Kt)
    assert abs(N[14, 16] - 1.0) < 1e-12
    rng = np.random.default_rng(6)
    I = rng.uniform(0, 1, (40, 40))
    a = localize.ncc_map(I, Kt)
    b = localize.ncc_map(3.7 * I + 2.2, Kt)
    assert np.max(np.abs(a[4:-4, 4:-4] - b[4:-4, 4:-4])) < 1e-10
    c = localize.ncc_map(1 - I, Kt)              # an inverted image flips the sign
    assert np.max(np.abs(a[4:-4, 4:-4] + c[4:-4, 4:-4])) < 1e-10


def test_subpixel_gaussian_fit_exact():
    """ln of a sampled Gaussian is a parabola, so the 3-point fit is exact."""
    for x0 in (-0.43, -0.1, 0.0, 0.27, 0.49):
        s = 1.7
        f = lambda x: 2.3 * np.exp(-(x - x0) ** 2 / (2 * s * s))
        d = localize.subpixel(f(-1.0), f(0.0), f(1.0))
        assert abs(d - x0) < 1e-12
    # parabolic fallback on a parabola with a non-positive sample
    p = lambda x: 1.0 - 2.0 * (x - 0.2) ** 2
    assert abs(localize.subpixel(p(-1.0), p(0.0), p(1.0)) - 0.2) < 1e-12
    assert localize.subpixel(1.0, 2.0, 1.0) == 0.0


def _spot_case(seed=21, sigma=1.2, nz=96, nu=100, n=18):
    img, centres = arrays.gaussian_spots(nz, nu, n, sigma, seed, spacing=3 * 9.0)
    return img, centres


def _detect(img, size=9, sigma=1.2, tau=0.5, alpha=0.05):
    Kt = localize.template(size, sigma, sigma)
    N = localize.ncc_map(img, Kt)
    return localize.detect_frame(img, N, img.max(), tau, alpha), N


def test_isolated_spots_within_005_px():
    """Isolated noise-free Gaussian spots (sigma = template sigma) are localised
    within 0.05 pixel of their true centres."""
    for seed in (21, 22, 23):
        img, centres = _spot_case(seed)
        det, _ = _detect(img)
        assert len(det) == len(centres)
        pos = np.array([(z + dz, u + du) for (z, u, dz, du, _) in det])
        for c in centres:
            d = np.min(np.hypot(*(pos - c).T))
            assert d < 0.05, (c, d)


def test_spot_at_pixel_centre_and_mirror():
    """A spot at a pixel centre gives zero offset; mirroring the image mirrors the
    positions; an integer shift shifts them exactly."""
    zz, uu = np.meshgrid(np.arange(40), np.arange(44), indexing="ij")
    img = np.exp(-((zz - 17) ** 2 + (uu - 23) ** 2) / (2 * 1.2 ** 2))
    det, _ = _detect(img)
    assert len(det) == 1 and det[0][:2] == (17, 23)
    assert abs(det[0][2]) < 1e-12 and abs(det[0][3]) < 1e-12
    img2 = np.exp(-((zz - 17.3) ** 2 + (uu - 20.6) ** 2) / (2 * 1.2 ** 2))
    d1, _ = _detect(img2)
    d2, _ = _detect(img2[:, ::-1])
    assert len(d1) == len(d2) == 1
    assert abs((d1[0][1] + d1[0][3]) - (43 - (d2[0][1] + d2[0][3]))) < 1e-12
    assert abs((d1[0][0] + d1[0][2]) - (d2[0][0] + d2[0][2])) < 1e-12
    shifted = np.zeros_like(img2)
    shifted[3:, 5:] = img2[:-3, :-5]
    d3, _ = _detect(shifted)
    assert d3[0][0] == d1[0][0] + 3 and d3[0][1] == d1[0][1] + 5
    assert abs(d3[0][2] - d1[0][2]) < 1e-12 and abs(d3[0][3] - d1[0][3]) < 1e-12


def test_thresholds_and_tie_break():
    """A plateau of two equal NCC maxima yields exactly one detection, the earlier
    one in raster order: a pixel must exceed its earlier neighbours and only match
    its later ones, so the later pixel of the pair fails against the earlier one.
    Weak spots below alpha * max are rejected."""
    N = np.zeros((7, 7))
    N[3, 2] = N[3, 3] = 0.9
    I = np.ones((7, 7))
    det = localize.detect_frame(I, N, 1.0, 0.5, 0.05)
    assert [(z, u) for (z, u, *_r) in det] == [(3, 2)]
    I2 = np.full((7, 7), 0.01)
    assert localize.detect_frame(I2, N, 1.0, 0.5, 0.05) == []


def test_density_map_bins():
    locs = np.zeros(4, dtype=localize.LOC_DTYPE)
    locs["plane"] = [0, 0, 1, 1]
    locs["z"] = [0.0, 0.26, 5.49, -0.6]
    locs["u"] = [0.0, -0.26, 2.01, 1.0]
    d = pipeline.density_map(locs, 2, 8, 8)
    assert d.sum() == 3                       # the last record falls off the grid
    assert d[0, 1, 1] == 1 and d[0, 1, 0] == 1 and d[1, 11, 5] == 1


def test_ssim_identity_and_range():
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 1, (40, 40))
    assert abs(pipeline.ssim(a, a) - 1.0) < 1e-12
    assert pipeline.ssim(a, rng.uniform(0, 1, (40, 40))) < 0.2


def test_ssim_constant_images_closed_form():
    """Constant images p and q have zero local variance, so SSIM reduces to its
    luminance term (2pq + C1)/(p^2 + q^2 + C1) with C1 = (0.01 R)^2 (Wang et al.
    2004): 0.3001/0.3401 for p = 0.3, q = 0.5, R = 1, at every pixel."""
    a = np.full((23, 31), 0.3)
    b = np.full((23, 31), 0.5)
    assert abs(pipeline.ssim(a, b, data_range=1.0) - 0.3001 / 0.3401) < 1e-13
    assert abs(pipeline.ssim(a, a, data_range=1.0) - 1.0) < 1e-13


def test_ssim_brute_force_windows():
    """SSIM equals the mean over pixels of the index computed from explicit
    Gaussian-weighted local statistics (sigma 1.5, radius 5, mirror boundary
    without repeating the edge sample), summed pixel by pixel; and it is
    symmetric and invariant under a joint transpose."""
    rng = np.random.default_rng(7)
    a = rng.uniform(0, 1, (14, 17))
    b = 0.6 * a + 0.4 * rng.uniform(0, 1, (14, 17))
    R = 1.0
    x = np.arange(-5, 6)
    w = np.exp(-x * x / (2 * 1.5 ** 2))
    w2 = np.outer(w, w) / w.sum() ** 2

    def mirror(i, n):
        while i < 0 or i >= n:
            i = -i if i < 0 else 2 * (n - 1) - i
        return i

    vals = []
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            s = {"a": 0.0, "b": 0.0, "aa": 0.0, "bb": 0.0, "ab": 0.0}
            for di in range(-5, 6):
                for dj in range(-5, 6):
                    ii, jj = mirror(i + di, a.shape[0]), mirror(j + dj, a.shape[1])
                    wt = w2[di + 5, dj + 5]
                    s["a"] += wt * a[ii, jj]
                    s["b"] += wt * b[ii, jj]
                    s["aa"] += wt * a[ii, jj] ** 2
                    s["bb"] += wt * b[ii, jj] ** 2
                    s["ab"] += wt * a[ii, jj] * b[ii, jj]
            va, vb = s["aa"] - s["a"] ** 2, s["bb"] - s["b"] ** 2
            cab = s["ab"] - s["a"] * s["b"]
            c1, c2 = (0.01 * R) ** 2, (0.03 * R) ** 2
            vals.append((2 * s["a"] * s["b"] + c1) * (2 * cab + c2) /
                        ((s["a"] ** 2 + s["b"] ** 2 + c1) * (va + vb + c2)))
    got = pipeline.ssim(a, b, data_range=R)
    assert abs(got - np.mean(vals)) < 1e-12
    assert abs(pipeline.ssim(b, a, data_range=R) - got) < 1e-13
    assert abs(pipeline.ssim(a.T, b.T, data_range=R) - got) < 1e-13


def test_fp32_sensitivity_file_is_current():
    """tests/golden/fp32_sensitivity_tiny.json (the oracle's own response to
    FP32-sized errors in its input projections, which sets how close a whole-path
    comparison with the FP32 GPU path can be) matches a fresh run of the script
    that wrote it; FP32 rounding alone already moves decidable detections by a
    few 1e-4 px, and the response grows with the input error."""
    import importlib.util
    import json
    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("mk", os.path.join(here, "make_fp32_sensitivity.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    stored = json.load(open(os.path.join(here, "fp32_sensitivity_tiny.json")))
    fresh = mk.measure()
    assert stored["reference_detections"] == fresh["reference_detections"]
    for name, vals in fresh["variants"].items():
        for k, v in vals.items():
            assert np.isclose(stored["variants"][name][k], v, rtol=1e-6, atol=0), (name, k)
    r, p = fresh["variants"]["fp32"], fresh["variants"]["fp32_perturbed"]
    assert 1e-5 < r["max_dpos_decidable_px"] < p["max_dpos_decidable_px"]
    assert r["max_abs_dncc"] < p["max_abs_dncc"]
