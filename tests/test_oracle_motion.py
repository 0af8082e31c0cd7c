"""Pins of the motion-estimation oracle (CPU only): the Fourier-domain NCC
against its plain definition, exact integer shifts, sub-pixel shifts made by
the Fourier shift theorem, swap antisymmetry, the window edge, and the
averaging into a 3D motion."""
import numpy as np

from oracle import motion


def _speckle(nz, nu, seed, smooth=1.5):
    """Band-limited random image (a smoothed Rayleigh-like envelope)."""
    g = np.random.default_rng(seed)
    x = g.standard_normal((nz, nu)) + 1j * g.standard_normal((nz, nu))
    kz = np.fft.fftfreq(nz)[:, None]
    ku = np.fft.fftfreq(nu)[None, :]
    h = np.exp(-2 * (np.pi * smooth) ** 2 * (kz ** 2 + ku ** 2))
    return np.abs(np.fft.ifft2(np.fft.fft2(x) * h))


def _fourier_shift(img, dz, du):
    """img moved by (dz, du) pixels (circularly, band-limited interpolation)."""
    nz, nu = img.shape
    kz = np.fft.fftfreq(nz)[:, None]
    ku = np.fft.fftfreq(nu)[None, :]
    return np.real(np.fft.ifft2(np.fft.fft2(img) * np.exp(-2j * np.pi * (kz * dz + ku * du))))


def test_fft_surface_is_the_plain_definition():
    rng = np.random.default_rng(1)
    a, b = rng.uniform(0, 1, (12, 10)), rng.uniform(0, 1, (12, 10))
    c = motion.ncc_surface(a, b)
    lags = [(0, 0), (1, 0), (0, 1), (-2, 3), (5, -4), (11, 9), (-6, -5)]
    want = motion.ncc_direct(a, b, lags)
    got = np.array([c[dz % 12, du % 10] for dz, du in lags])
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    assert abs(motion.ncc_surface(b, b)[0, 0] - 1.0) < 1e-12


def test_integer_shifts_exact():
    ref = _speckle(40, 48, 2)
    for dz, du in ((0, 0), (2, -3), (-5, 1), (7, 7), (-8, 0), (0, 8)):
        a = np.roll(ref, (dz, du), axis=(0, 1))
        ez, eu = motion.peak(motion.ncc_surface(a, ref), 8)
        assert abs(ez - dz) < 1e-6 and abs(eu - du) < 1e-6, ((dz, du), (ez, eu))


def test_window_edge_and_beyond():
    ref = _speckle(40, 48, 3)
    # exactly on the window edge: integer lag, no sub-pixel offset on that axis
    a = np.roll(ref, (4, 1), axis=(0, 1))
    assert motion.peak(motion.ncc_surface(a, ref), 4) == (4.0, 1.0)
    # beyond the window: not representable, the estimate stays inside it
    a = np.roll(ref, (9, 0), axis=(0, 1))
    ez, eu = motion.peak(motion.ncc_surface(a, ref), 6)
    assert abs(ez) <= 6 and abs(eu) <= 6 and abs(ez - 9) > 2


def test_subpixel_shifts():
    """Band-limited sub-pixel shifts are recovered to within 0.1 px (the paper
    reports errors up to about 0.06 px near half-pixel shifts)."""
    ref = _speckle(64, 64, 4, smooth=2.0)
    errs = []
    for s in (0.1, 0.25, 0.4, 0.5, -0.3):
        a = _fourier_shift(ref, s, -0.5 * s + 1.0)
        ez, eu = motion.peak(motion.ncc_surface(a, ref), 8)
        errs.append(max(abs(ez - s), abs(eu - (-0.5 * s + 1.0))))
    assert max(errs) < 0.1, errs


def test_swap_antisymmetry():
    """Correlating the reference against the frame gives the opposite lag."""
    ref = _speckle(50, 36, 5)
    a = _fourier_shift(ref, 1.3, -2.2)
    f = motion.peak(motion.ncc_surface(a, ref), 8)
    r = motion.peak(motion.ncc_surface(ref, a), 8)
    assert abs(f[0] + r[0]) < 1e-6 and abs(f[1] + r[1]) < 1e-6


def test_estimate_averages_and_composes_3d():
    """RC slices moved by (dz1, dx) and CR slices by (dz2, dy) per frame: every
    transmit sees its shift, and the 3D motion is (dx, dy, (dz1 + dz2) / 2)."""
    nz, nu, K, F = 32, 36, 3, 4
    shifts_rc = [(0, 0), (1, 2), (-2, 1), (3, -1)]
    shifts_cr = [(0, 0), (3, -2), (0, 4), (-1, -3)]
    S = np.zeros((2, K, F, nz, nu), np.complex128)
    for o, shifts in enumerate((shifts_rc, shifts_cr)):
        for k in range(K):
            base = _speckle(nz, nu, 10 * o + k) * np.exp(1j * 0.3 * k)
            for f, (dz, du) in enumerate(shifts):
                S[o, k, f] = np.roll(base, (dz, du), axis=(0, 1))
    disp, mot = motion.estimate(S, 0, 6)
    for f in range(F):
        for k in range(K):
            assert np.allclose(disp[0, k, f], shifts_rc[f], atol=1e-6)
            assert np.allclose(disp[1, k, f], shifts_cr[f], atol=1e-6)
        want = (shifts_rc[f][1], shifts_cr[f][1], 0.5 * (shifts_rc[f][0] + shifts_cr[f][0]))
        assert np.allclose(mot[f], want, atol=1e-6)
