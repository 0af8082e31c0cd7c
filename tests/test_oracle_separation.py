"""Pins of the MB-separation oracle (CPU only): the band layout, the subsets as
a partition of the spectrum, pure tones, the flow direction of a moving
scatterer's phase, and the DFT route against a direct slow-time convolution."""
import numpy as np

from oracle import separation


def test_band_layout():
    for F, S in ((300, 3), (20, 3), (21, 2), (300, 1), (7, 3)):
        bins = separation.band_bins(F, S)
        H = (F - 1) // 2
        flat = [k for b in bins for k in b]
        assert len(flat) == len(set(flat)) == 2 * H                 # disjoint, all non-DC bins
        assert 0 not in flat and (F % 2 == 1 or F // 2 not in flat)  # DC and Nyquist excluded
        assert sorted(k for b in bins[:S] for k in b) == list(range(1, H + 1))
        for s in range(S):                                           # down mirrors up
            assert sorted((-k) % F for k in bins[S + s]) == sorted(bins[s])
        sizes = [len(b) for b in bins[:S]]
        assert max(sizes) - min(sizes) <= 1
    assert separation.band_bins(300, 3)[0] == list(range(1, 50))


def test_subsets_partition_the_signal():
    """The subsets plus the DC and Nyquist components give back the input."""
    rng = np.random.default_rng(0)
    for F in (300, 21):
        x = rng.standard_normal((F, 3, 4)) + 1j * rng.standard_normal((F, 3, 4))
        sub = separation.separate(x, 3)
        X = np.fft.fft(x, axis=0)
        rest = np.zeros_like(X)
        rest[0] = X[0]
        if F % 2 == 0:
            rest[F // 2] = X[F // 2]
        assert np.allclose(sub.sum(axis=0) + np.fft.ifft(rest, axis=0), x, atol=1e-12)


def test_pure_tones_land_in_one_subset():
    F, S = 300, 3
    n = np.arange(F)
    bins = separation.band_bins(F, S)
    for k in (1, 49, 50, 99, 100, 149, 151, 200, 250, 299):
        x = np.exp(2j * np.pi * k * n / F)[:, None, None] * np.ones((1, 2, 2))
        sub = separation.separate(x, S)
        owner = [i for i, b in enumerate(bins) if k in b]
        assert len(owner) == 1
        for i in range(2 * S):
            want = x if i == owner[0] else 0 * x
            assert np.allclose(sub[i], want, atol=1e-12)


def test_upward_motion_is_positive_frequency():
    """A scatterer rising by v per frame gives the pixel the phase
    exp(-i 4 pi f0 z(t) / c) (the beamformer's baseband convention): slow
    upward motion lands in the slowest up subset, fast downward motion in the
    fastest down subset."""
    F, S = 300, 3
    f0, c, fr = 6e6, 1540.0, 400.0
    t = np.arange(F) / fr
    lam_half = c / (2 * f0)                     # axial speed of one bin: lam/2 * fr / F
    for v_bins, want in ((10, 0), (-140, 2 * S - 1), (75, 1)):
        v = v_bins * lam_half * fr / F          # m/s, towards the probe when positive
        z = 30e-3 - v * t
        x = np.exp(-4j * np.pi * f0 * z / c)[:, None, None]
        sub = separation.separate(x, S)
        energy = [float(np.sum(np.abs(s) ** 2)) for s in sub]
        assert int(np.argmax(energy)) == want, (v_bins, energy)


def test_dft_route_is_a_circular_convolution():
    """Each subset equals the circular convolution of the slow-time signal
    with the inverse DFT of its mask (brute force, small F)."""
    rng = np.random.default_rng(1)
    F, S = 12, 2
    x = rng.standard_normal((F, 1, 2)) + 1j * rng.standard_normal((F, 1, 2))
    sub = separation.separate(x, S)
    for i, bins in enumerate(separation.band_bins(F, S)):
        h = np.zeros(F, complex)
        for k in bins:
            h += np.exp(2j * np.pi * k * np.arange(F) / F) / F
        y = np.zeros_like(x)
        for n in range(F):
            for m in range(F):
                y[n] += h[(n - m) % F] * x[m]
        assert np.allclose(sub[i], y, atol=1e-12)
