"""Pins of the CNN localiser oracle (CPU only)."""
import numpy as np
from scipy import signal

from oracle import cnn


def test_conv_matches_library_correlation():
    """conv3x3 = sum over input channels of scipy's 2D correlation ('same', zero fill)."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 9, 11))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(signal.correlate2d(x[c], w[o, c], mode="same", boundary="fill")
                         for c in range(3))
        assert np.allclose(y[o], ref, atol=1e-12)


def test_delta_kernel_is_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 7, 6))
    w = np.zeros((5, 5, 3, 3))
    for c in range(5):
        w[c, c, 1, 1] = 1.0
    assert np.array_equal(cnn.conv3x3(x, w, np.zeros(5)), x)


def test_depth_to_space_roundtrip_and_placement():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((64, 3, 4))
    z = cnn.depth_to_space(y)
    assert z.shape == (24, 32)
    assert np.array_equal(cnn.space_to_depth(z), y)
    assert z[1 * 8 + 2, 3 * 8 + 5] == y[2 * 8 + 5, 1, 3]


def _tiny_params(rng, layers=2, ch=3):
    p = cnn.init_params(rng, channels=ch, layers=layers)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)   # non-zero biases too
    return p


def test_gradients_match_finite_differences():
    """Analytic gradients of every parameter vs central differences (rel <= 1e-6)."""
    rng = np.random.default_rng(3)
    layers = 2
    p = _tiny_params(rng, layers)
    img = rng.uniform(0, 1, (5, 6))
    T = cnn.target_map(np.array([[2.3, 3.1]]), 5, 6)
    _, g = cnn.loss_and_grad(p, img, T, layers)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = cnn.loss_and_grad(p, img, T, layers)
            flat[i] = old - h
            lm, _ = cnn.loss_and_grad(p, img, T, layers)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), abs(an), 1e-8) + 1e-10, (k, i, fd, an)


def test_target_peak_and_decode_roundtrip():
    """A blob centred on an MB decodes back to that MB within half a fine pixel."""
    pos = np.array([[3.27, 5.61], [10.0, 2.0]])
    T = cnn.target_map(pos, 14, 9)
    assert np.exp(-0.25) - 1e-12 <= T.max() <= 1.0     # a blob peak is at most half a fine pixel off a sample
    d = cnn.decode(T, 0.5)
    assert d.shape == (2, 2)
    for p in pos:
        assert np.min(np.abs(d - p).max(axis=1)) <= 0.5 / cnn.R + 1e-12


def test_adam_matches_closed_form_first_step():
    """First Adam step moves every weight by lr * sign(g) (bias correction)."""
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    cnn.adam_step(p, g, {}, lr=0.01, eps=0.0)
    assert np.allclose(p["a"], [0.99, -1.99, 2.99])


def test_adam_bias_correction_later_steps():
    """Adam's bias correction at t = 2 and 3, from hand-derived closed forms.

    Constant gradient g (eps = 0): m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so
    the corrected moments are g and g^2 and every step moves a weight by exactly
    lr sign(g).  Gradient +1 then -1: the corrected first moment at t = 2 is
    -(1 - b1)/(1 + b1) = -1/19 and the corrected second moment is 1, so the
    second step moves the weight by +lr/19.  Without the bias correction the
    second step would be (1 - b1^2)/sqrt(1 - b2^2) = 4.25 times larger."""
    lr = 0.01
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    st = {}
    for t in range(1, 4):
        cnn.adam_step(p, g, st, lr=lr, eps=0.0)
        assert np.allclose(p["a"], np.array([1.0, -2.0, 3.0]) - t * lr * np.sign(g["a"]),
                           rtol=0, atol=1e-14), t
    q = {"w": np.array([0.0])}
    st = {}
    cnn.adam_step(q, {"w": np.array([1.0])}, st, lr=lr, eps=0.0)
    assert abs(q["w"][0] + lr) < 1e-15
    cnn.adam_step(q, {"w": np.array([-1.0])}, st, lr=lr, eps=0.0)
    assert abs(q["w"][0] - (-lr + lr / 19.0)) < 1e-15
