"""Pins of the oracle's MLP environment (frequency encoding, ReLU layers,
linear head, bfloat16 rounding of the encoded input and hidden activations)."""
import math

import numpy as np
import pytest

from paper_2603_00413_amd import synth


def _net(n_layers=1, width=64, in_pad=64):
    Ws = [np.zeros((width, in_pad))] + [np.zeros((width, width)) for _ in range(n_layers - 1)]
    Ws.append(np.zeros((3, width)))
    Bs = [np.zeros(width) for _ in range(n_layers)] + [np.zeros(3)]
    return Ws, Bs


def test_hand_computed_tiny_net(oracle_lib):
    """d = (0.6, 0.8, 0) is already unit; bf16(0.6) = 0.6015625 and
    bf16(0.8) = 0.80078125 by hand (0x3F19999A -> 0x3F1A, 0x3F4CCCCD -> 0x3F4D)."""
    Ws, Bs = _net()
    Ws[0][0, 0] = 1.0          # h0 = relu(d_x)
    Ws[0][1, 1] = 1.0          # h1 = relu(d_y)
    Ws[0][2, 1] = -1.0         # h2 = relu(-d_y) = 0
    Ws[1][0, 0] = 1.0
    Ws[1][1, 1] = 2.0
    Ws[1][2, 0] = 0.5
    Ws[1][2, 1] = 0.25
    Bs[1][:] = [0.5, 0.0, -1.0]
    env = oracle_lib.Env(mlp=(Ws, Bs, 6))
    out = env.eval(np.array([[0.6, 0.8, 0.0], [1.2, 1.6, 0.0]]))
    x, y = 0.6015625, 0.80078125
    expect = [x + 0.5, 2 * y, 0.5 * x + 0.25 * y - 1.0]
    np.testing.assert_allclose(out[0], expect, atol=1e-15)
    np.testing.assert_allclose(out[1], expect, atol=1e-15)   # direction only
    ex = oracle_lib.Env(mlp=(Ws, Bs, 6), exact=True).eval(np.array([[0.6, 0.8, 0.0]]))
    np.testing.assert_allclose(ex[0], [1.1, 1.6, 0.3 + 0.2 - 1.0], atol=1e-15)


@pytest.mark.parametrize("k", [0, 2, 5])
def test_frequency_encoding_components(oracle_lib, k):
    """A net that passes one encoding band through +-ReLU pairs returns
    bf16(sin(2^k pi d_c)) and bf16(cos(2^k pi d_c))."""
    Ws, Bs = _net()
    cols = [3 + 6 * k + 0, 3 + 6 * k + 1, 3 + 6 * k + 5]   # sin x, sin y, cos z
    for o, c in enumerate(cols):
        Ws[0][2 * o, c] = 1.0
        Ws[0][2 * o + 1, c] = -1.0
        Ws[1][o, 2 * o] = 1.0
        Ws[1][o, 2 * o + 1] = -1.0
    env = oracle_lib.Env(mlp=(Ws, Bs, 6))
    rng = np.random.default_rng(k)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = env.eval(d)
    w = (2 ** k) * math.pi
    ref = np.stack([np.sin(w * d[:, 0]), np.sin(w * d[:, 1]), np.cos(w * d[:, 2])], 1)
    ref = synth.round_to_bf16(ref.astype(np.float32)).astype(np.float64)
    np.testing.assert_allclose(out, ref, atol=0, rtol=0)


def test_bf16_rounding_points_change_the_value(oracle_lib):
    """The emulated network differs from the exact FP64 one by bf16-sized
    amounts (about 2^-8 relative), not by more."""
    Ws, Bs = synth.env_mlp_weights(seed=3, n_layers=3, width=64)
    mlp = ([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6)
    rng = np.random.default_rng(1)
    d = rng.normal(size=(500, 3))
    a = oracle_lib.Env(mlp=mlp).eval(d)
    b = oracle_lib.Env(mlp=mlp, exact=True).eval(d)
    err = np.abs(a - b) / np.abs(b).mean()
    assert err.max() < 0.05 and err.mean() > 1e-5


def test_mlp_direction_gradient_fd(oracle_lib):
    """Input gradient of the exact network against central differences."""
    Ws, Bs = synth.env_mlp_weights(seed=3, n_layers=3, width=64)
    mlp = ([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6)
    env = oracle_lib.Env(mlp=mlp, exact=True)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.normal(size=d.shape)
    ad = env.eval_grad(d, g)
    h = 1e-6
    for c in range(3):
        dp, dm = d.copy(), d.copy()
        dp[:, c] += h
        dm[:, c] -= h
        fd = ((env.eval(dp) - env.eval(dm)) * g).sum(1) / (2 * h)
        ok = np.abs(fd - ad[:, c]) < 1e-4 * (np.abs(ad[:, c]) + 1)   # ReLU kinks inside +-h are rare
        assert ok.mean() > 0.98
        np.testing.assert_allclose(fd[ok], ad[ok, c], rtol=1e-6, atol=1e-6)
    # the gradient is tangential: the environment depends on direction only
    assert np.abs((ad * d).sum(1)).max() < 1e-10
