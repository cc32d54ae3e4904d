"""Pins of the oracle's MLP environment (frequency encoding, ReLU layers,
linear head, plain FP64) and of its gradient-kink margins."""
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
    """h = relu(W0 u): d_x, d_y and relu(-d_y) = 0 for d = (0.6, 0.8, 0);
    E = (h0 + 0.5, 2 h1, 0.5 h0 + 0.25 h1 - 1) = (1.1, 1.6, -0.5), and the
    same for a scaled direction (the environment sees the direction only)."""
    Ws, Bs = _net()
    Ws[0][0, 0] = 1.0          # h0 = relu(d_x)
    Ws[0][1, 1] = 1.0          # h1 = relu(d_y)
    Ws[0][2, 1] = -1.0         # h2 = relu(-d_y) = 0
    Ws[1][0, 0] = 1.0
    Ws[1][1, 1] = 2.0
    Ws[1][2, 0] = 0.5
    Ws[1][2, 1] = 0.25
    Ws[1][2, 2] = 7.0          # reads the dead unit: contributes nothing
    Bs[1][:] = [0.5, 0.0, -1.0]
    env = oracle_lib.Env(mlp=(Ws, Bs, 6))
    out = env.eval(np.array([[0.6, 0.8, 0.0], [1.2, 1.6, 0.0]]))
    np.testing.assert_allclose(out[0], [1.1, 1.6, -0.5], atol=1e-15)
    np.testing.assert_allclose(out[1], [1.1, 1.6, -0.5], atol=1e-15)


@pytest.mark.parametrize("k", [0, 2, 5])
def test_frequency_encoding_components(oracle_lib, k):
    """A net that passes one encoding band through +-ReLU pairs returns
    sin(2^k pi d_x), sin(2^k pi d_y) and cos(2^k pi d_z): the band's slots are
    3 + 6k + (0, 1, 2) for sin and 3 + 6k + (3, 4, 5) for cos."""
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
    np.testing.assert_allclose(out, ref, atol=1e-13, rtol=0)


def test_mlp_direction_gradient_fd(oracle_lib):
    """Input gradient of the network against central differences, away from
    the ReLU kinks (margin > 1e-5 rad, 10 x the step)."""
    Ws, Bs = synth.env_mlp_weights(seed=3, n_layers=3, width=64)
    mlp = ([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6)
    env = oracle_lib.Env(mlp=mlp)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    g = rng.normal(size=d.shape)
    ad = env.eval_grad(d, g)
    far = env.kink_margin(d) > 1e-5
    assert far.mean() > 0.8
    h = 1e-6
    for c in range(3):
        dp, dm = d.copy(), d.copy()
        dp[:, c] += h
        dm[:, c] -= h
        fd = ((env.eval(dp) - env.eval(dm)) * g).sum(1) / (2 * h)
        np.testing.assert_allclose(fd[far], ad[far, c], rtol=1e-6, atol=1e-6)
    # the gradient is tangential: the environment depends on direction only
    assert np.abs((ad * d).sum(1)).max() < 1e-10


def test_mlp_kink_margin(oracle_lib):
    """One hidden unit z = d_x: its kink is the great circle d_x = 0, and the
    margin of a unit direction is asin|d_x| to first order, i.e. |d_x| / sqrt(1 - d_x^2)."""
    Ws, Bs = _net()
    Ws[0][0, 0] = 1.0
    Ws[1][0, 0] = 1.0
    env = oracle_lib.Env(mlp=(Ws, Bs, 6))
    dx = np.array([1e-7, -3e-6, 0.3, -0.6])
    d = np.stack([dx, np.sqrt(1 - dx ** 2), np.zeros_like(dx)], 1)
    m = env.kink_margin(d)
    np.testing.assert_allclose(m, np.abs(dx) / np.sqrt(1 - dx ** 2), rtol=1e-12)
    # the value is continuous across the kink (relu(d_x)), only its slope jumps
    e = env.eval(d)
    np.testing.assert_allclose(e[:, 0], np.maximum(dx, 0), atol=1e-15)


def test_equirect_kink_margin(oracle_lib):
    """On an 8 x 4 map the texel-centre lines are phi = 2 pi ((i + 1/2) / 8 - 1/2)
    and theta = pi (j + 1/2) / 4.  On the equator, a direction on a phi line has
    margin 0; one half a texel off it has margin pi / 8 (min with the theta
    lines, pi / 8 away as well)."""
    tex = np.random.default_rng(0).uniform(0.2, 1.0, size=(4, 8, 3))
    env = oracle_lib.Env(tex=tex)
    phi_line = 2 * math.pi * (2.5 / 8 - 0.5)
    phis = np.array([phi_line, phi_line + math.pi / 8, phi_line + 1e-7])
    d = np.stack([np.sin(phis), np.zeros(3), -np.cos(phis)], 1)   # phi = atan2(x, -z), theta = pi/2
    m = env.kink_margin(d)
    assert m[0] < 1e-12
    np.testing.assert_allclose(m[1], math.pi / 8, rtol=1e-9)
    np.testing.assert_allclose(m[2], 1e-7, rtol=1e-6)
