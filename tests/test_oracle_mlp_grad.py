"""Pins of the oracle's gradient with respect to the environment MLP's
weights and biases (the network stands in for the paper's learned
environment field, whose parameters the ray-tracing stage optimises jointly
with the mesh): central finite differences of the FP64 render, the linearity
of the image in the linear head (an Euler identity), and, without absorption,
the head-bias gradient from energy conservation."""
import numpy as np
import pytest

from paper_2603_00413_amd import synth


def _scene(oracle_lib, sigma=(0.5, 0.2, 0.1), res=12, layers=2):
    V, F = synth.icosphere(2)
    Ws, Bs = synth.env_mlp_weights(seed=11, n_layers=layers, width=64)
    Ws = [w.astype(np.float64) for w in Ws]
    Bs = [b.astype(np.float64) for b in Bs]
    env = oracle_lib.Env(mlp=(Ws, Bs, 6))
    sc = oracle_lib.Scene(V, F, 1.5, sigma, env, 4)
    cam = synth.look_at_camera((0.3, 0.4, 2.9), res, res)
    o, d = oracle_lib.camera_rays(cam)
    return sc, Ws, Bs, o, d


def _loss(oracle_lib, sc, Ws, Bs, o, d, g):
    s2 = sc.with_(env=oracle_lib.Env(mlp=(Ws, Bs, 6)))
    return float((s2.trace(o, d)["rgb"] * g).sum())


def test_directional_fd(oracle_lib):
    """sum_k dP_k xi_k equals the central difference of the loss along a
    random direction xi in parameter space (every weight and bias moves)."""
    sc, Ws, Bs, o, d = _scene(oracle_lib)
    g = np.random.default_rng(1).normal(size=o.shape)
    res = sc.trace_grad(o, d, g, want_mlp=True)
    dW, dB = res["d_mlp"]
    rng = np.random.default_rng(2)
    xiW = [rng.normal(size=w.shape) * (w != 0) for w in Ws]   # keep the zero padding
    xiB = [rng.normal(size=b.shape) for b in Bs]
    an = sum((a * x).sum() for a, x in zip(dW, xiW)) + sum((a * x).sum() for a, x in zip(dB, xiB))
    h = 1e-6
    lp = _loss(oracle_lib, sc, [w + h * x for w, x in zip(Ws, xiW)], [b + h * x for b, x in zip(Bs, xiB)],
               o, d, g)
    lm = _loss(oracle_lib, sc, [w - h * x for w, x in zip(Ws, xiW)], [b - h * x for b, x in zip(Bs, xiB)],
               o, d, g)
    fd = (lp - lm) / (2 * h)
    assert abs(an - fd) <= 1e-6 * max(abs(fd), 1.0), (an, fd)


@pytest.mark.parametrize("which", [("W", 0, 5, 3), ("W", 1, 17, 40), ("W", 2, 1, 9),
                                   ("B", 0, 7, None), ("B", 1, 33, None), ("B", 2, 2, None)])
def test_single_parameter_fd(oracle_lib, which):
    """One weight or bias at a time (first layer, hidden layer, head)."""
    sc, Ws, Bs, o, d = _scene(oracle_lib)
    g = np.random.default_rng(3).normal(size=o.shape)
    dW, dB = sc.trace_grad(o, d, g, want_mlp=True)["d_mlp"]
    kind, layer, i, j = which
    h = 1e-6

    def moved(s):
        W2 = [w.copy() for w in Ws]
        B2 = [b.copy() for b in Bs]
        if kind == "W":
            W2[layer][i, j] += s
        else:
            B2[layer][i] += s
        return _loss(oracle_lib, sc, W2, B2, o, d, g)

    fd = (moved(h) - moved(-h)) / (2 * h)
    an = dW[layer][i, j] if kind == "W" else dB[layer][i]
    assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3), (an, fd)


def test_linear_head_euler_identity(oracle_lib):
    """The image is linear in the head (E = W_h a + b_h, and the pixel is a
    weighted sum of lookups), so sum(W_h * dW_h) + sum(b_h * db_h) equals the
    loss sum(g * C) itself."""
    sc, Ws, Bs, o, d = _scene(oracle_lib)
    g = np.random.default_rng(4).normal(size=o.shape)
    r = sc.trace_grad(o, d, g, want_mlp=True)
    dW, dB = r["d_mlp"]
    lhs = (Ws[-1] * dW[-1]).sum() + (Bs[-1] * dB[-1]).sum()
    rhs = (g * r["rgb"]).sum()
    assert abs(lhs - rhs) <= 1e-10 * max(abs(rhs), 1.0)


def test_head_bias_from_energy_conservation(oracle_lib):
    """Without absorption the weights of a pixel's environment lookups sum to
    1 - W_trunc (R + T = 1 at every split), so the gradient of sum(g * C) with
    respect to the head bias of channel c is sum_pixels g_c (1 - W_trunc,c)."""
    sc, Ws, Bs, o, d = _scene(oracle_lib, sigma=(0.0, 0.0, 0.0))
    g = np.random.default_rng(5).normal(size=o.shape)
    dB = sc.trace_grad(o, d, g, want_mlp=True)["d_mlp"][1]
    wt = sc.trace(o, d)["wtrunc"]
    np.testing.assert_allclose(dB[-1], (g * (1.0 - wt)).sum(0), rtol=1e-12, atol=1e-12)
