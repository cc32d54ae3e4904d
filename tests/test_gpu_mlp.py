"""Parity of the bf16-MFMA environment MLP with the oracle's FP64 network.

The device keeps every activation as three bf16 parts (all 24 bits of the
FP32 value) and accumulates in FP32, so it evaluates the same continuous
function as the FP64 network with FP32 rounding.  Bars: per direction,
||E_dev - E|| / max(||E||, mean/10) <= 1e-4 (the output is a signed sum of
terms as large as the mean output, so its rounding error is absolute); the
direction gradient to 1e-3 where no ReLU kink lies within 1e-5 rad.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from tests.gpu_helpers import (GradRef, check_elements, check_material, check_radiance, device, gradient_pixels, l2_upstream,
                               rgb_rel_err)

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _dirs(n, seed):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


def test_hand_computed_tiny_net_exact():
    """Same net as the oracle pin: E = (x + 0.5, 2y, 0.5x + 0.25y - 1) with
    (x, y) = d = (0.6, 0.8, 0), i.e. (1.1, 1.6, -0.5).  The three bf16 parts
    of an FP32 value sum to it exactly, so E is the FP32 evaluation of these
    expressions: within 2e-6 of the exact values."""
    dev = device()
    Ws = [np.zeros((64, 64), np.float32), np.zeros((3, 64), np.float32)]
    Bs = [np.zeros(64, np.float32), np.array([0.5, 0.0, -1.0], np.float32)]
    Ws[0][0, 0] = 1.0
    Ws[0][1, 1] = 1.0
    Ws[0][2, 1] = -1.0
    Ws[1][0, 0] = 1.0
    Ws[1][1, 1] = 2.0
    Ws[1][2, 0] = 0.5
    Ws[1][2, 1] = 0.25
    env = B.Env.mlp(Ws, Bs, 6, dev)
    d = torch.tensor([[0.6, 0.8, 0.0]] * 40, device=dev)
    E = B.dt_env_query(env, d).cpu().numpy()
    assert np.abs(E - np.array([1.1, 1.6, -0.5])).max() <= 2e-6


@pytest.mark.parametrize("width,layers", [(64, 3), (128, 4)])
def test_mlp_query_vs_oracle(width, layers):
    dev = device()
    Ws, Bs = synth.env_mlp_weights(seed=3, n_layers=layers, width=width)
    env = B.Env.mlp(Ws, Bs, 6, dev)
    oenv = oracle.Env(mlp=([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6))
    d = _dirs(20000, width + layers)
    E = B.dt_env_query(env, torch.from_numpy(d).to(dev)).cpu().numpy().astype(np.float64)
    Eo = oenv.eval(d.astype(np.float64))
    err = rgb_rel_err(E, Eo)
    _print(width, layers, "E: median", np.median(err), "max", err.max())
    assert err.max() <= 1e-4
    # input gradient, away from the ReLU kinks
    g = np.random.default_rng(1).normal(size=d.shape).astype(np.float32)
    gd = B.dt_env_query_backward(env, torch.from_numpy(d).to(dev),
                                 torch.from_numpy(g).to(dev)).cpu().numpy().astype(np.float64)
    gdo = oenv.eval_grad(d.astype(np.float64), g.astype(np.float64))
    far = oenv.kink_margin(d.astype(np.float64)) > 1e-5
    r = np.linalg.norm(gd - gdo, axis=1) / np.linalg.norm(gdo, axis=1)
    _print(width, layers, "grad: kink-free", far.mean(), "median", np.median(r[far]), "max", r[far].max())
    assert far.mean() > 0.8
    assert r[far].max() <= 1e-3


def test_trace_with_mlp_environment():
    """The icosphere scene lit by the 3 x 64 MLP: radiance and gradients."""
    from tests.gpu_helpers import Pair
    dev = device()
    wl = synth.icosphere_scene(sigma=(0.5, 0.2, 0.1), res=48)
    Ws, Bs = synth.env_mlp_weights(seed=3, n_layers=3, width=64)
    P = Pair(wl.V, wl.F, wl.ior, wl.sigma, wl.env, wl.cameras, wl.max_depth)
    P.env = B.Env.mlp(Ws, Bs, 6, dev)
    P.scene = B.Scene(P.mesh, P.ior_t, P.sigma_t, P.env)
    P.orc = oracle.Scene(P.V32.astype(np.float64), P.F, float(P.ior), P.sigma.astype(np.float64),
                         oracle.Env(mlp=([w.astype(np.float64) for w in Ws],
                                         [b.astype(np.float64) for b in Bs], 6)), wl.max_depth)
    buf, rgb, wt, fl = P.gpu_forward(tape=True)
    chk = check_radiance(P.orc, P.o, P.d, rgb, fl, P.sig, mlp=True, label="icosphere, 3 x 64 MLP")
    ref = chk["ref"]
    gr = GradRef(P.orc, P.o, P.d, ref["sig"])
    okg = gradient_pixels(chk, fl, gr.stable)
    _print("MLP trace: gradient pixels", okg.sum(), "of", len(okg))
    tgt = P.orc.with_(eta=1.52, sigma=(0.4, 0.25, 0.15)).trace(P.o, P.d)["rgb"]
    g = l2_upstream(ref["rgb"], tgt, okg)
    dV, de, ds = P.gpu_backward(buf, g)
    o, oa, sp = gr.grads(g)
    ev = check_elements(dV, o["dV"], oa["dV"], "MLP-lit dV", sp["dV"])
    ee, es = check_material(de, ds, o, oa, sp, "MLP trace")
    _print("MLP trace grads: dV", ev, "deta", ee, "dsigma", es)


@pytest.mark.parametrize("layers", [1, 3, 4])
def test_mlp_weight_gradient(layers):
    """dLoss/d(weights, biases) of the 64-wide environment MLP through the
    tracer, against the oracle's reverse-mode gradient of its FP64 network,
    element by element (against the ray-by-ray magnitudes, the oracle's
    perturbation spread and a tenth of the layer's RMS), on the pixels whose
    path is the same on both sides and off the ReLU kinks; and the device's own
    linear-head identity sum(W_h dW_h) + sum(b_h db_h) = sum(g C)."""
    from tests.gpu_helpers import Pair
    dev = device()
    wl = synth.icosphere_scene(sigma=(0.5, 0.2, 0.1), res=48)
    Ws, Bs = synth.env_mlp_weights(seed=7 + layers, n_layers=layers, width=64)
    P = Pair(wl.V, wl.F, wl.ior, wl.sigma, wl.env, wl.cameras, wl.max_depth)
    P.env = B.Env.mlp(Ws, Bs, 6, dev, want_grad=True)
    P.scene = B.Scene(P.mesh, P.ior_t, P.sigma_t, P.env)
    oenv = oracle.Env(mlp=([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6))
    P.orc = oracle.Scene(P.V32.astype(np.float64), P.F, float(P.ior), P.sigma.astype(np.float64), oenv,
                         wl.max_depth)
    buf, rgb, wt, fl = P.gpu_forward(tape=True)
    chk = check_radiance(P.orc, P.o, P.d, rgb, fl, P.sig, mlp=True, label=f"{layers} x 64 MLP")
    gr = GradRef(P.orc, P.o, P.d, chk["ref"]["sig"])
    okg = gradient_pixels(chk, fl, gr.stable)
    g = np.random.default_rng(layers).normal(size=rgb.shape) * okg[:, None]
    dV, de, ds = P.gpu_backward(buf, g)
    dW, dB = P.env.split_grad()
    o, oa, sp = gr.grads(g, want_mlp=True)
    oW, oB = o["d_mlp"]
    aW, aB = oa["d_mlp"]
    sW, sB = sp["d_mlp"]
    # the weight gradient is a matrix-core product of activations and
    # adjoints split into bf16 parts: its error is relative to the layer's
    # scale (an adjoint entry can be a cancelling sum of larger terms), so
    # each entry is also allowed 1e-3 of a tenth of the layer's RMS
    for l in range(layers + 1):
        check_elements(dW[l], oW[l], aW[l], f"dW[{l}]", sW[l], floor_frac=0.1)
        check_elements(dB[l], oB[l], aB[l], f"db[{l}]", sB[l], floor_frac=0.1)
    check_elements(dV, o["dV"], oa["dV"], "dV with the weight gradient", sp["dV"])
    lhs = float((Ws[-1].astype(np.float64) * dW[-1]).sum() + (Bs[-1].astype(np.float64) * dB[-1]).sum())
    rhs = float((g * rgb).sum())
    _print("head identity", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-4 * abs(rhs)
    # a repeated run agrees to the order of its FP32 sums (the miss list
    # that deals rays to blocks is built with atomics)
    P.gpu_backward(buf, g)
    dW2, dB2 = P.env.split_grad()
    for a, b in zip(dW + dB, dW2 + dB2):
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(a)


def test_mlp_weight_gradient_128_is_refused():
    """128-wide networks: the weight gradient is refused on the host."""
    dev = device()
    Ws, Bs = synth.env_mlp_weights(seed=5, n_layers=2, width=128)
    env = B.Env.mlp(Ws, Bs, 6, dev, want_grad=True)
    wl = synth.icosphere_scene(res=16)
    m = B.Mesh(torch.from_numpy(wl.V.astype(np.float32)).to(dev), torch.from_numpy(wl.F).to(dev))
    sc = B.Scene(m, torch.tensor([1.5], device=dev), torch.zeros(3, device=dev), env)
    rays = B.Rays(cameras=wl.cameras)
    p = B.Params(max_depth=2)
    buf = B.Buffers(p, rays, m, tape=True)
    with pytest.raises(B.DTError, match="64 only"):
        B.dt_trace_forward(sc, rays, p, buf)
