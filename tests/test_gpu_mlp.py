"""Parity of the bf16-MFMA environment MLP with the oracle's emulation.

Bars: the device rounds the encoded input and each hidden activation to bf16
after FP32 accumulation, the oracle after FP64 accumulation, so an activation
can land on the other side of a bf16 rounding boundary ("flip"), which moves
the output by about 2^-8 of one activation's contribution.  So: rays without a
flip agree to 1e-4 relative (>= 97% of rays), every ray agrees to 1e-2 of the
mean output magnitude, and a hand-computed net is reproduced exactly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from tests.gpu_helpers import BAD, HARD, KINK, device, rel_err

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _dirs(n, seed):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


def test_hand_computed_tiny_net_exact():
    """Same net as the oracle pin: E = (x + 0.5, 2y, 0.5x + 0.25y - 1) with
    x = bf16(0.6) = 0.6015625, y = bf16(0.8) = 0.80078125 (d = (0.6, 0.8, 0))."""
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
    x, y = 0.6015625, 0.80078125
    expect = np.array([x + 0.5, 2 * y, 0.5 * x + 0.25 * y - 1.0], np.float32)
    assert np.abs(E - expect).max() <= 2e-7


@pytest.mark.parametrize("width,layers", [(64, 3), (128, 4)])
def test_mlp_query_vs_oracle(width, layers):
    dev = device()
    Ws, Bs = synth.env_mlp_weights(seed=3, n_layers=layers, width=width)
    env = B.Env.mlp(Ws, Bs, 6, dev)
    oenv = oracle.Env(mlp=([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6))
    d = _dirs(20000, width + layers)
    E = B.dt_env_query(env, torch.from_numpy(d).to(dev)).cpu().numpy().astype(np.float64)
    Eo = oenv.eval(d.astype(np.float64))
    err = rel_err(E, Eo).max(1)
    aerr = np.abs(E - Eo).max(1) / np.abs(Eo).mean()
    _print(width, layers, "flip rate (> 1e-4)", (err > 1e-4).mean(), "max abs / mean", aerr.max())
    assert (err <= 1e-4).mean() >= 0.97
    # a flip moves the output by ~2^-8 of one activation's share; wider and
    # deeper nets carry more of them
    assert aerr.max() <= (1e-2 if width == 64 else 2e-2)
    # input gradient (bf16 rounding taken as identity on both sides)
    g = np.random.default_rng(1).normal(size=d.shape).astype(np.float32)
    gd = B.dt_env_query_backward(env, torch.from_numpy(d).to(dev),
                                 torch.from_numpy(g).to(dev)).cpu().numpy().astype(np.float64)
    gdo = oenv.eval_grad(d.astype(np.float64), g.astype(np.float64))
    num = np.linalg.norm(gd - gdo, axis=1)
    den = np.linalg.norm(gdo, axis=1) + 1e-3 * np.linalg.norm(gdo, axis=1).mean()
    r = num / den
    _print(width, layers, "grad frac > 1e-3", (r > 1e-3).mean(), "max", r.max())
    assert (r <= 1e-3).mean() >= 0.98
    assert np.median(r) < 1e-4


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
    ref = P.orc.trace(P.o, P.d)
    ok = ((fl | ref["flags"]) & (BAD | HARD)) == 0
    err = rel_err(rgb, ref["rgb"]).max(1)
    aerr = np.abs(rgb - ref["rgb"]).max(1) / np.abs(ref["rgb"]).mean()
    _print("MLP trace: frac > 1e-4", (err[ok] > 1e-4).mean(), "max rel", err[ok].max(),
           "max abs / mean", aerr[ok].max())
    # a pixel averages many leaves, each of which may carry a flip
    assert np.median(err[ok]) <= 1e-5 and aerr[ok].max() <= 1e-2
    okg = ok & ((ref["flags"] & KINK) == 0)
    _print("MLP trace: gradient pixels excluded near ReLU kinks", 1 - okg.mean() / ok.mean())
    g = np.random.default_rng(0).normal(size=rgb.shape) * okg[:, None]
    dV, de, ds = P.gpu_backward(buf, g)
    o = P.orc.trace_grad(P.o, P.d, g)
    ev = np.linalg.norm(dV - o["dV"]) / np.linalg.norm(o["dV"])
    ee = abs(de - o["d_eta"]) / abs(o["d_eta"])
    es = np.abs(ds - o["d_sigma"]) / np.abs(o["d_sigma"])
    _print("MLP trace grads: dV", ev, "deta", ee, "dsigma", es)
    assert ev <= 1e-3 and ee <= 1e-3 and (es <= 1e-3).all()
