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
from tests.gpu_helpers import BAD, HARD, KINK, device, l2_upstream, path_ill_conditioned, rgb_rel_err

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
    ref = P.orc.trace(P.o, P.d)
    ok = ((fl | ref["flags"]) & (BAD | HARD)) == 0
    same = P.sig == ref["sig"]
    err = rgb_rel_err(rgb, ref["rgb"])
    _print("MLP trace: excluded", 1 - ok.mean(), "median", np.median(err[ok]), "max", err[ok].max(),
           "paths differing", (~same[ok]).sum())
    assert 1 - ok.mean() < 0.05
    assert err[ok & same].max() <= 1e-4
    div = ok & ~same
    assert div.mean() <= 2e-3
    if div.any():
        assert path_ill_conditioned(P.orc, P.o[div], P.d[div], ref["sig"][div]).all()
    okg = ok & same & ((ref["flags"] & KINK) == 0)
    _print("MLP trace: gradient pixels excluded near ReLU kinks", 1 - okg.mean() / ok.mean())
    tgt = P.orc.with_(eta=1.52, sigma=(0.4, 0.25, 0.15)).trace(P.o, P.d)["rgb"]
    g = l2_upstream(ref["rgb"], tgt, okg)
    dV, de, ds = P.gpu_backward(buf, g)
    o = P.orc.trace_grad(P.o, P.d, g)
    ev = np.linalg.norm(dV - o["dV"]) / np.linalg.norm(o["dV"])
    ee = abs(de - o["d_eta"]) / abs(o["d_eta"])
    es = np.abs(ds - o["d_sigma"]) / np.abs(o["d_sigma"])
    _print("MLP trace grads: dV", ev, "deta", ee, "dsigma", es)
    assert ev <= 1e-3 and ee <= 1e-3 and (es <= 1e-3).all()
