"""The training-step and stress configurations at their full sizes, traced in
full on the device, checked against the oracle on sampled pixels (forward
radiance and the gradient of a loss restricted to those pixels)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from tests.gpu_helpers import (DV_ORDER_TOL, HARD, KINK, GradRef, check_elements, check_material, check_radiance, device,
                               gradient_pixels, l2_upstream)

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _setup(wl, sigma, ior):
    dev = device()
    V32 = wl.V.astype(np.float32)
    mesh = B.Mesh(torch.from_numpy(V32).to(dev), torch.from_numpy(wl.F).to(dev))
    Ws, Bs, nfq = wl.mlp
    env = B.Env.mlp(Ws, Bs, nfq, dev)
    scene = B.Scene(mesh, torch.tensor([ior], dtype=torch.float32, device=dev),
                    torch.tensor(sigma, dtype=torch.float32, device=dev), env)
    rays = B.Rays(cameras=wl.cameras)
    oenv = oracle.Env(mlp=([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], nfq))
    o, d = [], []
    for c in wl.cameras:
        oo, dd = oracle.camera_rays(c)
        o.append(oo)
        d.append(dd)
    return mesh, scene, rays, oenv, V32, np.concatenate(o), np.concatenate(d)


def _check(wl, stride, n_sample, ior=1.45, sigma=(0.3, 0.3, 0.3), target=(1.5, (0.4, 0.25, 0.1)),
           max_excluded=0.05, strict=False):
    mesh, scene, rays, oenv, V32, O, D = _setup(wl, sigma, ior)
    cap = int(1.3 * rays.n_rays)
    sig_t = torch.empty(rays.n_pixels, dtype=torch.int64, device=mesh.V.device)
    while True:
        p = B.Params(max_depth=wl.max_depth, checkpoint_stride=stride, queue_capacity=cap)
        buf = B.Buffers(p, rays, mesh, tape=True)
        rgb_t, _, fl_t = B.dt_trace_forward(scene, rays, p, buf, path_sig=sig_t)
        st = buf.stats.cpu().numpy()
        if st[B.STAT_DROPPED] == 0:
            break
        cap *= 2
    counts = st[:wl.max_depth + 1]
    _print(wl.name, "rays per generation", counts.tolist(), "capacity", cap,
           "queue use", np.round(counts[1:] / cap, 3).tolist())
    rgb, fl = rgb_t.cpu().numpy().astype(np.float64), fl_t.cpu().numpy()
    sig = sig_t.cpu().numpy().view(np.uint64)
    assert not (fl & HARD).any()
    orc = oracle.Scene(V32.astype(np.float64), wl.F, float(np.float32(ior)),
                       np.asarray(sigma, np.float32).astype(np.float64), oenv, wl.max_depth)
    # a quarter of the sample at random, the rest among pixels whose camera
    # ray the oracle finds hitting the object (the gradient lives there)
    rng = np.random.default_rng(3)
    cand = rng.choice(len(O), 4 * n_sample, replace=False)
    half = n_sample // 4
    rest = cand[half:]
    on_obj = rest[orc.trace(O[rest], D[rest])["nseg"] > 1][:n_sample - half]
    pix = np.sort(np.concatenate([cand[:half], on_obj]))
    # same-path pixels meet 1e-4, or the oracle's FP32 rounding bound where
    # that is larger; a path may part only where the oracle's own path is
    # ill-conditioned
    chk = check_radiance(orc, O[pix], D[pix], rgb[pix], fl[pix], sig[pix], mlp=True,
                         label=f"{wl.name}, {n_sample} sampled pixels", max_excluded=max_excluded)
    ref = chk["ref"]
    # gradient of an L2 loss on the sampled pixels against an oracle-rendered
    # target, on same-path pixels (under the oracle's perturbations too) off
    # the environment's gradient kinks
    tgt = orc.with_(eta=target[0], sigma=target[1]).trace(O[pix], D[pix])["rgb"]
    gr = GradRef(orc, O[pix], D[pix], ref["sig"])
    okg = gradient_pixels(chk, fl[pix], gr.stable, strict=strict)
    hits = okg & (ref["nseg"] > 1)
    kink = (ref["flags"] & KINK) != 0
    _print(wl.name, "sampled pixels hitting the object", int((ref["nseg"] > 1).sum()), "of", len(pix),
           "; same path", int(chk["same_path"].sum()), "; path stable under the perturbations",
           int(gr.stable.sum()), "; on a kink", int(kink.sum()), "; gradient pixels", int(okg.sum()),
           "of which hit the object", int(hits.sum()))
    # the MLP-lit scenes put many lookups within 1e-5 rad of a ReLU kink
    # (a 4 x 128 network has 512 of them, a path up to ~20 lookups), and
    # those pixels' gradients are not compared
    assert hits.sum() >= 50
    gs = l2_upstream(ref["rgb"], tgt, okg)
    g = np.zeros_like(rgb)
    g[pix] = gs
    dV, de, ds = B.dt_trace_backward(scene, rays, p, buf, torch.from_numpy(g.astype(np.float32)).to(mesh.V.device))
    dV, de, ds = dV.cpu().numpy(), float(de.cpu()[0]), ds.cpu().numpy()
    o, oa, sp = gr.grads(gs)
    ev = check_elements(dV, o["dV"], oa["dV"], f"{wl.name} dV", sp["dV"])
    ee, es = check_material(de, ds, o, oa, sp, wl.name)
    _print(wl.name, "grads: dV", ev, "deta", ee, "dsigma", es)
    return buf, p, scene, rays, g, (dV, de, ds)


def test_training_step_shape_sdf_union_300k():
    wl = synth.sdf_union_scene()
    assert 250_000 < len(wl.F) < 350_000
    assert wl.ior == 1.5 and tuple(wl.sigma) == (0.5, 0.2, 0.1)
    # rendered at eta 1.45, sigma 0.3 against targets the oracle renders at
    # eta* 1.5, sigma* (0.4, 0.25, 0.1), so every gradient is nonzero
    buf, p, scene, rays, g, (dV, de, ds) = _check(wl, 1, 2000, ior=1.45, sigma=(0.3, 0.3, 0.3),
                                                  target=(1.5, (0.4, 0.25, 0.1)), strict=False)
    # the recompute adjoint (checkpoint every 3 generations) gives the same gradients
    p3 = B.Params(max_depth=wl.max_depth, checkpoint_stride=3, queue_capacity=p.queue_capacity)
    b3 = B.Buffers(p3, rays, scene.mesh, tape=True)
    B.dt_trace_forward(scene, rays, p3, b3, want_aux=False)
    gt = torch.from_numpy(g.astype(np.float32)).to(scene.mesh.V.device)
    dV3, de3, ds3 = B.dt_trace_backward(scene, rays, p3, b3, gt)
    assert np.linalg.norm(dV3.cpu().numpy() - dV) <= DV_ORDER_TOL * np.linalg.norm(dV)
    assert abs(float(de3.cpu()[0]) - de) <= 1e-6 * abs(de)
    assert b3.tape_bytes < 0.6 * buf.tape_bytes


def test_stress_thin_shell_2m():
    wl = synth.thin_shell_scene()
    assert len(wl.F) > 1_500_000
    # thin walls make near-critical hits frequent (held to the FP32 rounding
    # bound, like every pixel), and over 8 bounces some FP32 paths part from
    # the FP64 ones at shared edges (each one checked to be ill-conditioned
    # in the oracle; their gradients belong to another path and are not
    # compared)
    buf, *_ = _check(wl, 2, 1500, ior=1.5, target=(1.55, (0.2, 0.3, 0.4)))
    st = buf.stats.cpu().numpy()
    _print("thin shell: BVH height", st[B.STAT_BVH_DEPTH], "total rays", st[B.STAT_TOTAL])
