"""A few optimisation steps of the ray-tracing stage through the tracer's
gradients recover a perturbed IoR (Sec. 3.3 "Optimization")."""
import numpy as np
import pytest
import torch

from paper_2603_00413_amd import autograd as A
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from paper_2603_00413_amd import train as T

pytestmark = pytest.mark.gpu


def test_ior_recovery_with_adam():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    dev = torch.device("cuda:0")
    wl = synth.icosphere_scene(sigma=(0.5, 0.2, 0.1), res=64)
    V = torch.from_numpy(wl.V.astype(np.float32)).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    env = B.Env(torch.from_numpy(wl.env).to(dev))
    sigma = torch.tensor(wl.sigma, dtype=torch.float32, device=dev)
    tr = A.Tracer(F, env, wl.cameras, max_depth=wl.max_depth)
    with torch.no_grad():
        gt = A.render(V, torch.tensor([1.45], device=dev), sigma, tr).clone()
    ior = torch.tensor([1.38], device=dev, requires_grad=True)
    trainer = T.Trainer(tr, V, ior, sigma=sigma, lr=0.005, l_color=1.0, l_tone=0.1)
    first = trainer.step(gt)
    for _ in range(60):
        last = trainer.step(gt)
    print("ior", float(ior.detach()), "colour loss", first["color"], "->", last["color"],
          "tone loss", first["tone"], "->", last["tone"], flush=True)
    # the IoR is recovered ...
    assert abs(float(ior.detach()) - 1.45) < 0.01
    # ... and the colour term, which has no constant part (L_tone carries the
    # constant -var(c), so the total can go negative), falls by 10x
    assert last["color"] < 0.1 * first["color"]


def test_vertex_steps_with_adam_uniform_reduce_the_loss():
    """The vertices of a radially perturbed sphere, optimised through the
    tracer's vertex gradient with AdamUniform on the Laplacian
    reparameterisation, move toward the target: the image loss falls."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    dev = torch.device("cuda:0")
    wl = synth.icosphere_scene(sigma=(0.5, 0.2, 0.1), res=64)
    V0 = torch.from_numpy(wl.V.astype(np.float32)).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    env = B.Env(torch.from_numpy(wl.env).to(dev))
    sigma = torch.tensor(wl.sigma, dtype=torch.float32, device=dev)
    ior = torch.tensor([wl.ior], dtype=torch.float32, device=dev)
    tr = A.Tracer(F, env, wl.cameras, max_depth=wl.max_depth)
    with torch.no_grad():
        gt = A.render(V0, ior, sigma, tr).clone()
    V = (V0 * 0.97).clone().requires_grad_(True)
    trainer = T.Trainer(tr, V, ior, sigma=sigma, large_steps=4.0, lr_mesh=4e-3)
    first = trainer.step(gt)["color"]
    errs = [float((V0 * 0.97 - V0).norm())]
    for _ in range(40):
        last = trainer.step(gt)["color"]
        # trainer.V is the mesh after the step's update
        errs.append(float((trainer.V.detach() - V0).norm()))
    print("colour loss", first, "->", last, "vertex error", errs[0], "->", errs[-1],
          "min", min(errs), flush=True)
    assert last < 0.5 * first
    assert errs[-1] < 0.8 * errs[0]
