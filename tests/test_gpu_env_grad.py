"""Parity of the gradient with respect to the equirect environment's texels
(rays leaving the object take a bilinear lookup, Sec. 3.2-3.3) between the
HIP path and the FP64 oracle: dLoss/dtexel within 1e-3, element by element
(against max(|o|, 0.1 rms)) and as a whole-array L2 ratio, and Euler's
identity (the image is linear in the map) on the device."""
import numpy as np
import pytest
import torch

from paper_2603_00413_amd import binding as B
from tests.gpu_helpers import GradRef, check_elements, check_radiance, gradient_pixels, icosphere_pair, torus_pair

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _with_tex_grad(P):
    dev = P.mesh.V.device
    P.env = B.Env(torch.from_numpy(P.tex).to(dev), want_grad=True)
    P.scene = B.Scene(P.mesh, P.ior_t, P.sigma_t, P.env)
    return P


def _check(P, seed):
    buf, rgb, wt, fl = P.gpu_forward(tape=True)
    chk = check_radiance(P.orc, P.o, P.d, rgb, fl, P.sig, label="texel gradient scene")
    gr = GradRef(P.orc, P.o, P.d, chk["ref"]["sig"])
    ok = gradient_pixels(chk, fl, gr.stable)
    g = np.random.default_rng(seed).normal(size=rgb.shape) * ok[:, None]
    P.gpu_backward(buf, g)
    dt = P.env.d_texels.cpu().numpy().astype(np.float64)
    o, oa, sp = gr.grads(g, want_tex=True)
    # texels no lookup touches have gradient 0 on both sides
    et = check_elements(dt, o["d_tex"], oa["d_tex"], "d_tex", sp["d_tex"])
    # Euler: sum d_tex * tex = sum g . C, both from the device
    lhs = float((dt * P.tex.astype(np.float64)).sum())
    rhs = float((g * rgb).sum())
    _print("d_tex rel err", et, "euler", lhs, rhs)
    # d_tex: checked element by element above
    assert abs(lhs - rhs) <= 1e-4 * abs(rhs)


@pytest.mark.parametrize("sigma", [(0.0, 0.0, 0.0), (0.5, 0.2, 0.1)])
def test_texel_gradient_icosphere(sigma):
    _check(_with_tex_grad(icosphere_pair(sigma=sigma)), seed=1)


def test_texel_gradient_terminal_env():
    """Rays stopped at the depth cap take A E(d) with terminal_env."""
    _check(_with_tex_grad(icosphere_pair(sigma=(0.5, 0.2, 0.1), terminal_env=True)), seed=2)


def test_texel_gradient_torus():
    _check(_with_tex_grad(torus_pair(n_views=2, res=64)), seed=3)
