"""Parity of the silhouette (mask) term between the HIP path and the FP64
oracle: the centre-sample mask, and the outline gradient of a loss on it
(same quadrature on both sides), on a convex mesh and on a self-occluding
one, with several cameras in one call."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from tests.gpu_helpers import device

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _f32_camera(eye, res):
    """A camera whose eye, target and up are exact float32 values, so both
    sides take their facing decisions from the same numbers."""
    c = synth.look_at_camera(np.asarray(eye, np.float32).astype(np.float64), res, res)
    c.eye = tuple(np.float32(c.eye).astype(np.float64).tolist())
    return c


def _meshes(which):
    if which == "icosphere":
        V, F = synth.icosphere(3)
        return V * 0.8, F
    return synth.displaced_torus(seed=5, nu=120, nv=60)


@pytest.mark.parametrize("which", ["icosphere", "torus"])
def test_mask_and_outline_gradient(which):
    dev = device()
    V, F = _meshes(which)
    V32 = V.astype(np.float32)
    mesh = B.Mesh(torch.from_numpy(V32).to(dev), torch.from_numpy(F).to(dev))
    cams = [_f32_camera(e, 64) for e in synth.views_on_sphere(3, 3.0, seed=31)]
    rays = B.Rays(cameras=cams)
    mask = B.dt_mask_forward(mesh, rays).cpu().numpy()
    env = oracle.Env(tex=synth.env_constant(8, 4))
    orc = oracle.Scene(V32.astype(np.float64), F, 1.5, 0.0, env, 1)
    g = np.random.default_rng(3).normal(size=mask.size).astype(np.float32)
    mg = B.MaskGrad(mesh)
    dV = mg(mesh, rays, torch.from_numpy(g).to(dev), rho=2.0).cpu().numpy().astype(np.float64)
    counts = mg.counts.cpu().numpy()
    dVo = np.zeros_like(V32, dtype=np.float64)
    n_in = n_vis = 0
    off = 0
    for c in cams:
        n = c.width * c.height
        mo = orc.mask(c)
        # centre samples: the same hit or miss but where the oracle's own first
        # hit changes when the rays are jittered by eight float32 ulps (a ray
        # grazing the outline)
        diff = np.flatnonzero(mask[off:off + n] != mo)
        if diff.size:
            o, d = oracle.camera_rays(c)
            from tests.gpu_helpers import path_ill_conditioned
            ref = orc.trace(o[diff], d[diff])
            assert path_ill_conditioned(orc, o[diff], d[diff], ref["sig"]).all()
        _print(which, "mask pixels differing", diff.size, "of", n)
        d_c, (a, b) = orc.mask_grad(c, g[off:off + n].astype(np.float64), rho=2.0)
        dVo += d_c
        n_in += a
        n_vis += b
        off += n
    _print(which, "outline points: device", counts.tolist(), "oracle", (n_in, n_vis))
    assert counts[2] == 0
    assert counts[0] == n_in and counts[1] == n_vis
    if which == "icosphere":
        assert n_vis == n_in          # convex: the whole silhouette is outline
    else:
        assert n_vis < n_in           # a torus hides part of its silhouette
    scale = np.abs(dVo).max()
    err = np.abs(dV - dVo).max() / scale
    l2 = np.linalg.norm(dV - dVo) / np.linalg.norm(dVo)
    _print(which, "outline gradient: max abs err / max", err, "L2", l2)
    assert l2 <= 1e-4 and err <= 1e-4
