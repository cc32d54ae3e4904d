"""Helpers shared by the GPU parity tests: build the same seeded scene for the
HIP path (float32 device tensors) and for the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth

# pixels whose trees contain a node in one of these states are excluded from
# the tolerance checks (degenerate normal, leak, grazing, TIR boundary)
BAD = B.FLAG_DEGEN | B.FLAG_LEAK | B.FLAG_GRAZING | B.FLAG_TIRB
HARD = B.FLAG_OVERFLOW | B.FLAG_STACK
# oracle-only flag: an environment lookup within 1e-5 rad of a direction where
# the environment's gradient jumps (texel-centre line, ReLU kink); FP32 and
# FP64 paths may straddle it, so gradients (not values) are compared off it
KINK = oracle.FLAG_KINK
# relative L2 bound between two device runs of the same vertex gradient: the
# per-vertex sums are FP32 atomic additions in run-dependent order, so with
# cancellation among the terms they agree to a few 1e-6, not bit for bit
DV_ORDER_TOL = 1e-5


def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


class Pair:
    """The same scene on the device and in the oracle."""

    def __init__(self, V, F, ior, sigma, tex, cams, depth, terminal_env=False,
                 capacity=0, stride=1):
        dev = device()
        self.V64, self.F = np.asarray(V, np.float64), np.asarray(F, np.int32)
        # both sides see exactly the float32-rounded geometry and texels
        self.V32 = self.V64.astype(np.float32)
        self.tex = np.asarray(tex, np.float32)
        self.cams = cams
        self.depth = depth
        self.sigma = np.broadcast_to(np.asarray(sigma, np.float64), (3,)).astype(np.float32)
        self.ior = np.float32(ior)
        self.mesh = B.Mesh(torch.from_numpy(self.V32).to(dev), torch.from_numpy(self.F).to(dev))
        self.env = B.Env(torch.from_numpy(self.tex).to(dev))
        self.ior_t = torch.tensor([self.ior], dtype=torch.float32, device=dev)
        self.sigma_t = torch.from_numpy(self.sigma.copy()).to(dev)
        self.scene = B.Scene(self.mesh, self.ior_t, self.sigma_t, self.env)
        self.rays = B.Rays(cameras=cams)
        self.params = B.Params(max_depth=depth, terminal_env=terminal_env,
                               checkpoint_stride=stride, queue_capacity=capacity)
        self.orc = oracle.Scene(self.V32.astype(np.float64), self.F, float(self.ior),
                                self.sigma.astype(np.float64), oracle.Env(tex=self.tex), depth,
                                terminal_env=terminal_env)
        o, d = [], []
        for c in cams:
            oo, dd = oracle.camera_rays(c)
            o.append(oo)
            d.append(dd)
        self.o, self.d = np.concatenate(o), np.concatenate(d)

    def gpu_forward(self, tape=True, params=None):
        """Device render; also leaves the per-pixel path signatures in self.sig."""
        p = params or self.params
        buf = B.Buffers(p, self.rays, self.mesh, tape=tape)
        sig = torch.empty(self.rays.n_pixels, dtype=torch.int64, device=self.mesh.V.device)
        rgb, wt, fl = B.dt_trace_forward(self.scene, self.rays, p, buf, path_sig=sig)
        torch.cuda.synchronize()
        self.sig = sig.cpu().numpy().view(np.uint64)
        return buf, rgb.cpu().numpy().astype(np.float64), wt.cpu().numpy().astype(np.float64), \
            fl.cpu().numpy()

    def gpu_backward(self, buf, grad, params=None):
        p = params or self.params
        g = torch.from_numpy(np.asarray(grad, np.float32)).to(self.mesh.V.device)
        dV, de, ds = B.dt_trace_backward(self.scene, self.rays, p, buf, g)
        torch.cuda.synchronize()
        return dV.cpu().numpy().astype(np.float64), float(de.cpu()[0]), ds.cpu().numpy().astype(np.float64)


def rel_err(g, o):
    """Per pixel-channel |g - o| / max(|o|, 1e-3 * mean(o))."""
    floor = 1e-3 * max(np.abs(o).mean(), 1e-30)
    return np.abs(g - o) / np.maximum(np.abs(o), floor)


def rgb_rel_err(g, o, floor_frac=0.1):
    """Per pixel ||g - o|| / max(||o||, floor_frac * mean ||o||) over the RGB
    triple.  Used where the environment is the MLP: its output is a signed sum
    of terms about as large as the mean radiance, so its FP32 rounding error
    (a few 1e-6 of the mean) is absolute, not relative: a single channel, or a
    whole pixel, that the linear head brings near zero by cancellation carries
    it as relative noise.  Measured against a tenth of the mean, that noise
    stays an order of magnitude inside 1e-4."""
    n = np.linalg.norm(o, axis=1)
    floor = floor_frac * max(n.mean(), 1e-30)
    return np.linalg.norm(g - o, axis=1) / np.maximum(n, floor)


def l2_upstream(ref_rgb, target_rgb, mask):
    """dLoss/dC of the L2 image loss sum_i mask_i ||C_i - T_i||^2 / n at the
    oracle's own render (so both sides take the same upstream gradient, and
    none of it comes from the device)."""
    return 2.0 * (ref_rgb - target_rgb) / max(int(mask.sum()), 1) * mask[:, None]


def icosphere_pair(sigma=(0.0, 0.0, 0.0), res=64, **kw):
    wl = synth.icosphere_scene(sigma=sigma, res=res)
    return Pair(wl.V, wl.F, wl.ior, wl.sigma, wl.env, wl.cameras, wl.max_depth, **kw)


def torus_pair(n_views=2, res=96, nu=320, nv=160, **kw):
    V, F = synth.displaced_torus(seed=2, nu=nu, nv=nv)
    tex = synth.env_equirect(512, 256, seed=2)
    eyes = synth.views_on_sphere(n_views, 3.0, seed=2)
    cams = [synth.look_at_camera(e, res, res) for e in eyes]
    return Pair(V, F, 1.45, 0.3, tex, cams, 6, **kw)


def path_ill_conditioned(orc, o, d, sig, eps=1e-5, k=8, seed=0):
    """True where the oracle's own discrete path (signature) changes when the
    camera ray is turned by eps radians in any of k random directions: a path
    that FP32 and FP64 may legitimately resolve differently (a hit within
    rounding of a shared edge or a silhouette, a near-critical TIR test)."""
    o, d = np.asarray(o, np.float64), np.asarray(d, np.float64)
    rng = np.random.default_rng(seed)
    out = np.zeros(len(o), bool)
    for _ in range(k):
        t = rng.normal(size=d.shape)
        t -= (t * d).sum(1, keepdims=True) * d
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        dp = d + eps * t
        dp /= np.linalg.norm(dp, axis=1, keepdims=True)
        out |= orc.trace(o, dp)["sig"] != sig
    return out


def radiance_sensitivity(orc, o, d, rgb, eps=1e-6, k=8, seed=1, floor=None):
    """Largest relative change of the oracle's radiance when the camera ray is
    turned by eps radians (k random directions), per pixel, in the metric of
    rgb_rel_err.  eps = 1e-6 rad is about 16 FP32 ulps of a unit direction, the
    size of the error an FP32 path has gathered after a few bounces; where the
    radiance moves more than 1e-4 under such a turn (a high-frequency
    environment seen through magnifying refractions), FP32 cannot resolve it
    to 1e-4."""
    o, d = np.asarray(o, np.float64), np.asarray(d, np.float64)
    rng = np.random.default_rng(seed)
    n = np.linalg.norm(rgb, axis=1)
    fl = floor if floor is not None else 0.1 * max(n.mean(), 1e-30)
    out = np.zeros(len(o))
    for _ in range(k):
        t = rng.normal(size=d.shape)
        t -= (t * d).sum(1, keepdims=True) * d
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        dp = d + eps * t
        dp /= np.linalg.norm(dp, axis=1, keepdims=True)
        c = orc.trace(o, dp)["rgb"]
        out = np.maximum(out, np.linalg.norm(c - rgb, axis=1) / np.maximum(n, fl))
    return out
