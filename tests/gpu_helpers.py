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


def path_ill_conditioned(orc, o, d, sig, k=8, seed=0, counts=None):
    """True where the oracle's own discrete path (signature) changes under a
    perturbation of the size a float32 evaluation makes: either every ray it
    starts, camera rays and each child, scaled per component by 1 + 2^-20 xi
    (the oracle's jitter instrument: eight float32 ulps, the rounding of a
    stored ray with SPREAD_MARGIN's allowance for the arithmetic between two
    stored rays), or the camera ray turned by 1e-5 rad, in any of k seeded
    runs: a path that FP32 and FP64 may legitimately resolve differently (a
    hit within rounding of a shared edge or a silhouette, a near-critical TIR
    test, two surfaces at nearly the same distance).  counts (a dict) receives
    how many were explained by the jitter and how many only by the turn."""
    o, d = np.asarray(o, np.float64), np.asarray(d, np.float64)
    jit = np.zeros(len(o), bool)
    for j in range(k):
        sc = orc.with_(jitter=SPREAD_MARGIN * PERTURB_U, jitter_seed=7000 + 100 * seed + j)
        jit |= sc.trace(o, d)["sig"] != np.asarray(sig)
    turn = np.zeros(len(o), bool)
    rest = np.flatnonzero(~jit)
    if rest.size:
        rng = np.random.default_rng(seed)
        for _ in range(k):
            t = rng.normal(size=d[rest].shape)
            t -= (t * d[rest]).sum(1, keepdims=True) * d[rest]
            t /= np.linalg.norm(t, axis=1, keepdims=True)
            dp = d[rest] + 1e-5 * t
            dp /= np.linalg.norm(dp, axis=1, keepdims=True)
            turn[rest] |= orc.trace(o[rest], dp)["sig"] != np.asarray(sig)[rest]
    if counts is not None:
        counts["jitter"] = int(jit.sum())
        counts["turn_only"] = int(turn.sum())
    return jit | turn


# pixels with no defined radiance comparison: a shading normal on the wrong
# side (the geometric one is used) or a ray that leaves the object from inside
UNDEFINED = B.FLAG_DEGEN | B.FLAG_LEAK


def check_radiance(orc, o, d, rgb, fl, sig, mlp=False, label="", max_excluded=0.05):
    """Device radiance against the oracle, pixel by pixel.

    * No pixel may carry a stack overflow or a dropped ray (HARD).
    * DEGEN / LEAK pixels have no defined comparison; they must be under
      max_excluded.
    * A pixel whose discrete path (signature) differs from the oracle's must
      be one whose oracle path changes when every ray is jittered by eight
      float32 ulps or the camera ray is turned by 1e-5 rad
      (path_ill_conditioned; every such pixel is checked, the fractions are
      reported).
    * Every same-path pixel, grazing and near-critical ones included, meets
      1e-4, or, where FP32 cannot reach 1e-4, the oracle's first-order bound on
      the rounding error of an FP32 evaluation of that pixel.
    Metric: per pixel-channel |g - o| / max(|o|, 1e-3 mean |o|) for map-lit
    scenes; per pixel ||g - o|| / max(||o||, 0.1 mean ||o||) for MLP-lit ones
    (the network's output is a signed sum, its rounding error absolute).
    Returns dict(ref, same_path, well) with well = same-path pixels whose bound
    is within 1e-4."""
    o, d = np.asarray(o, np.float64), np.asarray(d, np.float64)
    rgb = np.asarray(rgb, np.float64)
    ref = orc.trace(o, d)
    assert not (fl & HARD).any(), f"{label}: stack overflow or dropped rays"
    undef = ((fl | ref["flags"]) & UNDEFINED) != 0
    same = sig == ref["sig"]
    sp = ~undef & same
    bound = np.zeros_like(rgb)
    if sp.any():
        _, bound[sp] = orc.errbound(o[sp], d[sp])
    if mlp:
        n = np.linalg.norm(ref["rgb"], axis=1)
        den = np.maximum(n, 0.1 * max(n.mean(), 1e-30))
        err = np.linalg.norm(rgb - ref["rgb"], axis=1) / den
        brel = np.linalg.norm(bound, axis=1) / den
    else:
        den = np.maximum(np.abs(ref["rgb"]), 1e-3 * max(np.abs(ref["rgb"]).mean(), 1e-30))
        err = (np.abs(rgb - ref["rgb"]) / den).max(1)
        brel = (bound / den).max(1)
    well = sp & (brel <= 1e-4)
    ill = sp & ~well
    over = sp & (err > 1e-4)
    marked = ((fl | ref["flags"]) & (B.FLAG_GRAZING | B.FLAG_TIRB)) != 0
    print(f"{label}: {len(o)} px; undefined {undef.mean():.4f}; same path {sp.sum()} "
          f"(grazing / near-critical {int((sp & marked).sum())}); FP32 bound over 1e-4 on "
          f"{ill.mean():.4f}; max err where bound <= 1e-4: {err[well].max() if well.any() else 0:.2e}; "
          f"over 1e-4: {int(over.sum())} (max ratio to bound "
          f"{(err[over] / brel[over]).max() if over.any() else 0:.3f}); paths differing "
          f"{int((~undef & ~same).sum())}", flush=True)
    assert undef.mean() < max_excluded, f"{label}: {undef.mean():.4f} undefined"
    assert (err[sp] <= np.maximum(1e-4, brel[sp])).all(), \
        f"{label}: {int((err[sp] > np.maximum(1e-4, brel[sp])).sum())} same-path pixels over their bar"
    div = ~undef & ~same
    if div.any():
        cnt = {}
        ok = path_ill_conditioned(orc, o[div], d[div], ref["sig"][div], counts=cnt)
        print(f"{label}: differing paths explained by the 8-ulp jitter {cnt['jitter']}, "
              f"only by the 1e-5 rad turn {cnt['turn_only']}", flush=True)
        assert ok.all(), f"{label}: a path differs where the oracle's own path is well conditioned"
    return {"ref": ref, "same_path": sp, "well": well, "err": err}


def gradient_pixels(chk, fl, stable=None, strict=False):
    """Pixels whose gradient is compared: same discrete path, under the
    oracle's perturbations too (`stable`), and no environment lookup on a
    gradient kink.  Grazing and near-critical hits, and radiance that FP32
    does not resolve to 1e-4, are compared like every other pixel, each
    element held to its own perturbation spread (GradRef); strict leaves them
    out."""
    ref = chk["ref"]
    m = chk["same_path"] & ((ref["flags"] & KINK) == 0)
    if strict:
        m &= chk["well"] & (((fl | ref["flags"]) & (B.FLAG_GRAZING | B.FLAG_TIRB)) == 0)
    if stable is not None:
        m &= stable
    return m


# relative size of the perturbations that stand in for FP32 rounding: two
# units in the last place of a float32
PERTURB_U = 2.0 ** -23
# margin of the per-element gradient allowance over the perturbation spread
# (the intermediate steps round too, each at about the inputs' level)
SPREAD_MARGIN = 8.0


def _spread(a, b):
    if a is None:
        return None
    if isinstance(a, (list, tuple)):
        return type(a)(_spread(x, y) for x, y in zip(a, b))
    if isinstance(a, float):
        return abs(a - b)
    return np.abs(np.asarray(a) - np.asarray(b))


def _max(a, b):
    if a is None:
        return None
    if isinstance(a, (list, tuple)):
        return type(a)(_max(x, y) for x, y in zip(a, b))
    return np.maximum(a, b)


class GradRef:
    """The oracle's gradients for a device backward, with a per-element
    rounding allowance.

    A derivative can be far worse conditioned than the radiance it belongs to:
    a vertex that reaches the loss only through a barycentric weight near zero
    (a hit near the opposite edge), or a texel only through a bilinear weight
    near zero, carries the FP32 rounding error of that weight (absolute, about
    1e-7) as a large relative error.  The allowance is measured on the oracle
    alone.  K = 8 times, the vertices and the material are perturbed at random by
    a relative PERTURB_U (two float32 ulps, the backward error of rounding
    each input once), and the oracle's jitter instrument scales every ray it
    starts (camera rays and each child, as the device stores every ray in
    float32) per component by (1 + PERTURB_U xi); the FP64 gradients are taken
    again, and SPREAD_MARGIN times the spread max_k |g_k - g| of each element
    is added to its relative 1e-3 of the ray-by-ray magnitudes.  The spread is
    that of the summed gradient, where the deviations of different pixels may
    partly cancel in one run; with K = 2 a few elements in 10^5 came out
    below the device's deviation for that reason, and each further run makes
    such a chance underestimate rarer by a large factor.  An absorption grid's
    or a volumetric field's box is perturbed too, each bound by PERTURB_U of
    the box's extent: the device holds the bounds and the per-axis scale
    (n - 1) / (hi - lo) in float32, which moves a sample's grid coordinate by
    up to about n 2^-24, and a node reached only through a trilinear weight
    near zero carries that as a large relative error.  `stable`
    marks the pixels whose discrete path is the same under every perturbation:
    the others have no defined gradient comparison."""

    def __init__(self, orc, o, d, sig, k=8, seed=11):
        self.orc, self.o, self.d = orc, np.asarray(o, np.float64), np.asarray(d, np.float64)
        rng = np.random.default_rng(seed)
        u = PERTURB_U

        def jit(x):
            x = np.asarray(x, np.float64)
            return x * (1.0 + u * rng.uniform(-1.0, 1.0, x.shape))

        self.perturbed = []
        self.stable = np.ones(len(self.o), bool)
        def box(b):
            ext = b.hi - b.lo
            return b.lo + u * rng.uniform(-1.0, 1.0, 3) * ext, b.hi + u * rng.uniform(-1.0, 1.0, 3) * ext

        for j in range(k):
            extra = {}
            if orc.absorb is not None:
                lo, hi = box(orc.absorb)
                extra["absorb"] = oracle.Absorption(orc.absorb.mu, lo, hi, orc.absorb.samples)
            if orc.field is not None:
                lo, hi = box(orc.field)
                extra["field"] = oracle.Field(orc.field.grid, orc.field.planes, lo, hi, orc.field.samples)
            sc = orc.with_(V=jit(orc.V), eta=float(jit(orc.eta)), sigma=jit(orc.sigma), jitter=u,
                           jitter_seed=seed * 1000 + j, **extra)
            self.perturbed.append(sc)
            self.stable &= sc.trace(self.o, self.d)["sig"] == np.asarray(sig)

    def grads(self, gs, **kw):
        """(o, a, s): the oracle's gradients for upstream gs, their ray-by-ray
        magnitudes, and the perturbation spread (same structure)."""
        o = self.orc.trace_grad(self.o, self.d, gs, **kw)
        a = self.orc.trace_grad(self.o, self.d, gs, absolute=True, **kw)
        s = None
        for sc in self.perturbed:
            p = sc.trace_grad(self.o, self.d, gs, **kw)
            sk = {key: _spread(o[key], p[key]) for key in o if key != "rgb"}
            s = sk if s is None else {key: _max(s[key], sk[key]) for key in s}
        return o, a, s


def check_elements(g, o, a, name, spread=None, tol=1e-3, floor_frac=None, allow_zero=False):
    """Element by element: every entry of the device gradient within
    tol * a + SPREAD_MARGIN * spread of the oracle's, where a = the sum over
    camera rays of the magnitudes of each ray's contribution to that entry
    (the oracle's `absolute` gradient: each ray's term is held to tol, and an
    entry that is a sum cancelling to near zero is compared against the terms
    it cancels, not against the small remainder) and spread = the entry's
    perturbation spread (GradRef).  floor_frac: the allowance is at least
    tol * floor_frac * the RMS of the array's nonzero entries (for arrays whose
    arithmetic error is relative to the array's scale rather than to each
    entry).  Also the whole-array L2 distance, within
    tol ||o|| + SPREAD_MARGIN ||spread||.  An oracle gradient that is exactly
    zero is an error (nothing would be compared) unless allow_zero, and then
    the device's must be exactly zero too.  Returns the L2 ratio
    ||g - o|| / ||o||."""
    g, o, a = (np.asarray(x, np.float64).ravel() for x in (g, o, a))
    s = np.zeros_like(o) if spread is None else np.asarray(spread, np.float64).ravel()
    assert (a >= np.abs(o) * (1 - 1e-12)).all()
    assert np.isfinite(g).all(), f"{name}: non-finite device gradient"
    allow = tol * a + SPREAD_MARGIN * s
    if floor_frac is not None:
        nz = o != 0
        allow = np.maximum(allow, tol * floor_frac * np.sqrt(np.mean(o[nz] ** 2)) if nz.any() else 0.0)
    r = np.abs(g - o) / np.maximum(allow, 1e-300)
    on = np.linalg.norm(o)
    if on == 0 and allow_zero:
        assert np.all(g == 0.0) and np.all(a == 0.0), f"{name}: the oracle's gradient is zero, the device's not"
        print(f"{name}: zero on both sides", flush=True)
        return 0.0
    assert on > 0, f"{name}: the oracle's gradient is zero: nothing is compared"
    l2 = np.linalg.norm(g - o) / on
    l2_allow = tol + SPREAD_MARGIN * np.linalg.norm(s) / on
    spread_led = int((SPREAD_MARGIN * s > tol * a).sum())
    print(f"{name}: L2 {l2:.2e} (allowed {l2_allow:.2e}); per element max {r.max():.2e} of its "
          f"allowance, p99.9 {np.quantile(r, 0.999):.2e}; over: {int((r > 1).sum())} of {r.size}; "
          f"allowance set by the spread on {spread_led}", flush=True)
    assert l2 <= l2_allow, f"{name}: L2 ratio {l2} over {l2_allow}"
    assert r.max() <= 1.0, f"{name}: {int((r > 1).sum())} elements over their allowance"
    return l2


def check_material(de, ds, o, a, s, label, sigma=True):
    """dIoR (and dsigma) against the oracle to check_elements' bar, with the
    oracle's gradients o, ray-by-ray magnitudes a and spreads s (GradRef).
    Returns their relative errors, for the log."""
    check_elements(np.array([de]), np.array([o["d_eta"]]), np.array([a["d_eta"]]), f"{label} d_eta",
                   np.array([s["d_eta"]]))
    if sigma:
        # zero where no interior segment reaches the image (depth 1 without
        # terminal_env: the rays inside end at the cap)
        check_elements(ds, o["d_sigma"], a["d_sigma"], f"{label} d_sigma", s["d_sigma"], allow_zero=True)
    return (abs(de - o["d_eta"]) / abs(o["d_eta"]),
            np.abs(ds - o["d_sigma"]) / np.maximum(np.abs(o["d_sigma"]), 1e-300))
