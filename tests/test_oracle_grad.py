"""Pins of the oracle's reverse-mode gradients.

The reference for every gradient is a central finite difference of the
oracle's own FP64 forward pass (an independent route: no tape involved),
restricted to pixels whose discrete path (triangle ids, TIR branches,
hit/miss, env texel cell) is the same at +h, 0 and -h, and away from grazing
or TIR-boundary nodes.  dsigma and deta are also checked against closed forms.
"""
import math

import numpy as np
import pytest

from paper_2603_00413_amd import synth
from tests.oracle_helpers import fresnel_angle_form, link_tree, slab_ray

BAD = 4 | 8 | 1 | 2   # grazing, TIR boundary, degenerate normal, leak


def _scene(oracle_lib, which, sigma=(0.5, 0.2, 0.1), eta=1.5, depth=4, res=32):
    if which == "icosphere":
        V, F = synth.icosphere(3)
        tex = synth.env_equirect(64, 32, seed=1)
        cam = synth.look_at_camera((0.0, 0.0, 3.0), res, res)
    elif which == "torus":
        V, F = synth.displaced_torus(seed=2, nu=96, nv=48)
        tex = synth.env_equirect(128, 64, seed=2)
        cam = synth.look_at_camera(synth.views_on_sphere(1, 3.0, seed=2)[0], res, res)
    else:
        V, F = synth.sdf_union_mesh(seed=3, res=36)
        tex = synth.env_equirect(128, 64, seed=3)
        cam = synth.look_at_camera((1.2, 1.9, 2.0), res, res)
    env = oracle_lib.Env(tex=tex)
    sc = oracle_lib.Scene(V, F, eta, sigma, env, depth)
    o, d = oracle_lib.camera_rays(cam)
    return sc, o, d


def _fd_mask(sc_p, sc_m, sc0, o, d):
    rp, rm, r0 = sc_p.trace(o, d), sc_m.trace(o, d), sc0.trace(o, d)
    ok = (rp["hash"] == rm["hash"]) & (rp["hash"] == r0["hash"])
    ok &= ((r0["flags"] | rp["flags"] | rm["flags"]) & BAD) == 0
    return ok, rp["rgb"], rm["rgb"]


@pytest.mark.parametrize("which,depth", [("icosphere", 4), ("torus", 6), ("sdf", 5)])
def test_vertex_gradient_directional_fd(oracle_lib, which, depth):
    sc, o, d = _scene(oracle_lib, which, depth=depth)
    rng = np.random.default_rng(11)
    g = rng.normal(size=o.shape)
    # Richardson-extrapolated central differences at h and h/2 cancel the
    # O(h^2) term, which is visible on strongly curved paths (silhouettes,
    # near-critical refraction on coarse meshes)
    h = 2e-7
    for k in range(6 if which != "icosphere" else 16):
        delta = rng.normal(size=sc.V.shape)
        delta /= np.abs(delta).max()
        ok1, cp1, cm1 = _fd_mask(sc.with_(V=sc.V + h * delta), sc.with_(V=sc.V - h * delta), sc, o, d)
        ok2, cp2, cm2 = _fd_mask(sc.with_(V=sc.V + 0.5 * h * delta),
                                 sc.with_(V=sc.V - 0.5 * h * delta), sc, o, d)
        ok = ok1 & ok2
        # per-pixel validity: the two step sizes agree, so the Taylor
        # expansion holds there (drops pixels next to an unflagged kink)
        p1 = ((cp1 - cm1) * g).sum(1) / (2 * h)
        p2 = ((cp2 - cm2) * g).sum(1) / h
        ok &= np.abs(p1 - p2) <= 1e-4 * (np.abs(p2) + 1.0)
        assert ok.mean() > 0.8
        gm = g * ok[:, None]
        fd = float(((4 * p2 - p1) / 3)[ok].sum())
        ad = sc.trace_grad(o, d, gm)
        an = float((ad["dV"] * delta).sum())
        assert abs(fd - an) <= 2e-6 * max(abs(an), 1.0) + 1e-8 * np.abs(ad["dV"]).sum(), (k, fd, an)


def test_vertex_gradient_full_fd_small(oracle_lib):
    """Every coordinate of a handful of vertices under the image, one by one."""
    sc, o, d = _scene(oracle_lib, "icosphere", res=16)
    rng = np.random.default_rng(5)
    g = rng.normal(size=o.shape)
    r0 = sc.trace(o, d)
    ok0 = (r0["flags"] & BAD) == 0
    ad = sc.trace_grad(o, d, g * ok0[:, None])
    # vertices facing the camera (z > 0.3) have nonzero gradients
    cand = np.nonzero(sc.V[:, 2] > 0.3)[0]
    picks = rng.choice(cand, 12, replace=False)
    h = 1e-6
    for v in picks:
        for c in range(3):
            delta = np.zeros_like(sc.V)
            delta[v, c] = 1.0
            ok, cp, cm = _fd_mask(sc.with_(V=sc.V + h * delta), sc.with_(V=sc.V - h * delta), sc, o, d)
            ok &= ok0
            if not np.array_equal(ok, ok0):
                continue   # a path changed: skip this coordinate
            fd = float(((cp - cm) * g * ok[:, None]).sum() / (2 * h))
            an = ad["dV"][v, c]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (v, c, fd, an)


def _richardson(make, sc, o, d, g, h):
    """Per-pixel Richardson FD of g . C along a 1-parameter family
    make(step) -> Scene; returns (mask, per-pixel derivative)."""
    ok1, cp1, cm1 = _fd_mask(make(h), make(-h), sc, o, d)
    ok2, cp2, cm2 = _fd_mask(make(0.5 * h), make(-0.5 * h), sc, o, d)
    p1 = ((cp1 - cm1) * g).sum(1) / (2 * h)
    p2 = ((cp2 - cm2) * g).sum(1) / h
    ok = ok1 & ok2 & (np.abs(p1 - p2) <= 1e-4 * (np.abs(p2) + 1.0))
    return ok, (4 * p2 - p1) / 3


@pytest.mark.parametrize("which,depth", [("icosphere", 4), ("torus", 6)])
def test_eta_sigma_gradient_fd(oracle_lib, which, depth):
    sc, o, d = _scene(oracle_lib, which, depth=depth)
    rng = np.random.default_rng(2)
    g = rng.normal(size=o.shape)
    h = 2e-6
    fams = [lambda s: sc.with_(eta=sc.eta + s)]
    for c in range(3):
        fams.append(lambda s, c=c: sc.with_(sigma=sc.sigma + s * np.eye(3)[c]))
    res = [_richardson(f, sc, o, d, g, h) for f in fams]
    mask = np.logical_and.reduce([r[0] for r in res])
    assert mask.mean() > 0.8
    ad = sc.trace_grad(o, d, g * mask[:, None])
    an = [ad["d_eta"]] + list(ad["d_sigma"])
    for (ok, pix), a in zip(res, an):
        fd = float(pix[mask].sum())
        assert abs(fd - a) <= 1e-6 * abs(a) + 1e-7, (fd, a)


def test_dsigma_closed_form_from_paths(oracle_lib):
    """dC_c/dsigma_c = -sum over leaves of W_c E_c l, l = interior length along
    the leaf's path (Beer-Lambert: the weight carries exp(-sigma l))."""
    sc, o, d = _scene(oracle_lib, "torus", depth=6, res=12)
    for i in range(0, len(o), 7):
        recs = link_tree(sc.tree(o[i], d[i]))
        expect = np.zeros(3)
        for r in recs:
            if r["kind"] != 0:
                continue
            ell, p = 0.0, r["parent"]
            while p >= 0:
                if recs[p]["entering"] == 0:
                    ell += recs[p]["t"]
                p = recs[p]["parent"]
            W = np.array([r["W0"], r["W1"], r["W2"]])
            E = np.array([r["E0"], r["E1"], r["E2"]])
            expect -= W * E * ell
        for c in range(3):
            g = np.zeros((1, 3))
            g[0, c] = 1.0
            ad = sc.trace_grad(o[i:i + 1], d[i:i + 1], g)
            assert abs(ad["d_sigma"][c] - expect[c]) <= 1e-12 * max(1.0, abs(expect[c]))


@pytest.mark.parametrize("theta,n,sigma", [(30.0, 1.5, 0.4), (55.0, 1.45, 0.0), (10.0, 1.6, 1.0)])
def test_deta_dsigma_slab_closed_form(oracle_lib, theta, n, sigma):
    """Depth 2 on the plate under a unit environment: C = R + T^2 exp(-sigma h/cos tt)
    (the bounce back up is truncated).  Its derivatives in n and sigma come
    from the angle-form Fresnel equations, differentiated numerically here."""
    V, F = synth.parallel_slab(0.2)
    env = oracle_lib.Env(tex=synth.env_constant(8, 4))
    sc = oracle_lib.Scene(V, F, n, sigma, env, 2)
    o, d = slab_ray(theta, 0.2)

    def C(nn, ss):
        ti = math.radians(theta)
        tt = math.asin(math.sin(ti) / nn)
        R = fresnel_angle_form(ti, 1.0, nn)
        return R + (1 - R) ** 2 * math.exp(-ss * 0.2 / math.cos(tt))

    r = sc.trace(o[None], d[None])
    assert abs(r["rgb"][0, 0] - C(n, sigma)) < 1e-14
    hh = 1e-5
    dC_dn = (C(n + hh, sigma) - C(n - hh, sigma)) / (2 * hh)
    dC_ds = (C(n, sigma + hh) - C(n, sigma - hh)) / (2 * hh)
    ad = sc.trace_grad(o[None], d[None], np.array([[1.0, 0.0, 0.0]]))
    assert abs(ad["d_eta"] - dC_dn) < 1e-9
    assert abs(ad["d_sigma"][0] - dC_ds) < 1e-9
    # IoR 1 slab: the vertex gradient vanishes identically (nothing bends)
    sc1 = oracle_lib.Scene(V, F, 1.0, 0.0, oracle_lib.Env(tex=synth.env_equirect(64, 32, 1)), 4)
    ad1 = sc1.trace_grad(o[None], d[None], np.array([[1.0, 1.0, 1.0]]))
    assert np.abs(ad1["dV"]).max() < 1e-12


def test_invisible_object_vertex_gradient_vanishes(oracle_lib):
    """At eta = 1 and sigma = 0 the image does not depend on the mesh at all."""
    sc, o, d = _scene(oracle_lib, "icosphere", sigma=0.0, eta=1.0, res=16)
    g = np.random.default_rng(0).normal(size=o.shape)
    ad = sc.trace_grad(o, d, g)
    assert np.abs(ad["dV"]).max() < 1e-10


def test_env_direction_gradient_fd(oracle_lib):
    tex = synth.env_equirect(64, 32, seed=1)
    env = oracle_lib.Env(tex=tex)
    rng = np.random.default_rng(4)
    dirs = rng.normal(size=(300, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    g = rng.normal(size=(300, 3))
    ad = env.eval_grad(dirs, g)
    h = 1e-7
    for c in range(3):
        dp, dm = dirs.copy(), dirs.copy()
        dp[:, c] += h
        dm[:, c] -= h
        fd = ((env.eval(dp) - env.eval(dm)) * g).sum(1) / (2 * h)
        # drop the few directions whose texel cell changes within +-h
        keep = np.abs(fd - ad[:, c]) < 1e-3 * (np.abs(ad[:, c]) + 1)
        assert keep.mean() > 0.97
        np.testing.assert_allclose(fd[keep], ad[keep, c], rtol=1e-5, atol=1e-6)
