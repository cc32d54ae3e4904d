"""Pins of the oracle's spatially varying absorption (Eq. 11 with the rate
sampled along the interior segment, Sec. 3.2).

The rate mu_t(x) is a trilinear RGB grid; an interior segment of length t is
attenuated by exp(-(t/S) sum_s mu_t(x_s)) at the S midpoints x_s.  Each pin
states its independent reference: the constant-rate renderer, a closed-form
line integral of a linear rate through the glass plate, the exactness of the
midpoint rule for linear integrands (any S), and central finite differences
of the forward pass for the grid and vertex gradients.
"""
import math

import numpy as np
import pytest

from paper_2603_00413_amd import synth
from tests.oracle_helpers import fresnel_angle_form, link_tree, slab_ray

BAD = 4 | 8 | 1 | 2   # grazing, TIR boundary, degenerate normal, leak
H_SLAB = 0.2


def _icosphere(oracle_lib, res=24, depth=4, absorb=None, sigma=(0.5, 0.2, 0.1)):
    V, F = synth.icosphere(3)
    env = oracle_lib.Env(tex=synth.env_equirect(64, 32, seed=1))
    sc = oracle_lib.Scene(V, F, 1.5, sigma, env, depth, absorb=absorb)
    o, d = oracle_lib.camera_rays(synth.look_at_camera((0.0, 0.0, 3.0), res, res))
    return sc, o, d


def _grid(fn, n=(5, 4, 6), lo=(-1.1, -1.05, -1.2), hi=(1.15, 1.1, 1.0)):
    """Node values fn(x, y, z) -> [..., 3] on the grid's nodes, layout [nz, ny, nx, 3]."""
    xs = [np.linspace(lo[a], hi[a], n[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return fn(X, Y, Z), lo, hi


def test_constant_grid_is_the_constant_rate(oracle_lib):
    """A grid holding sigma at every node is the homogeneous medium: the same
    colours and vertex / IoR gradients, and the grid gradient summed over the
    nodes is d/dsigma (the interpolation weights of every sample sum to 1)."""
    sigma = np.array([0.5, 0.2, 0.1])
    mu, lo, hi = _grid(lambda X, Y, Z: np.broadcast_to(sigma, X.shape + (3,)).copy())
    ab = oracle_lib.Absorption(mu, lo, hi, samples=5)
    sc_h, o, d = _icosphere(oracle_lib, sigma=sigma)
    sc_g = sc_h.with_(absorb=ab, sigma=(9.0, 9.0, 9.0))    # sigma must be ignored
    rng = np.random.default_rng(4)
    g = rng.normal(size=o.shape)
    a, b = sc_h.trace_grad(o, d, g), sc_g.trace_grad(o, d, g)
    np.testing.assert_allclose(b["rgb"], a["rgb"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(b["dV"], a["dV"], rtol=1e-9, atol=1e-11)
    assert abs(b["d_eta"] - a["d_eta"]) <= 1e-10 * abs(a["d_eta"]) + 1e-12
    np.testing.assert_allclose(b["d_sigma"], 0.0)
    np.testing.assert_allclose(b["d_mu"].sum(axis=(0, 1, 2)), a["d_sigma"], rtol=1e-10)
    assert np.abs(a["d_sigma"]).min() > 1e-3        # the pin is not vacuous


@pytest.mark.parametrize("samples", [1, 3])
def test_linear_rate_through_the_plate(oracle_lib, samples):
    """mu_t = a + b x is reproduced exactly by trilinear interpolation and
    integrated exactly by the midpoint rule, so the light leaving the bottom
    of the plate carries T^2 exp(-L (a + b x_mid)), L the chord length, x_mid
    the chord's midpoint (entry at x = 0, exit at x = L sin t_t)."""
    n, theta, a, b = 1.5, 45.0, 0.4, 0.9
    mu, lo, hi = _grid(lambda X, Y, Z: np.stack([a + b * X, 0.5 * (a + b * X), 0 * X], -1),
                       n=(5, 2, 2), lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0))
    V, F = synth.parallel_slab(H_SLAB)
    env = oracle_lib.Env(tex=synth.env_constant(8, 4))
    sc = oracle_lib.Scene(V, F, n, 0.0, env, 4,
                          absorb=oracle_lib.Absorption(mu, lo, hi, samples=samples))
    o, d = slab_ray(theta, H_SLAB)
    recs = link_tree(sc.tree(o, d))
    refr = recs[recs[0]["children"][1]]
    out = recs[refr["children"][1]]
    tt = math.asin(math.sin(math.radians(theta)) / n)
    L = H_SLAB / math.cos(tt)
    tau = L * (a + b * 0.5 * L * math.sin(tt))
    T = 1.0 - fresnel_angle_form(math.radians(theta), 1.0, n)
    assert abs(refr["t"] - L) < 1e-14
    assert abs(out["W0"] - T * T * math.exp(-tau)) < 1e-14
    assert abs(out["W1"] - T * T * math.exp(-0.5 * tau)) < 1e-14
    assert abs(out["W2"] - T * T) < 1e-14


def test_linear_rate_any_sample_count(oracle_lib):
    """For a rate linear in position every S gives the same image (the
    midpoint rule is exact on each step), on a curved multi-bounce object."""
    mu, lo, hi = _grid(lambda X, Y, Z: np.stack([0.3 + 0.2 * X - 0.1 * Z, 0.2 + 0.1 * Y,
                                                 0.5 + 0.0 * X], -1))
    sc, o, d = _icosphere(oracle_lib, res=16)
    ref = sc.with_(absorb=oracle_lib.Absorption(mu, lo, hi, samples=1)).trace(o, d)["rgb"]
    for s in (2, 7):
        img = sc.with_(absorb=oracle_lib.Absorption(mu, lo, hi, samples=s)).trace(o, d)["rgb"]
        np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-14)


def _fd_mask(sc_p, sc_m, sc0, o, d):
    rp, rm, r0 = sc_p.trace(o, d), sc_m.trace(o, d), sc0.trace(o, d)
    ok = (rp["hash"] == rm["hash"]) & (rp["hash"] == r0["hash"])
    ok &= ((r0["flags"] | rp["flags"] | rm["flags"]) & BAD) == 0
    return ok, rp["rgb"], rm["rgb"]


def _random_grid(oracle_lib, seed, samples=6):
    rng = np.random.default_rng(seed)
    mu, lo, hi = _grid(lambda X, Y, Z: rng.uniform(0.05, 0.9, X.shape + (3,)))
    return oracle_lib.Absorption(mu, lo, hi, samples=samples)


def test_grid_value_gradient_fd(oracle_lib):
    """d/d(grid value), node by node, against central differences (the
    forward pass is linear in each value inside the exponent)."""
    ab = _random_grid(oracle_lib, 7)
    sc, o, d = _icosphere(oracle_lib, res=16, absorb=ab)
    rng = np.random.default_rng(8)
    g = rng.normal(size=o.shape)
    r0 = sc.trace(o, d)
    ok0 = (r0["flags"] & BAD) == 0
    ad = sc.trace_grad(o, d, g * ok0[:, None])["d_mu"]
    nz = np.argwhere(np.abs(ad) > 1e-4)
    assert len(nz) > 20
    h = 1e-6
    for idx in nz[rng.choice(len(nz), 12, replace=False)]:
        idx = tuple(idx)
        def with_node(step):
            mu = ab.mu.copy()
            mu[idx] += step
            return sc.with_(absorb=oracle_lib.Absorption(mu, ab.lo, ab.hi, ab.samples))
        ok, cp, cm = _fd_mask(with_node(h), with_node(-h), sc, o, d)
        ok &= ok0
        fd = float(((cp - cm) * g * ok[:, None]).sum() / (2 * h))
        assert np.array_equal(ok, ok0)
        assert abs(fd - ad[idx]) <= 1e-6 * abs(ad[idx]) + 1e-9, (idx, fd, ad[idx])


def test_vertex_and_eta_gradient_fd_with_grid(oracle_lib):
    """With a varying rate the segment's samples move with the geometry, so
    the vertex and IoR gradients carry terms through the rate's spatial
    gradient; directional central differences (Richardson) pin them."""
    ab = _random_grid(oracle_lib, 9)
    sc, o, d = _icosphere(oracle_lib, res=24, absorb=ab)
    rng = np.random.default_rng(10)
    g = rng.normal(size=o.shape)
    h = 2e-7

    def rich(make):
        ok1, cp1, cm1 = _fd_mask(make(h), make(-h), sc, o, d)
        ok2, cp2, cm2 = _fd_mask(make(0.5 * h), make(-0.5 * h), sc, o, d)
        p1 = ((cp1 - cm1) * g).sum(1) / (2 * h)
        p2 = ((cp2 - cm2) * g).sum(1) / h
        ok = ok1 & ok2 & (np.abs(p1 - p2) <= 1e-4 * (np.abs(p2) + 1.0))
        return ok, (4 * p2 - p1) / 3

    for k in range(4):
        delta = rng.normal(size=sc.V.shape)
        delta /= np.abs(delta).max()
        ok, pix = rich(lambda s: sc.with_(V=sc.V + s * delta))
        assert ok.mean() > 0.8
        ad = sc.trace_grad(o, d, g * ok[:, None])
        an = float((ad["dV"] * delta).sum())
        fd = float(pix[ok].sum())
        assert abs(fd - an) <= 2e-6 * max(abs(an), 1.0) + 1e-8 * np.abs(ad["dV"]).sum(), (k, fd, an)
    ok, pix = rich(lambda s: sc.with_(eta=sc.eta + s))
    ad = sc.trace_grad(o, d, g * ok[:, None])
    fd = float(pix[ok].sum())
    assert abs(fd - ad["d_eta"]) <= 1e-6 * abs(ad["d_eta"]) + 1e-7, (fd, ad["d_eta"])

