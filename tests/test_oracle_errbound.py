"""Pins of the oracle's first-order bound on the rounding error of an FP32
evaluation of a pixel (the test-side yardstick for pixels where FP32 cannot
reach 1e-4): it dominates the actual change of the FP64 radiance when the
camera direction is rounded to FP32, it is homogeneous of degree one in the
environment, and it grows without limit as a refracted ray approaches the
critical angle (the derivative of cos(theta_t) diverges there)."""
import math

import numpy as np

from paper_2603_00413_amd import synth
from tests.oracle_helpers import slab_ray

H_SLAB = 0.2


def _torus(oracle_lib, env_scale=1.0):
    V, F = synth.displaced_torus(seed=5, nu=120, nv=60)
    tex = synth.env_equirect(128, 64, seed=2) * env_scale
    sc = oracle_lib.Scene(V.astype(np.float32).astype(np.float64), F, float(np.float32(1.45)),
                          np.full(3, np.float32(0.3)).astype(np.float64), oracle_lib.Env(tex=tex), 6)
    cam = synth.look_at_camera(synth.views_on_sphere(3, 3.0, seed=21)[1], 32, 32)
    o, d = oracle_lib.camera_rays(cam)
    return sc, o, d


def test_bound_covers_fp32_rounding_of_the_camera_ray(oracle_lib):
    """Rounding each camera direction to FP32 (a relative change of at most
    2^-24 per component) moves the FP64 radiance by no more than the bound,
    which charges every operation, the direction included, its rounding."""
    sc, o, d = _torus(oracle_lib)
    rgb, b = sc.errbound(o, d)
    d32 = d.astype(np.float32).astype(np.float64)
    r64 = sc.trace(o, d)
    r32 = sc.trace(o, d32)
    same = r64["sig"] == r32["sig"]
    assert same.mean() > 0.99
    np.testing.assert_array_equal(rgb, r64["rgb"])
    moved = np.abs(r32["rgb"] - r64["rgb"])[same]
    assert (moved <= b[same]).all()
    # and it is not vacuous: the bound is a small multiple of machine
    # precision on the typical pixel
    lit = np.abs(rgb) > 1e-3 * np.abs(rgb).mean()
    assert np.median(b[lit] / np.abs(rgb[lit])) < 1e-5


def test_bound_is_homogeneous_in_the_environment(oracle_lib):
    """The image is linear in the environment map, and so is every term
    |dC/dz| |z| of the bound: scaling the map by 4 scales it by 4."""
    sc, o, d = _torus(oracle_lib)
    sc4, _, _ = _torus(oracle_lib, env_scale=4.0)
    rgb, b = sc.errbound(o, d)
    rgb4, b4 = sc4.errbound(o, d)
    np.testing.assert_allclose(rgb4, 4.0 * rgb, rtol=1e-12, atol=0)
    np.testing.assert_allclose(b4, 4.0 * b, rtol=1e-12, atol=1e-300)


def test_bound_grows_toward_the_critical_angle(oracle_lib):
    """A ray inside a glass plate meets the bottom face at angle theta: as
    theta approaches asin(1/n) from below, cos(theta_t) -> 0 and the
    refracted direction's sensitivity ~ 1/cos(theta_t) diverges, and with it
    the bound (ratio at 1e-4 rad vs 0.2 rad from the critical angle above
    the ratio of the 1/cos(theta_t) factors' square roots)."""
    V, F = synth.parallel_slab(H_SLAB)
    n = 1.5
    tex = synth.env_equirect(64, 32, seed=1)
    sc = oracle_lib.Scene(V, F, n, 0.0, oracle_lib.Env(tex=tex), 1)
    thc = math.asin(1.0 / n)

    def bound(dth):
        th = thc - dth
        o = np.array([[0.0, 0.0, 0.37]])
        dd = np.array([[math.sin(th), -math.cos(th), 0.0]])
        rgb, b = sc.errbound(o, dd)
        return b.sum() / np.abs(rgb).sum()

    def cos_t(dth):
        s = n * math.sin(thc - dth)
        return math.sqrt(1.0 - s * s)

    near, far = bound(1e-4), bound(0.2)
    assert near > far * math.sqrt(cos_t(0.2) / cos_t(1e-4))
    # and a slab ray far from every critical angle is well conditioned (a
    # few tens of unit roundoffs)
    o, dd = slab_ray(30.0, H_SLAB)
    rgb, b = sc.errbound(o[None], dd[None])
    assert (b / np.abs(rgb)).max() < 1e-5


def test_jitter_instrument(oracle_lib):
    """The ray jitter used to size gradient allowances: off, it leaves every
    output bit-identical; on, it is deterministic per seed, changes the
    radiance by an amount of the order of the jitter (within the first-order
    bound scaled by the jitter over float32's unit roundoff, on pixels whose
    path stays), and is refused beyond 1e-3."""
    sc, o, d = _torus(oracle_lib)
    r0 = sc.trace(o, d)
    s0 = sc.with_(jitter=0.0, jitter_seed=5).trace(o, d)
    for k in ("rgb", "sig", "flags"):
        np.testing.assert_array_equal(r0[k], s0[k])
    u = 2.0 ** -23
    j1 = sc.with_(jitter=u, jitter_seed=5)
    a, b = j1.trace(o, d), j1.trace(o, d)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    c = sc.with_(jitter=u, jitter_seed=6).trace(o, d)
    assert not np.array_equal(a["rgb"], c["rgb"])
    same = (a["sig"] == r0["sig"]) & (c["sig"] == r0["sig"])
    assert same.mean() > 0.98
    _, bound = sc.errbound(o, d)
    moved = np.abs(a["rgb"] - r0["rgb"])[same]
    assert moved.max() > 0
    # the bound charges each operation 2^-24; the jitter moves every ray by up
    # to u = 2^-23 per component, and FP64 itself adds nothing visible
    assert (moved <= 4 * (u / 2.0 ** -24) * bound[same] + 1e-15).all()
    g = np.random.default_rng(1).normal(size=r0["rgb"].shape)
    g0 = sc.trace_grad(o, d, g)
    g1 = j1.trace_grad(o, d, g)
    assert 0 < np.linalg.norm(g1["dV"] - g0["dV"]) <= 1e-3 * np.linalg.norm(g0["dV"])
    import pytest
    with pytest.raises(AssertionError):
        sc.with_(jitter=2e-3).trace(o, d)
