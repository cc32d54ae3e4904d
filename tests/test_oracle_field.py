"""Pins of the oracle's volumetric environment field (the exterior half of
the sampling split: emission and transmittance of every segment outside the
object, composited before what lies beyond it).

* A constant field renders the closed form of the volume rendering integral,
  c (1 - e^{-sigma l}) + e^{-sigma l} E, for every sample count (the midpoint
  sum telescopes), with l the segment's length inside the box.
* Through an invisible object (IoR 1, no absorption) l is the box chord minus
  the object's chord (numpy line/mesh crossings): interior segments do not
  sample the field.
* A vanishing density leaves the plain render.
* Central differences of the FP64 render pin the gradient with respect to the
  grid and plane values, the vertices and the IoR."""
import math

import numpy as np
import pytest

from paper_2603_00413_amd import synth
from tests.oracle_helpers import chord_length

LO, HI = (-1.2, -1.1, -1.3), (1.25, 1.15, 1.05)


def _field(oracle_lib, f0=0.3, color=(0.2, 0.5, 0.9), seed=None, n=(5, 4, 6), res=7, samples=16):
    nx, ny, nz = n
    if seed is None:
        grid = np.zeros((nz, ny, nx, 4))
        grid[..., 0] = f0
        grid[..., 1:] = color
        planes = np.zeros((3, res, res, 4))
    else:
        rng = np.random.default_rng(seed)
        grid = rng.uniform(-1.0, 0.5, (nz, ny, nx, 4))
        planes = rng.uniform(-0.3, 0.3, (3, res, res, 4))
    return oracle_lib.Field(grid, planes, LO, HI, samples)


def _box_chord(o, d):
    t0, t1 = 0.0, math.inf
    for a in range(3):
        ta, tb = (LO[a] - o[a]) / d[a], (HI[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(t1 - t0, 0.0)


def _rays(n, seed, miss_radius=None):
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o = 3.0 * o / np.linalg.norm(o, axis=1, keepdims=True)
    tgt = rng.uniform(-0.6, 0.6, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


@pytest.mark.parametrize("samples", [1, 7, 32])
def test_constant_field_closed_form(oracle_lib, samples):
    """Rays that miss a small sphere: pixel = c (1 - e^{-s l}) + e^{-s l} E."""
    V, F = synth.icosphere(1)
    V = V * 0.05 + np.array([0.0, 0.0, 5.0])          # far outside the rays' paths and the box
    E = 0.7
    env = oracle_lib.Env(tex=np.full((4, 8, 3), E))
    fld = _field(oracle_lib, samples=samples)
    sc = oracle_lib.Scene(V, F, 1.5, 0.0, env, 2, field=fld)
    o, d = _rays(200, 1)
    rgb = sc.trace(o, d)["rgb"]
    sig = math.log1p(math.exp(0.3))
    for i in range(len(o)):
        l = _box_chord(o[i], d[i])
        ref = np.array([0.2, 0.5, 0.9]) * (1 - math.exp(-sig * l)) + math.exp(-sig * l) * E
        np.testing.assert_allclose(rgb[i], ref, rtol=1e-12, atol=1e-14)


def test_invisible_object_skips_the_interior(oracle_lib):
    V, F = synth.displaced_torus(seed=2, nu=80, nv=40)
    E = 0.7
    env = oracle_lib.Env(tex=np.full((4, 8, 3), E))
    sc = oracle_lib.Scene(V, F, 1.0, 0.0, env, 8, field=_field(oracle_lib))
    o, d = _rays(300, 2)
    r = sc.trace(o, d)
    sig = math.log1p(math.exp(0.3))
    checked = 0
    for i in range(len(o)):
        L, n, margin = chord_length(V, F, o[i], d[i])
        if not (margin > 1e-6) or n > 8 or not np.isfinite(L):
            continue
        lext = _box_chord(o[i], d[i]) - L
        ref = np.array([0.2, 0.5, 0.9]) * (1 - math.exp(-sig * lext)) + math.exp(-sig * lext) * E
        np.testing.assert_allclose(r["rgb"][i], ref, rtol=1e-10, atol=1e-12)
        checked += n > 0
    assert checked > 50


def test_vanishing_density_is_the_plain_render(oracle_lib):
    V, F = synth.icosphere(2)
    tex = synth.env_equirect(32, 16, seed=3)
    env = oracle_lib.Env(tex=tex)
    fld = _field(oracle_lib, f0=-60.0)
    plain = oracle_lib.Scene(V, F, 1.5, (0.5, 0.2, 0.1), env, 4)
    with_f = plain.with_(field=fld)
    cam = synth.look_at_camera((0.3, 0.4, 2.9), 24, 24)
    o, d = oracle_lib.camera_rays(cam)
    np.testing.assert_allclose(with_f.trace(o, d)["rgb"], plain.trace(o, d)["rgb"], rtol=0, atol=1e-20)


def _grad_scene(oracle_lib):
    V, F = synth.icosphere(2)
    V = V * 0.8
    tex = synth.env_equirect(32, 16, seed=3)
    fld = _field(oracle_lib, seed=4)
    sc = oracle_lib.Scene(V, F, 1.5, (0.5, 0.2, 0.1), oracle_lib.Env(tex=tex), 4, field=fld)
    cam = synth.look_at_camera((0.3, 0.4, 2.9), 12, 12)
    o, d = oracle_lib.camera_rays(cam)
    return sc, V, F, fld, o, d


def test_field_gradient_fd(oracle_lib):
    sc, V, F, fld, o, d = _grad_scene(oracle_lib)
    ref = sc.trace(o, d)
    keep = (ref["flags"] & (1 | 2 | 4 | 8 | 128)) == 0
    g = np.random.default_rng(5).normal(size=o.shape) * keep[:, None]
    r = sc.trace_grad(o, d, g)
    dG, dP = r["d_field"]
    rng = np.random.default_rng(6)
    xg, xp = rng.normal(size=fld.grid.shape), rng.normal(size=fld.planes.shape)
    an = float((dG * xg).sum() + (dP * xp).sum())
    h = 1e-6

    def loss(s):
        f2 = oracle_lib.Field(fld.grid + s * xg, fld.planes + s * xp, LO, HI, fld.samples)
        return float((sc.with_(field=f2).trace(o, d)["rgb"] * g).sum())

    fd = (loss(h) - loss(-h)) / (2 * h)
    assert abs(an - fd) <= 1e-6 * abs(fd), (an, fd)


def test_vertex_and_ior_gradient_fd_with_field(oracle_lib):
    """The field's segments end at the hit points, so their emission and
    transmittance move with the vertices; and the IoR gradient."""
    sc, V, F, fld, o, d = _grad_scene(oracle_lib)
    ref = sc.trace(o, d)
    keep = (ref["flags"] & (1 | 2 | 4 | 8 | 128)) == 0
    g = np.random.default_rng(7).normal(size=o.shape) * keep[:, None]
    r = sc.trace_grad(o, d, g)
    xi = np.random.default_rng(8).normal(size=V.shape)
    h = 1e-6

    def loss(VV, eta=1.5):
        rr = sc.with_(V=VV, eta=eta).trace(o, d)
        same = rr["hash"] == ref["hash"]
        assert same[keep].all()
        return float((rr["rgb"] * g).sum())

    fd = (loss(V + h * xi) - loss(V - h * xi)) / (2 * h)
    an = float((r["dV"] * xi).sum())
    assert abs(an - fd) <= 1e-5 * abs(fd), (an, fd)
    fe = (loss(V, 1.5 + h) - loss(V, 1.5 - h)) / (2 * h)
    assert abs(r["d_eta"] - fe) <= 1e-5 * abs(fe)
