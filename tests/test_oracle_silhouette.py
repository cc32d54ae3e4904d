"""Pins of the oracle's silhouette (mask) term: the derivative of each
pixel's coverage by the object through the motion of its outline.

* A convex mesh projects to the convex hull of its projected vertices, so
  summed over the image the outline gradient along any vertex motion is the
  derivative of that polygon's area (central difference of the exact area,
  scipy's hull), and every outline point is visible.
* For one triangle the coverage of each pixel is the exact area of the
  triangle clipped to the pixel's square (Sutherland-Hodgman here, in numpy);
  the quadrature converges to its central difference as the point density
  grows.
* A mesh hidden behind another one has no outline: its vertices get no
  gradient, and the front mesh's gradient is what it is alone.
"""
import numpy as np
import pytest
from scipy.spatial import ConvexHull

from paper_2603_00413_amd import synth


def _cam(res=64, eye=(0.4, 0.5, 3.0)):
    return synth.look_at_camera(eye, res, res)


def _project(cam, X):
    """Continuous image coordinates of points X [n, 3] (pixel (x, y) covers
    [x, x+1) x [y, y+1)), written from the pinhole model: the point's
    direction in the camera frame over its depth, scaled by the image size
    over the tangent of the half field of view."""
    e = np.asarray(cam.eye, float)
    f = np.asarray(cam.target, float) - e
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(cam.up, float))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = np.tan(np.deg2rad(cam.fov_deg) / 2)
    w = X - e
    z = w @ f
    x = (w @ r) / z / (th * cam.width / cam.height)
    y = (w @ u) / z / th
    return np.stack([(x + 1) * cam.width / 2, (1 - y) * cam.height / 2], 1)


def _sphere_scene(oracle_lib, scale=0.6, offset=(0.0, 0.0, 0.0)):
    V, F = synth.icosphere(2)
    V = V * scale + np.asarray(offset)
    env = oracle_lib.Env(tex=synth.env_constant(8, 4))
    return oracle_lib.Scene(V, F, 1.5, 0.0, env, 2), V, F


@pytest.mark.parametrize("seed", [0, 1])
def test_convex_outline_is_the_hull_area_derivative(oracle_lib, seed):
    sc, V, F = _sphere_scene(oracle_lib)
    cam = _cam()
    g = np.ones(cam.width * cam.height)
    dV, (n_in, n_vis) = sc.mask_grad(cam, g, rho=64.0)
    assert n_in > 0 and n_vis == n_in          # every outline point of a convex mesh is visible
    xi = np.random.default_rng(seed).normal(size=V.shape)
    h = 1e-6
    area = lambda VV: ConvexHull(_project(cam, VV)).volume
    fd = (area(V + h * xi) - area(V - h * xi)) / (2 * h)
    an = float((dV * xi).sum())
    assert abs(an - fd) <= 1e-4 * abs(fd), (an, fd)


def _clip_area(poly, x0, y0):
    """Area of a convex polygon clipped to the square [x0, x0+1] x [y0, y0+1]."""
    def clip(P, inside, cut):
        out = []
        for i in range(len(P)):
            a, b = P[i - 1], P[i]
            ia, ib = inside(a), inside(b)
            if ib:
                if not ia:
                    out.append(cut(a, b))
                out.append(b)
            elif ia:
                out.append(cut(a, b))
        return out

    def at_x(c):
        return lambda a, b: a + (b - a) * ((c - a[0]) / (b[0] - a[0]))

    def at_y(c):
        return lambda a, b: a + (b - a) * ((c - a[1]) / (b[1] - a[1]))

    P = [np.asarray(p, float) for p in poly]
    for inside, cut in [(lambda p: p[0] >= x0, at_x(x0)), (lambda p: p[0] <= x0 + 1, at_x(x0 + 1)),
                        (lambda p: p[1] >= y0, at_y(y0)), (lambda p: p[1] <= y0 + 1, at_y(y0 + 1))]:
        P = clip(P, inside, cut)
        if not P:
            return 0.0
    P = np.array(P)
    return 0.5 * abs(np.dot(P[:, 0], np.roll(P[:, 1], -1)) - np.dot(P[:, 1], np.roll(P[:, 0], -1)))


def test_triangle_coverage_per_pixel_converges(oracle_lib):
    """One triangle facing the camera (its three edges are the outline): the
    gradient of each pixel's coverage with respect to a vertex, against the
    central difference of the exact clipped area; the error falls as the
    quadrature density grows (pixel assignment of a point is exact to half
    a point spacing)."""
    V = np.array([[-0.55, -0.4, 0.1], [0.6, -0.3, -0.1], [-0.05, 0.62, 0.05]])
    F = np.array([[0, 1, 2]], np.int32)
    env = oracle_lib.Env(tex=synth.env_constant(8, 4))
    sc = oracle_lib.Scene(V, F, 1.5, 0.0, env, 1)
    cam = synth.look_at_camera((0.0, 0.0, 3.0), 12, 12)
    W = H = 12
    rng = np.random.default_rng(3)
    g = rng.normal(size=W * H)
    xi = rng.normal(size=V.shape)
    h = 1e-6

    def loss(VV):
        P = _project(cam, VV)
        # counter-clockwise or not, the clipped area is unsigned
        return sum(g[y * W + x] * _clip_area(P, x, y) for y in range(H) for x in range(W))

    fd = (loss(V + h * xi) - loss(V - h * xi)) / (2 * h)
    errs = []
    for rho in (4.0, 4096.0):
        dV, _ = sc.mask_grad(cam, g, rho=rho)
        errs.append(abs(float((dV * xi).sum()) - fd) / abs(fd))
    # 10 % at 4 points per pixel, 1.5e-4 at 4096
    assert errs[1] < 1e-3
    assert errs[1] < errs[0] / 50


def test_hidden_mesh_gets_no_outline_gradient(oracle_lib):
    """A small sphere right behind a large one (from the camera): none of its
    outline is visible, and the large sphere's gradient is unchanged."""
    cam = _cam(eye=(0.0, 0.0, 3.0))
    Vb, F1 = synth.icosphere(2)
    Vb = Vb * 0.6
    Vs, F2 = synth.icosphere(1)
    Vs = Vs * 0.2 + np.array([0.05, -0.03, -1.2])
    V = np.concatenate([Vb, Vs])
    F = np.concatenate([F1, F2 + len(Vb)]).astype(np.int32)
    env = oracle_lib.Env(tex=synth.env_constant(8, 4))
    both = oracle_lib.Scene(V, F, 1.5, 0.0, env, 2)
    alone = oracle_lib.Scene(Vb, F1, 1.5, 0.0, env, 2)
    g = np.random.default_rng(5).normal(size=cam.width * cam.height)
    dV, _ = both.mask_grad(cam, g, rho=4.0)
    dVb, _ = alone.mask_grad(cam, g, rho=4.0)
    assert np.abs(dV[len(Vb):]).max() == 0.0
    np.testing.assert_array_equal(dV[:len(Vb)], dVb)
