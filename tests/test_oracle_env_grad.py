"""Pins of the oracle's gradient with respect to the equirect environment's
texels (the exterior half of the sampling split, Sec. 3.3: a ray leaving the
object takes the environment radiance, a bilinear lookup, Sec. 3.2).

Independent references: Euler's identity for a function homogeneous of
degree 1 in the texels, and central finite differences texel by texel.
"""
import numpy as np

from tests.test_oracle_absorption import _icosphere, _random_grid

def test_texel_gradient_euler_identity(oracle_lib):
    """The image is linear in the environment map (every path ends in one
    lookup, weighted by quantities that do not depend on the texels), so for
    any upstream gradient g: sum over texels of d_tex * tex = sum over pixels
    of g . C (Euler's identity for a function homogeneous of degree 1)."""
    for absorb in (None, _random_grid(oracle_lib, 3)):
        sc, o, d = _icosphere(oracle_lib, res=20, absorb=absorb)
        g = np.random.default_rng(12).normal(size=o.shape)
        ad = sc.trace_grad(o, d, g, want_tex=True)
        lhs = float((ad["d_tex"] * sc.env.tex).sum())
        rhs = float((ad["rgb"] * g).sum())
        assert abs(lhs - rhs) <= 1e-11 * abs(rhs) + 1e-12, (lhs, rhs)


def test_texel_gradient_fd(oracle_lib):
    """d/d(texel), texel by texel, against central differences."""
    sc, o, d = _icosphere(oracle_lib, res=16)
    rng = np.random.default_rng(13)
    g = rng.normal(size=o.shape)
    ad = sc.trace_grad(o, d, g, want_tex=True)["d_tex"]
    nz = np.argwhere(np.abs(ad) > 1e-3)
    assert len(nz) > 20
    h = 1e-4
    for idx in nz[rng.choice(len(nz), 10, replace=False)]:
        idx = tuple(idx)
        tp, tm = sc.env.tex.copy(), sc.env.tex.copy()
        tp[idx] += h
        tm[idx] -= h
        cp = sc.with_(env=oracle_lib.Env(tex=tp)).trace(o, d)["rgb"]
        cm = sc.with_(env=oracle_lib.Env(tex=tm)).trace(o, d)["rgb"]
        fd = float(((cp - cm) * g).sum() / (2 * h))
        assert abs(fd - ad[idx]) <= 1e-9 * max(abs(ad[idx]), 1.0), (idx, fd, ad[idx])
