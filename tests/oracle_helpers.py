"""Shared helpers for the oracle pin tests (test-side code, no tracer arithmetic
beyond what each test states as its independent reference)."""
from __future__ import annotations

import numpy as np


def link_tree(recs):
    """Attach parent / children indices to depth-first tree records."""
    stack = []
    for i, r in enumerate(recs):
        while stack and recs[stack[-1]]["depth"] >= r["depth"]:
            stack.pop()
        r["parent"] = stack[-1] if stack else -1
        r["children"] = []
        if stack:
            recs[stack[-1]]["children"].append(i)
        stack.append(i)
    return recs


def slab_ray(theta_deg: float, h: float, z: float = 0.37, dist: float = 2.0):
    """A ray in the x-y plane hitting the top face (y = h/2) of the slab at
    angle theta from the normal, aimed at the point (0, h/2, z)."""
    th = np.deg2rad(theta_deg)
    d = np.array([np.sin(th), -np.cos(th), 0.0])
    p = np.array([0.0, h / 2.0, z])
    return p - dist * d, d


def fresnel_angle_form(theta_i: float, n1: float, n2: float) -> float:
    """Textbook unpolarised reflectance from the angle forms
    r_s = -sin(ti - tt)/sin(ti + tt), r_p = tan(ti - tt)/tan(ti + tt)."""
    if theta_i == 0.0:
        return ((n1 - n2) / (n1 + n2)) ** 2
    tt = np.arcsin(n1 / n2 * np.sin(theta_i))
    rs = -np.sin(theta_i - tt) / np.sin(theta_i + tt)
    rp = np.tan(theta_i - tt) / np.tan(theta_i + tt)
    return 0.5 * (rs * rs + rp * rp)


def chord_length(V, F, o, d):
    """Total length of the line o + s d (s > 0) inside a closed mesh, from all
    line/triangle crossings (numpy, independent plane + edge-sign test).
    Returns (length, n_crossings, min_edge_margin)."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    den = n @ d
    with np.errstate(divide="ignore", invalid="ignore"):
        s = ((a - o) * n).sum(1) / den
    x = o + s[:, None] * d
    # signed areas of the sub-triangles relative to the face normal
    wa = (np.cross(c - b, x - b) * n).sum(1)
    wb = (np.cross(a - c, x - c) * n).sum(1)
    wc = (np.cross(b - a, x - a) * n).sum(1)
    nn = (n * n).sum(1)
    inside = (wa >= 0) & (wb >= 0) & (wc >= 0) & (s > 1e-9) & (den != 0)
    ss = np.sort(s[inside])
    margin = np.min(np.minimum(np.minimum(wa, wb), wc)[inside] / nn[inside]) if inside.any() else 1.0
    L = float(np.sum(ss[1::2] - ss[0::2])) if len(ss) % 2 == 0 else np.nan
    return L, len(ss), margin
