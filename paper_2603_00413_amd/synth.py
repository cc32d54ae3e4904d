"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *creates data*: meshes, environment maps, camera poses and
MLP weights.  It holds none of the tracer's arithmetic (no intersection,
shading, Fresnel, absorption, normal construction, environment lookup or
camera-ray generation), so both the FP64 oracle and the HIP path can consume
its outputs without sharing any of the method's code.

The paper's datasets (multi-view captures, HDR maps) are not available; these
generators stand in for them with object-centred closed meshes that fit inside
the unit sphere, cameras on a sphere of radius 3 looking at the origin, and a
smooth HDR-like sky with bright blobs (Sec. 4 and the implementation appendix
describe object-centred captures of glass objects under HDR environments).

All arrays are numpy: vertices float64 [Nv,3], faces int32 [Nf,3] with
counter-clockwise winding seen from outside (outward geometric normal).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------


def _orient_outward(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Flip all faces if the signed volume of a closed mesh is negative."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    if vol < 0:
        F = F[:, [0, 2, 1]].copy()
    return F


def icosphere(subdiv: int = 3, radius: float = 1.0):
    """Icosahedron subdivided `subdiv` times, projected to the sphere.

    subdiv=3 gives 642 vertices and 1,280 faces.  The 12 original icosahedron
    vertices keep indices 0..11.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = V[i] + V[j]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        nf = []
        for (a, b, c) in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    Va = np.stack(V) * radius
    Fa = _orient_outward(Va, np.asarray(F, dtype=np.int32))
    return Va, Fa.astype(np.int32)


def displaced_torus(seed: int = 2, R: float = 0.65, r: float = 0.3,
                    nu: int = 320, nv: int = 160, n_waves: int = 8,
                    amplitude: float = 0.03):
    """Genus-1 torus around the y axis, displaced along its normal.

    The displacement is a sum of `n_waves` seamless sinusoids
    a_k sin(m_k u + n_k v + phi_k) with integer m_k in [1,6], n_k in [1,4]
    and sum |a_k| = amplitude.  nu x nv = 320 x 160 gives 51,200 vertices
    and 102,400 faces.
    """
    rng = np.random.default_rng(seed)
    m = rng.integers(1, 7, size=n_waves)
    n = rng.integers(1, 5, size=n_waves)
    ph = rng.uniform(0, 2 * np.pi, size=n_waves)
    a = rng.uniform(0.5, 1.0, size=n_waves)
    a = a / a.sum() * amplitude
    u = np.arange(nu) * (2 * np.pi / nu)
    v = np.arange(nv) * (2 * np.pi / nv)
    U, Vv = np.meshgrid(u, v, indexing="ij")          # [nu, nv]
    h = np.zeros_like(U)
    for k in range(n_waves):
        h += a[k] * np.sin(m[k] * U + n[k] * Vv + ph[k])
    cu, su, cv, sv = np.cos(U), np.sin(U), np.cos(Vv), np.sin(Vv)
    nrm = np.stack([cv * cu, sv, cv * su], axis=-1)
    ctr = np.stack([R * cu, np.zeros_like(U), R * su], axis=-1)
    P = ctr + (r + h)[..., None] * nrm
    Vx = P.reshape(-1, 3)
    idx = np.arange(nu * nv).reshape(nu, nv)
    i00 = idx
    i10 = np.roll(idx, -1, axis=0)
    i01 = np.roll(idx, -1, axis=1)
    i11 = np.roll(i10, -1, axis=1)
    f1 = np.stack([i00, i10, i11], axis=-1).reshape(-1, 3)
    f2 = np.stack([i00, i11, i01], axis=-1).reshape(-1, 3)
    F = np.empty((2 * nu * nv, 3), dtype=np.int32)
    F[0::2] = f1
    F[1::2] = f2
    F = _orient_outward(Vx, F)
    return Vx.astype(np.float64), F.astype(np.int32)


def parallel_slab(h: float = 0.2, half: float = 20.0):
    """Two disjoint parallel quads y = +h/2 (facing +y) and y = -h/2 (facing -y).

    Each quad is two triangles whose four vertices are all on the plane, so
    every vertex normal equals the plane normal exactly.  Not a closed mesh:
    it models an infinite glass plate of thickness h for closed-form checks.
    """
    y0, y1 = h / 2.0, -h / 2.0
    V = np.array([
        [-half, y0, -half], [half, y0, -half], [half, y0, half], [-half, y0, half],
        [-half, y1, -half], [half, y1, -half], [half, y1, half], [-half, y1, half],
    ], dtype=np.float64)
    # top quad: counter-clockwise seen from +y  -> normal +y
    # bottom quad: counter-clockwise seen from -y -> normal -y
    F = np.array([[0, 2, 1], [0, 3, 2], [4, 5, 6], [4, 6, 7]], dtype=np.int32)
    return V, F


def planar_sheet(n: int = 8, seed: int = 0, jitter: float = 0.3):
    """A jittered planar triangulated sheet in the plane z = 0 (normal +z)."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(-1, 1, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    step = 2.0 / n
    J = rng.uniform(-jitter, jitter, size=X.shape + (2,)) * step
    J[0, :, 0] = J[-1, :, 0] = 0
    J[:, 0, 1] = J[:, -1, 1] = 0
    V = np.stack([X + J[..., 0], Y + J[..., 1], np.zeros_like(X)], -1).reshape(-1, 3)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    a, b = idx[:-1, :-1], idx[1:, :-1]
    c, d = idx[1:, 1:], idx[:-1, 1:]
    F = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                        np.stack([a, c, d], -1).reshape(-1, 3)]).astype(np.int32)
    return V, F


# --------------------------------------------------------------------------
# SDF union meshed by marching tetrahedra
# --------------------------------------------------------------------------

# Kuhn split of the unit cube into 6 tetrahedra along the main diagonal
# (corner 0 = (0,0,0) to corner 7 = (1,1,1)); corner c has offset
# ((c>>0)&1, (c>>1)&1, (c>>2)&1).
_KUHN = np.array([[0, 1, 3, 7], [0, 3, 2, 7], [0, 2, 6, 7],
                  [0, 6, 4, 7], [0, 4, 5, 7], [0, 5, 1, 7]], dtype=np.int64)


@dataclass
class SdfUnion:
    """Union (pointwise min) of tori and spheres, all inside radius ~0.9."""
    tori: list      # (center[3], axis[3], R, r)
    spheres: list   # (center[3], radius)

    def __call__(self, P: np.ndarray) -> np.ndarray:
        d = np.full(P.shape[:-1], np.inf)
        for (c, ax, R, r) in self.tori:
            q = P - c
            h = q @ ax
            rad = np.sqrt(np.maximum((q * q).sum(-1) - h * h, 0.0))
            d = np.minimum(d, np.sqrt((rad - R) ** 2 + h * h) - r)
        for (c, rr) in self.spheres:
            d = np.minimum(d, np.linalg.norm(P - c, axis=-1) - rr)
        return d


def random_sdf_union(seed: int, n_tori: int = 3, n_spheres: int = 2) -> SdfUnion:
    rng = np.random.default_rng(seed)
    tori, spheres = [], []
    for _ in range(n_tori):
        R = rng.uniform(0.25, 0.35)
        r = rng.uniform(0.07, 0.11)
        lim = 0.9 - R - r
        c = rng.uniform(-1, 1, 3)
        c = c / max(np.linalg.norm(c), 1e-9) * rng.uniform(0.0, lim)
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        tori.append((c, ax, R, r))
    for _ in range(n_spheres):
        rr = rng.uniform(0.15, 0.25)
        c = rng.uniform(-1, 1, 3)
        c = c / max(np.linalg.norm(c), 1e-9) * rng.uniform(0.0, 0.9 - rr)
        spheres.append((c, rr))
    return SdfUnion(tori, spheres)


def marching_tetrahedra(sdf, res: int, lo: float = -1.0, hi: float = 1.0,
                        shell: float | None = None):
    """Extract the zero level set of `sdf` on a res^3 grid of cubes.

    Each cube is split into 6 Kuhn tetrahedra; each tetrahedron with a sign
    change emits 1 or 2 triangles whose vertices lie on the tetrahedron's
    edges, linearly interpolated.  Vertices are welded by grid-edge key, so
    the mesh is closed and manifold (grid values are nudged away from 0).
    Each face is oriented so its normal points from the negative (inside)
    corners of its tetrahedron toward the positive (outside) ones.
    If `shell` is given the field is |sdf| - shell (a thin hollow wall).
    """
    n = res + 1
    xs = np.linspace(lo, hi, n)
    G = np.stack(np.meshgrid(xs, xs, xs, indexing="ij"), -1)
    P = G.reshape(-1, 3)
    fv = np.concatenate([sdf(P[i:i + (1 << 20)]) for i in range(0, len(P), 1 << 20)])
    if shell is not None:
        fv = np.abs(fv) - shell
    fv = np.where(fv == 0.0, 1e-12, fv)
    gid = np.arange(n ** 3, dtype=np.int64).reshape(n, n, n)
    neg = (fv < 0).reshape(n, n, n)
    cs = np.zeros((res, res, res), dtype=np.int8)
    for c in range(8):
        dx, dy, dz = (c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1
        cs += neg[dx:dx + res, dy:dy + res, dz:dz + res]
    cube = np.nonzero((cs > 0) & (cs < 8))
    base = gid[cube]
    offs = np.array([((c >> 0) & 1) * n * n + ((c >> 1) & 1) * n + ((c >> 2) & 1)
                     for c in range(8)], dtype=np.int64)
    cid = base[:, None] + offs[None, :]
    tets = cid[:, _KUHN].reshape(-1, 4)
    ts = fv[tets] < 0
    cnt = ts.sum(1)
    m = (cnt > 0) & (cnt < 4)
    tets, ts, cnt = tets[m], ts[m], cnt[m]

    tri_edges = []                   # ([F,3] edge end a, [F,3] edge end b, [F,3] outward ref)
    for odd_inside in (True, False):
        sel = (cnt == 1) if odd_inside else (cnt == 3)
        T, S = tets[sel], ts[sel]
        if len(T) == 0:
            continue
        odd = np.argmax(S if odd_inside else ~S, axis=1)
        others = np.array([[j for j in range(4) if j != k] for k in range(4)])[odd]
        a = T[np.arange(len(T)), odd]
        b = T[np.arange(len(T))[:, None], others]
        A = np.repeat(a[:, None], 3, 1)
        ref = P[b].mean(1) - P[a]
        if not odd_inside:
            ref = -ref
        tri_edges.append((A, b, ref))
    sel = cnt == 2
    T, S = tets[sel], ts[sel]
    if len(T):
        order = np.argsort(~S, axis=1, kind="stable")   # inside corners first
        ins = np.take_along_axis(T, order[:, :2], 1)
        out = np.take_along_axis(T, order[:, 2:], 1)
        ref = P[out].mean(1) - P[ins].mean(1)
        qa = np.stack([ins[:, 0], ins[:, 0], ins[:, 1], ins[:, 1]], 1)
        qb = np.stack([out[:, 0], out[:, 1], out[:, 1], out[:, 0]], 1)
        tri_edges.append((qa[:, [0, 1, 2]], qb[:, [0, 1, 2]], ref))
        tri_edges.append((qa[:, [0, 2, 3]], qb[:, [0, 2, 3]], ref))
    EA = np.concatenate([t[0] for t in tri_edges])
    EB = np.concatenate([t[1] for t in tri_edges])
    REF = np.concatenate([t[2] for t in tri_edges])
    lo_, hi_ = np.minimum(EA, EB), np.maximum(EA, EB)
    key = (lo_ * (n ** 3) + hi_).reshape(-1)
    uk, inv = np.unique(key, return_inverse=True)
    ka, kb = uk // (n ** 3), uk % (n ** 3)
    wa, wb = fv[ka], fv[kb]
    tt = wa / (wa - wb)
    V = P[ka] + tt[:, None] * (P[kb] - P[ka])
    F = inv.reshape(-1, 3).astype(np.int64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = (nrm * REF).sum(-1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    area2 = np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=-1)
    F = F[area2 > 0]
    return V, F.astype(np.int32)


def sdf_union_mesh(seed: int = 3, res: int = 128, shell: float | None = None):
    """Seeded union of 3 tori + 2 spheres meshed on a res^3 grid over [-1,1]^3."""
    return marching_tetrahedra(random_sdf_union(seed), res, shell=shell)


def sdf_union_faces(target_faces: int, seed: int, shell: float | None = None,
                    max_res: int = 512):
    """SDF-union mesh with about `target_faces` triangles: the face count of
    marching tetrahedra grows with the square of the grid resolution, so the
    resolution is scaled from a coarse trial mesh."""
    V0, F0 = sdf_union_mesh(seed, 48, shell=shell)
    res = int(round(48 * math.sqrt(target_faces / max(len(F0), 1))))
    res = max(16, min(res, max_res))
    return sdf_union_mesh(seed, res, shell=shell)


def mesh_stats(V: np.ndarray, F: np.ndarray) -> dict:
    """Closedness / manifoldness / Euler characteristic of a triangle mesh."""
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    und = np.sort(e, axis=1)
    key = und[:, 0].astype(np.int64) * (len(V) + 1) + und[:, 1]
    uk, cnt = np.unique(key, return_counts=True)
    dk = e[:, 0].astype(np.int64) * (len(V) + 1) + e[:, 1]
    directed_unique = len(np.unique(dk)) == len(dk)
    used = np.unique(F)
    chi = len(used) - len(uk) + len(F)
    return {
        "closed_manifold": bool((cnt == 2).all()),
        "consistently_oriented": bool(directed_unique),
        "euler": int(chi),
        "genus_if_connected": (2 - chi) / 2.0,
        "n_edges": int(len(uk)),
    }


# --------------------------------------------------------------------------
# environment data
# --------------------------------------------------------------------------


def _texel_dirs(W: int, H: int) -> np.ndarray:
    """Directions of equirect texel centres: row 0 at the zenith (+y),
    column angle phi measured as atan2(x, -z), phi = (u - 1/2) 2 pi."""
    u = (np.arange(W) + 0.5) / W
    v = (np.arange(H) + 0.5) / H
    phi = (u - 0.5) * 2 * np.pi
    th = v * np.pi
    TH, PH = np.meshgrid(th, phi, indexing="ij")      # [H, W]
    return np.stack([np.sin(TH) * np.sin(PH), np.cos(TH), -np.sin(TH) * np.cos(PH)], -1)


def sky_radiance(dirs: np.ndarray, seed: int, n_blobs: int = 16) -> np.ndarray:
    """Smooth HDR-like sky: ground/horizon/zenith gradient + Gaussian blobs.

    blob k adds a_k c_k exp(-(1 - d.mu_k)/s_k^2), mu_k uniform on the sphere,
    s_k ~ U[0.05, 0.3], a_k ~ U[1, 8], c_k ~ U[0.2, 1]^3.
    """
    rng = np.random.default_rng(seed)
    mu = rng.normal(size=(n_blobs, 3))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    s = rng.uniform(0.05, 0.3, n_blobs)
    a = rng.uniform(1.0, 8.0, n_blobs)
    c = rng.uniform(0.2, 1.0, (n_blobs, 3))
    y = dirs[..., 1:2]
    ground = np.array([0.25, 0.22, 0.18])
    horizon = np.array([0.85, 0.85, 0.9])
    zenith = np.array([0.25, 0.45, 0.95])
    up = np.clip(y, 0, 1)
    dn = np.clip(-y, 0, 1)
    col = horizon * (1 - up) * (1 - dn) + zenith * up + ground * dn
    for k in range(n_blobs):
        col = col + a[k] * c[k] * np.exp(-(1.0 - dirs @ mu[k])[..., None] / s[k] ** 2)
    return col


def env_equirect(W: int, H: int, seed: int = 1) -> np.ndarray:
    """[H, W, 3] float32 equirect map point-sampled at texel centres."""
    return sky_radiance(_texel_dirs(W, H), seed).astype(np.float32)


def env_constant(W: int, H: int, rgb=(1.0, 1.0, 1.0)) -> np.ndarray:
    return np.broadcast_to(np.asarray(rgb, np.float32), (H, W, 3)).copy()


def env_mlp_weights(seed: int, n_layers: int = 3, width: int = 64,
                    n_freq: int = 6, in_pad: int = 64):
    """Kaiming-uniform weights of the environment MLP from a seed.

    Input is the 3 + 6*n_freq frequency encoding of a direction, zero-padded
    to `in_pad`; `n_layers` hidden layers of `width` with ReLU; a linear RGB
    head whose bias is 0.5.  Weights are returned as bfloat16-representable
    float32 (rounded to nearest even on the bf16 grid), biases float32.
    Layout: W[l] is [out, in] row-major.
    """
    rng = np.random.default_rng(seed)
    enc = 3 + 6 * n_freq
    dims = [in_pad] + [width] * n_layers + [3]
    Ws, Bs = [], []
    for l in range(n_layers + 1):
        fan_in = enc if l == 0 else dims[l]
        bound = math.sqrt(6.0 / fan_in) if l < n_layers else math.sqrt(3.0 / fan_in)
        Wl = rng.uniform(-bound, bound, size=(dims[l + 1], dims[l]))
        if l == 0:
            Wl[:, enc:] = 0.0
        Bl = rng.uniform(-0.1, 0.1, size=dims[l + 1]) if l < n_layers else np.full(3, 0.5)
        Ws.append(round_to_bf16(Wl.astype(np.float32)))
        Bs.append(Bl.astype(np.float32))
    return Ws, Bs


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------


@dataclass
class Camera:
    """Pinhole camera: eye, look-at target, up hint, vertical FOV (degrees)."""
    eye: tuple
    target: tuple
    up: tuple
    fov_deg: float
    width: int
    height: int

    def as_array(self) -> np.ndarray:
        return np.array(list(self.eye) + list(self.target) + list(self.up)
                        + [self.fov_deg], dtype=np.float64)


def look_at_camera(eye, width: int, height: int, fov_deg: float = 40.0,
                   target=(0.0, 0.0, 0.0)) -> Camera:
    """Object-centred camera; the up hint is +y unless the view is within
    1e-3 of parallel to it, then +z."""
    e = np.asarray(eye, np.float64)
    t = np.asarray(target, np.float64)
    f = (t - e) / np.linalg.norm(t - e)
    up = (0.0, 1.0, 0.0) if abs(f[1]) < 1.0 - 1e-3 else (0.0, 0.0, 1.0)
    return Camera(tuple(e.tolist()), tuple(t.tolist()), up, float(fov_deg), int(width), int(height))


def views_on_sphere(n: int, radius: float = 3.0, seed: int = 0,
                    upper_hemisphere: bool = False) -> np.ndarray:
    """n eye positions uniform on a sphere (or its upper half) of `radius`."""
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(n, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    if upper_hemisphere:
        p[:, 1] = np.abs(p[:, 1])
    return p * radius


# --------------------------------------------------------------------------
# the benchmark workloads (scene + cameras)
# --------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    V: np.ndarray
    F: np.ndarray
    ior: float
    sigma: tuple
    env: np.ndarray | None       # [H,W,3] equirect or None when an MLP is used
    cameras: list
    max_depth: int
    mlp: tuple | None = None     # (Ws, Bs, n_freq)


def icosphere_scene(sigma=(0.0, 0.0, 0.0), res: int = 64) -> Workload:
    """Icosphere r=1 (1,280 tris), IoR 1.5, 64x32 env, eye (0,0,3), FOV 40, depth 4."""
    V, F = icosphere(3)
    env = env_equirect(64, 32, seed=1)
    cam = look_at_camera((0.0, 0.0, 3.0), res, res)
    return Workload("icosphere-1280", V, F, 1.5, tuple(sigma), env, [cam], 4)


def torus_scene(n_views: int = 8, res: int = 512) -> Workload:
    """Displaced torus (102,400 tris), IoR 1.45, sigma 0.3, 512x256 env,
    8 views on a sphere of radius 3 at 512x512, depth 6."""
    V, F = displaced_torus(seed=2)
    env = env_equirect(512, 256, seed=2)
    eyes = views_on_sphere(n_views, 3.0, seed=2)
    cams = [look_at_camera(e, res, res) for e in eyes]
    return Workload("torus-102k", V, F, 1.45, (0.3, 0.3, 0.3), env, cams, 6)


def sdf_union_scene(n_views: int = 8, res: int = 800) -> Workload:
    """Training-step shape: SDF union of 3 tori + 2 spheres (~300k tris, several
    handles), IoR 1.5, sigma (0.5, 0.2, 0.1), 8 views at 800x800, depth 6,
    environment = frequency-encoded MLP 3 x 64 (bf16 weights).  A gradient
    check renders it at other material values against targets at these, so
    that the gradients are nonzero."""
    V, F = sdf_union_faces(300_000, seed=3)
    eyes = views_on_sphere(n_views, 3.0, seed=3)
    cams = [look_at_camera(e, res, res) for e in eyes]
    Ws, Bs = env_mlp_weights(seed=3, n_layers=3, width=64)
    return Workload("sdf-union-300k", V, F, 1.5, (0.5, 0.2, 0.1), None, cams, 6,
                    mlp=(Ws, Bs, 6))


def thin_shell_scene(res: int = 2048) -> Workload:
    """Stress shape: the SDF union turned into a hollow wall |sdf| - 0.01 on a
    360^3 grid (~2M tris, walls ~4 cells thick, frequent total internal
    reflection), IoR 1.5, sigma 0.3, one 2048x2048 view, depth 8, environment
    MLP 4 x 128."""
    V, F = sdf_union_mesh(seed=5, res=360, shell=0.01)
    cams = [look_at_camera(views_on_sphere(1, 3.0, seed=5)[0], res, res)]
    Ws, Bs = env_mlp_weights(seed=5, n_layers=4, width=128)
    return Workload("thin-shell-2M", V, F, 1.5, (0.3, 0.3, 0.3), None, cams, 8, mlp=(Ws, Bs, 6))
