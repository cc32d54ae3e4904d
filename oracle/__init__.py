"""FP64 CPU oracle of the recursive differentiable transparent-mesh tracer.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the HIP library; both consume the same seeded numpy inputs.

The C++ source (oracle.cpp) states what each function computes and which
passage of the paper it follows.  This module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FLAG_DEGEN, FLAG_LEAK, FLAG_GRAZING, FLAG_TIRB, FLAG_TRUNC, FLAG_KINK = 1, 2, 4, 8, 16, 128
TREE_FIELDS = (["depth", "kind", "tri"] + ["o%d" % i for i in range(3)]
               + ["d%d" % i for i in range(3)] + ["W%d" % i for i in range(3)]
               + ["R", "T"] + ["A%d" % i for i in range(3)]
               + ["t", "entering", "tir", "cos_i"] + ["E%d" % i for i in range(3)])


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so (g++, FP64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Env(C.Structure):
    _fields_ = [("kind", C.c_int), ("W", C.c_int), ("H", C.c_int),
                ("tex", C.POINTER(C.c_double)), ("n_freq", C.c_int),
                ("n_layers", C.c_int), ("width", C.c_int), ("in_pad", C.c_int),
                ("weights", C.POINTER(C.c_double)), ("biases", C.POINTER(C.c_double))]


class _Absorption(C.Structure):
    _fields_ = [("mu", C.POINTER(C.c_double)), ("nx", C.c_int), ("ny", C.c_int),
                ("nz", C.c_int), ("samples", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class _Field(C.Structure):
    _fields_ = [("grid", C.POINTER(C.c_double)), ("nx", C.c_int), ("ny", C.c_int),
                ("nz", C.c_int), ("planes", C.POINTER(C.c_double)), ("res", C.c_int),
                ("samples", C.c_int), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class _Scene(C.Structure):
    _fields_ = [("V", C.POINTER(C.c_double)), ("nv", C.c_int),
                ("F", C.POINTER(C.c_int)), ("nf", C.c_int),
                ("eta", C.c_double), ("sigma", C.c_double * 3),
                ("env", C.POINTER(_Env)), ("max_depth", C.c_int),
                ("terminal_env", C.c_int), ("t_eps", C.c_double), ("use_bvh", C.c_int),
                ("absorb", C.POINTER(_Absorption)), ("field", C.POINTER(_Field)),
                ("jitter", C.c_double), ("jitter_seed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp, ip, i64 = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_int64
        L.or_vertex_normals.argtypes = [dp, C.c_int, ip, C.c_int, dp]
        L.or_camera_rays.argtypes = [dp, C.c_int, C.c_int, dp, dp]
        L.or_intersect.argtypes = [C.POINTER(_Scene), dp, dp, ip, i64, ip, dp, dp, dp]
        L.or_env_eval.argtypes = [C.POINTER(_Env), dp, i64, dp]
        L.or_env_eval_grad.argtypes = [C.POINTER(_Env), dp, i64, dp, dp]
        L.or_env_kink_margin.argtypes = [C.POINTER(_Env), dp, i64, dp]
        L.or_trace.argtypes = [C.POINTER(_Scene), dp, dp, i64, dp, dp, ip,
                               C.POINTER(C.c_uint64), ip, C.POINTER(C.c_uint64)]
        L.or_trace_grad.argtypes = [C.POINTER(_Scene), dp, dp, i64, dp, dp, dp, dp, dp, dp, dp, dp,
                                    dp, C.c_int]
        L.or_trace_tree.argtypes = [C.POINTER(_Scene), dp, dp, dp, C.c_int]
        L.or_trace_errbound.argtypes = [C.POINTER(_Scene), dp, dp, i64, dp, dp]
        L.or_mask.argtypes = [C.POINTER(_Scene), dp, C.c_int, C.c_int, dp]
        L.or_mask_grad.argtypes = [C.POINTER(_Scene), dp, C.c_int, C.c_int, dp, C.c_double, dp,
                                   C.POINTER(C.c_int64)]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


class Env:
    """Equirect map [H,W,3] or MLP (weights list [out,in], biases list, n_freq),
    evaluated in plain FP64."""

    def __init__(self, tex=None, mlp=None):
        self._keep = []
        self.tex = None
        self.mlp_shapes = None
        s = _Env()
        if tex is not None:
            t = _d(tex)
            self.tex = t
            self._keep.append(t)
            s.kind, s.H, s.W = 0, t.shape[0], t.shape[1]
            s.tex = _p(t)
        else:
            Ws, Bs, n_freq = mlp
            w = _d(np.concatenate([np.asarray(x, np.float64).ravel() for x in Ws]))
            b = _d(np.concatenate([np.asarray(x, np.float64).ravel() for x in Bs]))
            self._keep += [w, b]
            self.mlp_shapes = [(np.asarray(x).shape, np.asarray(y).shape) for x, y in zip(Ws, Bs)]
            self.n_weights, self.n_params = w.size, w.size + b.size
            s.kind = 1
            s.n_freq = n_freq
            s.n_layers = len(Ws) - 1
            s.width = Ws[0].shape[0]
            s.in_pad = Ws[0].shape[1]
            s.weights, s.biases = _p(w), _p(b)
        self.s = s

    def split_params(self, flat):
        """Flat MLP parameter vector (every weight, then every bias) ->
        (list of weight matrices [out, in], list of bias vectors)."""
        Ws, Bs, k = [], [], 0
        for ws, _ in self.mlp_shapes:
            n = int(np.prod(ws))
            Ws.append(flat[k:k + n].reshape(ws))
            k += n
        for _, bs in self.mlp_shapes:
            n = int(np.prod(bs))
            Bs.append(flat[k:k + n].reshape(bs))
            k += n
        return Ws, Bs

    def eval(self, dirs):
        d = _d(dirs).reshape(-1, 3)
        out = np.empty_like(d)
        assert lib().or_env_eval(C.byref(self.s), _p(d), len(d), _p(out)) == 0
        return out

    def kink_margin(self, dirs):
        """Angular distance (rad) to the nearest gradient discontinuity."""
        d = _d(dirs).reshape(-1, 3)
        out = np.empty(len(d))
        assert lib().or_env_kink_margin(C.byref(self.s), _p(d), len(d), _p(out)) == 0
        return out

    def eval_grad(self, dirs, grad_rgb):
        d = _d(dirs).reshape(-1, 3)
        g = _d(grad_rgb).reshape(-1, 3)
        out = np.empty_like(d)
        assert lib().or_env_eval_grad(C.byref(self.s), _p(d), len(d), _p(g), _p(out)) == 0
        return out


class Absorption:
    """Spatially varying absorption rate: an RGB grid mu [nz, ny, nx, 3] over the
    box [lo, hi], trilinear, S midpoint samples per interior segment."""

    def __init__(self, mu, lo, hi, samples: int):
        self.mu = _d(mu)
        assert self.mu.ndim == 4 and self.mu.shape[3] == 3
        self.lo = np.asarray(lo, np.float64).reshape(3)
        self.hi = np.asarray(hi, np.float64).reshape(3)
        self.samples = int(samples)
        nz, ny, nx, _ = self.mu.shape
        self.s = _Absorption()
        self.s.mu = _p(self.mu)
        self.s.nx, self.s.ny, self.s.nz, self.s.samples = nx, ny, nz, self.samples
        for k in range(3):
            self.s.lo[k], self.s.hi[k] = float(self.lo[k]), float(self.hi[k])


class Field:
    """Volumetric environment field outside the object: a dense grid
    [nz, ny, nx, 4] and three planes [3, res, res, 4] over the box [lo, hi]
    (channel 0 -> density by softplus, 1-3 -> RGB), S midpoint samples per
    exterior segment."""

    def __init__(self, grid, planes, lo, hi, samples: int):
        self.grid, self.planes = _d(grid), _d(planes)
        assert self.grid.ndim == 4 and self.grid.shape[3] == 4
        assert self.planes.ndim == 4 and self.planes.shape[0] == 3 and self.planes.shape[3] == 4
        assert self.planes.shape[1] == self.planes.shape[2]
        self.lo = np.asarray(lo, np.float64).reshape(3)
        self.hi = np.asarray(hi, np.float64).reshape(3)
        self.samples = int(samples)
        nz, ny, nx, _ = self.grid.shape
        self.s = _Field()
        self.s.grid, self.s.nx, self.s.ny, self.s.nz = _p(self.grid), nx, ny, nz
        self.s.planes, self.s.res, self.s.samples = _p(self.planes), self.planes.shape[1], self.samples
        for k in range(3):
            self.s.lo[k], self.s.hi[k] = float(self.lo[k]), float(self.hi[k])

    @property
    def n_params(self):
        return self.grid.size + self.planes.size

    def split(self, flat):
        """Flat parameter vector -> (grid-shaped, planes-shaped) arrays."""
        return flat[:self.grid.size].reshape(self.grid.shape), flat[self.grid.size:].reshape(self.planes.shape)


class Scene:
    """Mesh + material + environment + tracing parameters for the oracle."""

    def __init__(self, V, F, eta, sigma, env: Env, max_depth: int,
                 terminal_env: bool = False, t_eps: float = 1e-5, use_bvh: bool = True,
                 absorb: "Absorption | None" = None, field: "Field | None" = None):
        self.V = _d(V).reshape(-1, 3)
        self.F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
        self.env = env
        self.eta = float(eta)
        sg = np.broadcast_to(np.asarray(sigma, np.float64), (3,))
        self.sigma = sg.copy()
        self.max_depth = int(max_depth)
        self.terminal_env = bool(terminal_env)
        self.t_eps = float(t_eps)
        self.use_bvh = bool(use_bvh)
        self.absorb = absorb
        self.field = field
        # test instrument (0 = off): every ray the tracer starts is scaled per
        # component by (1 + jitter xi), xi uniform in [-1, 1), seeded
        self.jitter = 0.0
        self.jitter_seed = 0

    def _s(self):
        s = _Scene()
        s.V, s.nv = _p(self.V), len(self.V)
        s.F, s.nf = _p(self.F, C.c_int), len(self.F)
        s.eta = self.eta
        for k in range(3):
            s.sigma[k] = float(self.sigma[k])
        s.env = C.pointer(self.env.s)
        s.max_depth = self.max_depth
        s.terminal_env = int(self.terminal_env)
        s.t_eps = self.t_eps
        s.use_bvh = int(self.use_bvh)
        s.absorb = C.pointer(self.absorb.s) if self.absorb is not None else None
        s.field = C.pointer(self.field.s) if self.field is not None else None
        s.jitter, s.jitter_seed = float(self.jitter), int(self.jitter_seed)
        return s

    def with_(self, **kw):
        sc = Scene(self.V, self.F, self.eta, self.sigma, self.env, self.max_depth,
                   self.terminal_env, self.t_eps, self.use_bvh, self.absorb, self.field)
        sc.jitter, sc.jitter_seed = self.jitter, self.jitter_seed
        for k, v in kw.items():
            if k == "V":
                v = _d(v).reshape(-1, 3)
            if k == "sigma":
                v = np.broadcast_to(np.asarray(v, np.float64), (3,)).copy()
            setattr(sc, k, v)
        return sc

    def trace(self, o, d):
        """Returns dict(rgb [n,3], wtrunc [n,3], flags [n], hash [n], nseg [n],
        sig [n]).  hash: ordered hash of the depth-first visit (triangles,
        branches, texel cells); sig: order-independent path signature, the
        sum mod 2^64 of splitmix64((g << 40) | (tir << 32) | (tri + 1)) over
        the tree's segments (tri = -1 for a miss, tir = 0 when truncated)."""
        o, d = _d(o).reshape(-1, 3), _d(d).reshape(-1, 3)
        n = len(o)
        rgb, wt = np.empty((n, 3)), np.empty((n, 3))
        fl, ns = np.empty(n, np.int32), np.empty(n, np.int32)
        hs, sg = np.empty(n, np.uint64), np.empty(n, np.uint64)
        s = self._s()
        rc = lib().or_trace(C.byref(s), _p(o), _p(d), n, _p(rgb), _p(wt), _p(fl, C.c_int),
                            _p(hs, C.c_uint64), _p(ns, C.c_int), _p(sg, C.c_uint64))
        assert rc == 0, "or_trace rejected its arguments"
        return {"rgb": rgb, "wtrunc": wt, "flags": fl, "hash": hs, "nseg": ns, "sig": sg}

    def trace_grad(self, o, d, grad_rgb, want_tex: bool = False, want_mlp: bool = False,
                   absolute: bool = False):
        """Returns dict(rgb, dV [nv,3], d_eta, d_sigma [3], d_mu [nz,ny,nx,3] or None,
        d_tex [H,W,3] (equirect environment, with want_tex) or None, d_mlp
        (MLP environment, with want_mlp: (weight gradients [out, in] per
        layer, bias gradients per layer)) or None).  absolute: every gradient
        is instead the sum over camera rays of the magnitude of each ray's
        contribution."""
        o, d = _d(o).reshape(-1, 3), _d(d).reshape(-1, 3)
        g = _d(grad_rgb).reshape(-1, 3)
        n = len(o)
        rgb = np.empty((n, 3))
        dV = np.empty_like(self.V)
        de = np.zeros(1)
        ds = np.zeros(3)
        dm = np.zeros_like(self.absorb.mu) if self.absorb is not None else None
        dt = np.zeros_like(self.env.tex) if want_tex and self.env.tex is not None else None
        dw = np.zeros(self.env.n_params) if want_mlp and self.env.mlp_shapes else None
        df = np.zeros(self.field.n_params) if self.field is not None else None
        s = self._s()
        rc = lib().or_trace_grad(C.byref(s), _p(o), _p(d), n, _p(g), _p(rgb), _p(dV),
                                 _p(de), _p(ds), _p(dm) if dm is not None else None,
                                 _p(dt) if dt is not None else None,
                                 _p(dw) if dw is not None else None,
                                 _p(df) if df is not None else None, int(bool(absolute)))
        assert rc == 0, "or_trace_grad rejected its arguments"
        return {"rgb": rgb, "dV": dV, "d_eta": float(de[0]), "d_sigma": ds, "d_mu": dm,
                "d_tex": dt, "d_mlp": self.env.split_params(dw) if dw is not None else None,
                "d_field": self.field.split(df) if df is not None else None}

    def errbound(self, o, d):
        """First-order bound on the rounding error of an FP32 evaluation of
        each pixel's radiance, per channel [n, 3] (with the FP64 rgb [n, 3])."""
        o, d = _d(o).reshape(-1, 3), _d(d).reshape(-1, 3)
        n = len(o)
        rgb, b = np.empty((n, 3)), np.empty((n, 3))
        s = self._s()
        assert lib().or_trace_errbound(C.byref(s), _p(o), _p(d), n, _p(rgb), _p(b)) == 0
        return rgb, b

    def mask(self, cam):
        """Centre-sample coverage [H*W] of one camera (1 = the pixel centre's
        ray hits the mesh)."""
        a = _d(cam.as_array())
        out = np.empty(cam.width * cam.height)
        s = self._s()
        assert lib().or_mask(C.byref(s), _p(a), cam.width, cam.height, _p(out)) == 0
        return out

    def mask_grad(self, cam, grad_mask, rho: float = 2.0):
        """Gradient of sum_p grad_mask[p] M_p with respect to the vertices
        [nv, 3] through the motion of the outline (quadrature at rho points
        per pixel of projected edge length); also (points in the image,
        points on the outline)."""
        a = _d(cam.as_array())
        g = _d(grad_mask).reshape(-1)
        assert g.size == cam.width * cam.height
        dV = np.empty_like(self.V)
        cnt = np.zeros(2, np.int64)
        s = self._s()
        assert lib().or_mask_grad(C.byref(s), _p(a), cam.width, cam.height, _p(g), float(rho),
                                  _p(dV), _p(cnt, C.c_int64)) == 0
        return dV, (int(cnt[0]), int(cnt[1]))

    def tree(self, o, d, max_rec: int = 4096):
        """Depth-first node records of one camera ray (list of dicts)."""
        o, d = _d(o).reshape(3), _d(d).reshape(3)
        nd = len(TREE_FIELDS)
        out = np.zeros((max_rec, nd))
        s = self._s()
        k = lib().or_trace_tree(C.byref(s), _p(o), _p(d), _p(out), max_rec)
        assert k >= 0
        return [dict(zip(TREE_FIELDS, row)) for row in out[:min(k, max_rec)]]

    def intersect(self, o, d, skip=None):
        o, d = _d(o).reshape(-1, 3), _d(d).reshape(-1, 3)
        n = len(o)
        tri = np.empty(n, np.int32)
        t, b1, b2 = np.empty(n), np.empty(n), np.empty(n)
        sk = None if skip is None else np.ascontiguousarray(skip, np.int32)
        s = self._s()
        rc = lib().or_intersect(C.byref(s), _p(o), _p(d),
                                None if sk is None else _p(sk, C.c_int), n,
                                _p(tri, C.c_int), _p(t), _p(b1), _p(b2))
        assert rc == 0
        return tri, t, b1, b2


def vertex_normals(V, F):
    V = _d(V).reshape(-1, 3)
    F = np.ascontiguousarray(F, np.int32).reshape(-1, 3)
    N = np.empty_like(V)
    assert lib().or_vertex_normals(_p(V), len(V), _p(F, C.c_int), len(F), _p(N)) == 0
    return N


def camera_rays(cam):
    """Camera (synth.Camera) -> o, d arrays [H*W,3], pixel index y*W + x."""
    a = _d(cam.as_array())
    n = cam.width * cam.height
    o, d = np.empty((n, 3)), np.empty((n, 3))
    assert lib().or_camera_rays(_p(a), cam.width, cam.height, _p(o), _p(d)) == 0
    return o, d


def num_threads() -> int:
    return int(lib().or_num_threads())


def assert_tree_record_size():
    assert lib().or_tree_record_doubles() == len(TREE_FIELDS)
