"""ctypes binding of libdifftrans.so (argument marshalling only).

Every compute step runs in the HIP library; this module converts torch
tensors (device memory, owned by the caller) into pointers, passes the current
HIP stream, and turns non-OK status codes into exceptions.  The functions
keep the C entry points' names.  Buffers the library needs (BVH blob,
workspace, tape) are sized with the *_bytes queries and allocated here with
torch, because the library itself never allocates.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdifftrans.so")

DT_OK = 0
(DT_ERR_INVALID_ARGUMENT, DT_ERR_WORKSPACE_TOO_SMALL, DT_ERR_CAPACITY, DT_ERR_HIP, DT_ERR_UNSUPPORTED,
 DT_ERR_NOT_CONVERGED) = 1, 2, 3, 4, 5, 6
FLAG_DEGEN, FLAG_LEAK, FLAG_GRAZING, FLAG_TIRB, FLAG_TRUNC, FLAG_OVERFLOW, FLAG_STACK = \
    1, 2, 4, 8, 16, 32, 64
MAX_DEPTH = 16
STATS_LEN = 64
STAT_HITS = 17
STAT_TOTAL, STAT_DROPPED, STAT_GENERATIONS, STAT_BVH_DEPTH, STAT_TOTAL_HITS = 48, 49, 50, 51, 52
ENV_EQUIRECT, ENV_MLP = 0, 1
RAYS_EXPLICIT, RAYS_CAMERAS = 0, 1


class DTError(RuntimeError):
    pass


class _Env(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("texels", C.c_void_p), ("n_freq", C.c_int32), ("n_layers", C.c_int32),
                ("hidden", C.c_int32), ("in_pad", C.c_int32), ("weights", C.c_void_p),
                ("biases", C.c_void_p), ("d_texels", C.c_void_p), ("d_weights", C.c_void_p),
                ("d_biases", C.c_void_p)]


class _Absorption(C.Structure):
    _fields_ = [("mu", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("samples", C.c_int32), ("lo", C.c_float * 3), ("hi", C.c_float * 3),
                ("d_mu", C.c_void_p)]


class _Field(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("planes", C.c_void_p), ("res", C.c_int32), ("samples", C.c_int32),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("d_grid", C.c_void_p),
                ("d_planes", C.c_void_p)]


class _Scene(C.Structure):
    _fields_ = [("V", C.c_void_p), ("nv", C.c_int32), ("F", C.c_void_p), ("nf", C.c_int32),
                ("bvh", C.c_void_p), ("ior", C.c_void_p), ("sigma", C.c_void_p),
                ("env", C.POINTER(_Env)), ("absorb", C.POINTER(_Absorption)),
                ("field", C.POINTER(_Field))]


class _Timing(C.Structure):
    _fields_ = [("trace_events", C.POINTER(C.c_void_p)), ("adjoint_events", C.POINTER(C.c_void_p)),
                ("mlp_events", C.POINTER(C.c_void_p)), ("mlp_adjoint_events", C.POINTER(C.c_void_p))]


class _Params(C.Structure):
    _fields_ = [("max_depth", C.c_int32), ("terminal_env", C.c_int32), ("t_eps", C.c_float),
                ("checkpoint_stride", C.c_int32), ("queue_capacity", C.c_int64),
                ("timing", C.POINTER(_Timing))]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("pixel_offset", C.c_int64)]


class _Rays(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("o", C.c_void_p), ("d", C.c_void_p),
                ("n_cameras", C.c_int32), ("cameras", C.POINTER(_Camera)), ("n_pixels", C.c_int64)]


_lib = None
EXPORTS = ["dt_bvh_bytes", "dt_build_bvh", "dt_build_bvh_noalloc", "dt_bvh_vertex_normals", "dt_env_query",
           "dt_env_query_backward", "dt_trace_bytes", "dt_trace_forward", "dt_trace_backward",
           "dt_intersect", "dt_mask_bytes", "dt_mask_forward", "dt_mask_backward",
           "dt_smooth_bytes", "dt_smooth_solve", "dt_status_string", "dt_last_error"]


def load(path: str = LIB_PATH):
    """Open the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DTError(f"{path} is missing: build it with paper_2603_00413_amd/csrc/build.py "
                      "(there is no fallback path)")
    L = C.CDLL(path)
    vp, sz, i32, i64 = C.c_void_p, C.POINTER(C.c_size_t), C.c_int32, C.c_int64
    L.dt_bvh_bytes.argtypes = [i32, i32, sz, sz]
    L.dt_build_bvh.argtypes = [vp, i32, vp, i32, vp, C.c_size_t, vp, C.c_size_t, vp]
    L.dt_build_bvh_noalloc.argtypes = [vp, i32, vp, i32, vp, C.c_size_t, vp]
    L.dt_bvh_vertex_normals.argtypes = [vp, i32, i32, vp, vp]
    L.dt_env_query.argtypes = [C.POINTER(_Env), vp, i64, vp, vp]
    L.dt_env_query_backward.argtypes = [C.POINTER(_Env), vp, i64, vp, vp, vp]
    L.dt_trace_bytes.argtypes = [C.POINTER(_Params), i64, i32, i32, sz, sz]
    L.dt_trace_forward.argtypes = [C.POINTER(_Scene), C.POINTER(_Rays), C.POINTER(_Params), vp, vp,
                                   vp, vp, vp, vp, C.c_size_t, vp, C.c_size_t, vp]
    L.dt_trace_backward.argtypes = [C.POINTER(_Scene), C.POINTER(_Rays), C.POINTER(_Params), vp, vp,
                                    C.c_size_t, vp, vp, vp, vp, C.c_size_t, vp]
    L.dt_intersect.argtypes = [C.POINTER(_Scene), vp, vp, vp, i64, C.c_float, i32, vp, vp, vp, vp]
    L.dt_mask_bytes.argtypes = [i32, i32, sz]
    L.dt_mask_forward.argtypes = [C.POINTER(_Scene), C.POINTER(_Rays), C.c_float, vp, vp]
    L.dt_mask_backward.argtypes = [C.POINTER(_Scene), C.POINTER(_Rays), vp, C.c_float, vp, vp, vp,
                                   C.c_size_t, vp]
    L.dt_smooth_bytes.argtypes = [i32, sz]
    L.dt_smooth_solve.argtypes = [vp, vp, i32, C.c_double, vp, vp, C.c_double, i32, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_double), vp, C.c_size_t, vp]
    L.dt_status_string.argtypes = [i32]
    L.dt_status_string.restype = C.c_char_p
    L.dt_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if not hasattr(L, name):
            raise DTError(f"{path} does not export {name}")
    _lib = L
    return L


def _check(st: int):
    if st != DT_OK:
        L = load()
        raise DTError(f"{L.dt_status_string(st).decode()}: {L.dt_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_check(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise DTError("the HIP library takes device tensors only")
        if t is not None and not t.is_contiguous():
            raise DTError("tensors must be contiguous")


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ mesh
def dt_bvh_bytes(nv: int, nf: int):
    a, b = C.c_size_t(), C.c_size_t()
    _check(load().dt_bvh_bytes(nv, nf, C.byref(a), C.byref(b)))
    return a.value, b.value


class Mesh:
    """Device mesh + its acceleration blob.  `build()` re-runs the device
    build (normals + LBVH) after V changes."""

    def __init__(self, V: torch.Tensor, F: torch.Tensor):
        _dev_check(V, F)
        assert V.dtype == torch.float32 and F.dtype == torch.int32
        self.V, self.F = V, F
        self.nv, self.nf = V.shape[0], F.shape[0]
        nb, nw = dt_bvh_bytes(self.nv, self.nf)
        self.blob = _bytes(nb, V.device)
        self.ws = _bytes(nw, V.device)
        self.build()

    def build(self):
        dt_build_bvh(self.V, self.F, self.blob, self.ws)
        return self

    def vertex_normals(self) -> torch.Tensor:
        N = torch.empty_like(self.V)
        _check(load().dt_bvh_vertex_normals(_ptr(self.blob), self.nv, self.nf, _ptr(N),
                                            _stream(self.V.device)))
        return N


def dt_build_bvh(V, F, blob, ws):
    _dev_check(V, F, blob, ws)
    _check(load().dt_build_bvh(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(blob), blob.numel(),
                               _ptr(ws), ws.numel(), _stream(V.device)))


def dt_build_bvh_noalloc(V, F, blob):
    """dt_build_bvh with the library's own per-device build array as its
    workspace: nothing is allocated (meshes up to DT_BVH_SCRATCH_BYTES of
    build workspace, about 500k faces)."""
    _dev_check(V, F, blob)
    _check(load().dt_build_bvh_noalloc(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(blob),
                                       blob.numel(), _stream(V.device)))


# ------------------------------------------------------------------ environment
class Env:
    """Environment on the device: an equirect map [H, W, 3] float32, or (via
    Env.mlp) a frequency-encoded MLP with bfloat16 weights.  With want_grad,
    d_texels ([H, W, 3]) receives dLoss/dtexel from dt_trace_backward."""

    def __init__(self, texels: torch.Tensor = None, want_grad: bool = False):
        s = _Env()
        self.d_texels = None
        if texels is not None:
            _dev_check(texels)
            assert texels.dtype == torch.float32 and texels.dim() == 3 and texels.shape[2] == 3
            self.texels = texels
            s.kind = ENV_EQUIRECT
            s.height, s.width = texels.shape[0], texels.shape[1]
            s.texels = texels.data_ptr()
            if want_grad:
                self.d_texels = torch.zeros_like(texels)
                s.d_texels = self.d_texels.data_ptr()
        self.s = s

    @staticmethod
    def mlp(Ws, Bs, n_freq: int, device, want_grad: bool = False) -> "Env":
        """Ws: per-layer [out, in] weights (bf16-representable), Bs: biases;
        hidden layers of equal width, last layer [3, width], first [width, 64].
        want_grad: the backward also writes d_weights / d_biases (float32,
        flat in the same layout; `split_grad` returns them per layer)."""
        e = Env()
        w = torch.cat([torch.as_tensor(x, dtype=torch.float32).reshape(-1) for x in Ws])
        e.weights = w.to(torch.bfloat16).view(torch.int16).to(device).contiguous()
        e.biases = torch.cat([torch.as_tensor(x, dtype=torch.float32).reshape(-1)
                              for x in Bs]).to(device).contiguous()
        e.shapes = [(tuple(np.shape(x)), tuple(np.shape(y))) for x, y in zip(Ws, Bs)]
        s = e.s
        s.kind = ENV_MLP
        s.n_freq, s.n_layers = int(n_freq), len(Ws) - 1
        s.hidden, s.in_pad = int(Ws[0].shape[0]), int(Ws[0].shape[1])
        s.weights, s.biases = e.weights.data_ptr(), e.biases.data_ptr()
        if want_grad:
            e.d_weights = torch.zeros(e.weights.numel(), dtype=torch.float32, device=device)
            e.d_biases = torch.zeros_like(e.biases)
            s.d_weights, s.d_biases = e.d_weights.data_ptr(), e.d_biases.data_ptr()
        return e

    def split_grad(self):
        """(list of weight gradients [out, in], list of bias gradients) as
        numpy arrays, from the last backward."""
        w = self.d_weights.cpu().numpy()
        b = self.d_biases.cpu().numpy()
        Wg, Bg, kw, kb = [], [], 0, 0
        for ws, bs in self.shapes:
            nw, nb = int(np.prod(ws)), int(np.prod(bs))
            Wg.append(w[kw:kw + nw].reshape(ws))
            Bg.append(b[kb:kb + nb].reshape(bs))
            kw += nw
            kb += nb
        return Wg, Bg


def dt_env_query(env: Env, dirs: torch.Tensor) -> torch.Tensor:
    _dev_check(dirs)
    out = torch.empty_like(dirs)
    _check(load().dt_env_query(C.byref(env.s), _ptr(dirs), dirs.shape[0], _ptr(out),
                               _stream(dirs.device)))
    return out


def dt_env_query_backward(env: Env, dirs: torch.Tensor, grad_rgb: torch.Tensor) -> torch.Tensor:
    _dev_check(dirs, grad_rgb)
    out = torch.empty_like(dirs)
    _check(load().dt_env_query_backward(C.byref(env.s), _ptr(dirs), dirs.shape[0], _ptr(grad_rgb),
                                        _ptr(out), _stream(dirs.device)))
    return out


# ------------------------------------------------------------------ tracing
@dataclass
class Params:
    max_depth: int = 4
    terminal_env: bool = False
    t_eps: float = 1e-5
    checkpoint_stride: int = 1
    queue_capacity: int = 0
    timing: object = None   # KernelTimer or None

    def c(self) -> _Params:
        p = _Params()
        p.max_depth, p.terminal_env, p.t_eps = self.max_depth, int(self.terminal_env), self.t_eps
        p.checkpoint_stride, p.queue_capacity = self.checkpoint_stride, int(self.queue_capacity)
        if self.timing is not None:
            p.timing = C.pointer(self.timing.s)
        return p


class KernelTimer:
    """hipEvent pairs the library records around its traversal, adjoint and
    environment-MLP kernels (one pair per generation), read back as
    milliseconds."""

    def __init__(self, max_depth: int):
        # the HIP runtime the library itself is bound to (dlsym searches the
        # library's dependencies), so events and streams share one runtime
        self.hip = load()
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        n = 2 * (max_depth + 1)
        self.n = n
        self.trace = (C.c_void_p * n)()
        self.adjoint = (C.c_void_p * n)()
        self.mlp = (C.c_void_p * n)()
        self.mlp_adjoint = (C.c_void_p * n)()
        for arr in (self.trace, self.adjoint, self.mlp, self.mlp_adjoint):
            for i in range(n):
                ev = C.c_void_p()
                if self.hip.hipEventCreate(C.byref(ev)) != 0:
                    raise DTError("hipEventCreate failed")
                arr[i] = ev
        self.s = _Timing()
        self.s.trace_events = C.cast(self.trace, C.POINTER(C.c_void_p))
        self.s.adjoint_events = C.cast(self.adjoint, C.POINTER(C.c_void_p))
        self.s.mlp_events = C.cast(self.mlp, C.POINTER(C.c_void_p))
        self.s.mlp_adjoint_events = C.cast(self.mlp_adjoint, C.POINTER(C.c_void_p))

    def _ms(self, arr, g):
        self.hip.hipEventSynchronize(arr[2 * g + 1])
        ms = C.c_float()
        if self.hip.hipEventElapsedTime(C.byref(ms), arr[2 * g], arr[2 * g + 1]) != 0:
            return float("nan")
        return ms.value

    def trace_ms(self, gens: int):
        return [self._ms(self.trace, g) for g in range(gens)]

    def adjoint_ms(self, gens: int):
        return [self._ms(self.adjoint, g) for g in range(gens)]

    def mlp_ms(self, gens: int):
        return [self._ms(self.mlp, g) for g in range(gens)]

    def mlp_adjoint_ms(self, gens: int):
        return [self._ms(self.mlp_adjoint, g) for g in range(gens)]


class Rays:
    """Explicit rays (o, d device [n,3]) or a list of synth.Camera-like objects."""

    def __init__(self, o=None, d=None, cameras=None):
        self._keep = []
        r = _Rays()
        if cameras is None:
            _dev_check(o, d)
            r.kind, r.n, r.o, r.d = RAYS_EXPLICIT, o.shape[0], o.data_ptr(), d.data_ptr()
            self.n_rays = self.n_pixels = o.shape[0]
            self._keep += [o, d]
        else:
            arr = (_Camera * len(cameras))()
            off = 0
            for i, c in enumerate(cameras):
                for k in range(3):
                    arr[i].eye[k], arr[i].target[k], arr[i].up[k] = c.eye[k], c.target[k], c.up[k]
                arr[i].fov_deg, arr[i].width, arr[i].height = c.fov_deg, c.width, c.height
                arr[i].pixel_offset = off
                off += c.width * c.height
            self._keep.append(arr)
            r.kind, r.n_cameras, r.cameras, r.n_pixels = RAYS_CAMERAS, len(cameras), arr, off
            self.n_rays = self.n_pixels = off
        self.s = r


class Absorption:
    """Spatially varying absorption rate: device float32 grid mu [nz, ny, nx, 3]
    over the box [lo, hi], trilinear, `samples` midpoint samples per interior
    segment.  d_mu (same shape) receives dLoss/dmu from dt_trace_backward."""

    def __init__(self, mu: torch.Tensor, lo, hi, samples: int, want_grad: bool = True):
        _dev_check(mu)
        assert mu.dtype == torch.float32 and mu.dim() == 4 and mu.shape[3] == 3
        self.mu = mu.contiguous()
        self.lo, self.hi, self.samples = tuple(map(float, lo)), tuple(map(float, hi)), int(samples)
        self.d_mu = torch.zeros_like(self.mu) if want_grad else None
        nz, ny, nx, _ = self.mu.shape
        self.s = _Absorption()
        self.s.mu, self.s.nx, self.s.ny, self.s.nz = self.mu.data_ptr(), nx, ny, nz
        self.s.samples = self.samples
        for k in range(3):
            self.s.lo[k], self.s.hi[k] = self.lo[k], self.hi[k]
        self.s.d_mu = self.d_mu.data_ptr() if self.d_mu is not None else None


class Field:
    """Volumetric environment field outside the object: device float32 grid
    [nz, ny, nx, 4] plus three planes [3, res, res, 4] over the box [lo, hi]
    (channel 0 -> density by softplus, 1-3 -> colour), `samples` midpoint
    samples per exterior segment.  d_grid / d_planes (same shapes) receive
    dLoss/d(grid, planes) from dt_trace_backward."""

    def __init__(self, grid: torch.Tensor, planes: torch.Tensor, lo, hi, samples: int,
                 want_grad: bool = True):
        _dev_check(grid, planes)
        assert grid.dtype == torch.float32 and grid.dim() == 4 and grid.shape[3] == 4
        assert planes.dtype == torch.float32 and planes.dim() == 4 and planes.shape[0] == 3
        assert planes.shape[1] == planes.shape[2] and planes.shape[3] == 4
        self.grid, self.planes = grid.contiguous(), planes.contiguous()
        self.lo, self.hi, self.samples = tuple(map(float, lo)), tuple(map(float, hi)), int(samples)
        self.d_grid = torch.zeros_like(self.grid) if want_grad else None
        self.d_planes = torch.zeros_like(self.planes) if want_grad else None
        nz, ny, nx, _ = self.grid.shape
        self.s = _Field()
        self.s.grid, self.s.nx, self.s.ny, self.s.nz = self.grid.data_ptr(), nx, ny, nz
        self.s.planes, self.s.res, self.s.samples = self.planes.data_ptr(), self.planes.shape[1], self.samples
        for k in range(3):
            self.s.lo[k], self.s.hi[k] = self.lo[k], self.hi[k]
        self.s.d_grid = self.d_grid.data_ptr() if want_grad else None
        self.s.d_planes = self.d_planes.data_ptr() if want_grad else None


class Scene:
    """Mesh + device IoR [1] + device sigma [3] + environment (+ optional
    absorption grid, which replaces sigma on interior segments, + optional
    volumetric field sampled along exterior segments)."""

    def __init__(self, mesh: Mesh, ior: torch.Tensor, sigma: torch.Tensor, env: Env,
                 absorb: Absorption | None = None, field: Field | None = None):
        _dev_check(ior, sigma)
        self.mesh, self.ior, self.sigma, self.env, self.absorb = mesh, ior, sigma, env, absorb
        self.field = field

    def c(self) -> _Scene:
        s = _Scene()
        m = self.mesh
        s.V, s.nv, s.F, s.nf = m.V.data_ptr(), m.nv, m.F.data_ptr(), m.nf
        s.bvh, s.ior, s.sigma = m.blob.data_ptr(), self.ior.data_ptr(), self.sigma.data_ptr()
        s.env = C.pointer(self.env.s)
        s.absorb = C.pointer(self.absorb.s) if self.absorb is not None else None
        s.field = C.pointer(self.field.s) if self.field is not None else None
        return s


def dt_trace_bytes(params: Params, n_rays: int, nv: int, nf: int):
    a, b = C.c_size_t(), C.c_size_t()
    _check(load().dt_trace_bytes(C.byref(params.c()), n_rays, nv, nf, C.byref(a), C.byref(b)))
    return a.value, b.value


class Buffers:
    """Workspace + tape sized for (params, rays, mesh); reusable across calls."""

    def __init__(self, params: Params, rays: Rays, mesh: Mesh, tape: bool):
        self.ws_bytes, self.tape_bytes = dt_trace_bytes(params, rays.n_rays, mesh.nv, mesh.nf)
        dev = mesh.V.device
        self.ws = _bytes(self.ws_bytes, dev)
        self.tape = _bytes(self.tape_bytes, dev) if tape else None
        self.stats = torch.zeros(STATS_LEN, dtype=torch.int64, device=dev)


def dt_trace_forward(scene: Scene, rays: Rays, params: Params, buf: Buffers,
                     want_aux: bool = True, path_sig: torch.Tensor | None = None):
    """Returns (rgb [npix,3], wtrunc [npix,3] or None, flags [npix] or None).
    path_sig: optional int64 [npix] device tensor that receives each pixel's
    path signature (the bits of the unsigned 64-bit value)."""
    dev = scene.mesh.V.device
    npix = rays.n_pixels
    rgb = torch.empty(npix, 3, dtype=torch.float32, device=dev)
    wtrunc = torch.empty(npix, 3, dtype=torch.float32, device=dev) if want_aux else None
    flags = torch.empty(npix, dtype=torch.int32, device=dev) if want_aux else None
    if path_sig is not None:
        _dev_check(path_sig)
        if path_sig.dtype != torch.int64 or path_sig.numel() != npix:
            raise DTError("path_sig must be an int64 tensor of n_pixels elements")
    sc, p = scene.c(), params.c()
    tape = buf.tape
    _check(load().dt_trace_forward(C.byref(sc), C.byref(rays.s), C.byref(p), _ptr(rgb), _ptr(wtrunc),
                                   _ptr(flags), _ptr(path_sig), _ptr(buf.stats), _ptr(tape),
                                   0 if tape is None else tape.numel(), _ptr(buf.ws), buf.ws.numel(),
                                   _stream(dev)))
    return rgb, wtrunc, flags


def dt_trace_backward(scene: Scene, rays: Rays, params: Params, buf: Buffers,
                      grad_rgb: torch.Tensor):
    """Returns (dV [nv,3], d_ior [1], d_sigma [3]) for the last forward on buf."""
    if buf.tape is None:
        raise DTError("the forward pass was run without a tape")
    _dev_check(grad_rgb)
    dev = scene.mesh.V.device
    dV = torch.empty(scene.mesh.nv, 3, dtype=torch.float32, device=dev)
    d_ior = torch.empty(1, dtype=torch.float32, device=dev)
    d_sigma = torch.empty(3, dtype=torch.float32, device=dev)
    sc, p = scene.c(), params.c()
    _check(load().dt_trace_backward(C.byref(sc), C.byref(rays.s), C.byref(p), _ptr(grad_rgb),
                                    _ptr(buf.tape), buf.tape.numel(), _ptr(dV), _ptr(d_ior),
                                    _ptr(d_sigma), _ptr(buf.ws), buf.ws.numel(), _stream(dev)))
    return dV, d_ior, d_sigma


def dt_intersect(scene: Scene, o, d, skip=None, t_eps: float = 1e-5, brute_force: bool = False):
    _dev_check(o, d, skip)
    n = o.shape[0]
    dev = o.device
    tri = torch.empty(n, dtype=torch.int32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    b = torch.empty(n, 2, dtype=torch.float32, device=dev)
    sc = scene.c()
    _check(load().dt_intersect(C.byref(sc), _ptr(o), _ptr(d), _ptr(skip), n, t_eps,
                               int(brute_force), _ptr(tri), _ptr(t), _ptr(b), _stream(dev)))
    return tri, t, b


# ------------------------------------------------------------------ silhouette (mask) term
def _mesh_scene(mesh: "Mesh") -> _Scene:
    s = _Scene()
    s.V, s.nv, s.F, s.nf = mesh.V.data_ptr(), mesh.nv, mesh.F.data_ptr(), mesh.nf
    s.bvh = mesh.blob.data_ptr()
    return s


def dt_mask_forward(mesh: "Mesh", rays: "Rays", t_eps: float = 1e-5) -> torch.Tensor:
    """Centre-sample coverage [n_pixels] of the cameras in `rays` (1 where the
    pixel centre's camera ray meets the mesh)."""
    out = torch.empty(rays.n_pixels, dtype=torch.float32, device=mesh.V.device)
    _check(load().dt_mask_forward(C.byref(_mesh_scene(mesh)), C.byref(rays.s), C.c_float(t_eps),
                                  _ptr(out), _stream(mesh.V.device)))
    return out


class MaskGrad:
    """Workspace for dt_mask_backward on one mesh topology."""

    def __init__(self, mesh: "Mesh"):
        n = C.c_size_t()
        _check(load().dt_mask_bytes(mesh.nv, mesh.nf, C.byref(n)))
        self.ws = _bytes(n.value, mesh.V.device)
        self.counts = torch.zeros(3, dtype=torch.int64, device=mesh.V.device)

    def __call__(self, mesh: "Mesh", rays: "Rays", grad_mask: torch.Tensor, rho: float = 2.0):
        """dLoss/dV [nv, 3] through the motion of the outline, for dLoss/dM
        given per pixel; self.counts then holds (outline points with a nonzero
        pixel gradient, visible ones, stack overflows)."""
        _dev_check(grad_mask)
        dV = torch.empty_like(mesh.V)
        _check(load().dt_mask_backward(C.byref(_mesh_scene(mesh)), C.byref(rays.s), _ptr(grad_mask),
                                       C.c_float(rho), _ptr(dV), _ptr(self.counts), _ptr(self.ws),
                                       self.ws.numel(), _stream(mesh.V.device)))
        return dV


# ------------------------------------------------------------------ vertex reparameterisation
class Smooth:
    """(I + lam L) x = b on the device for one mesh topology, L the
    combinatorial Laplacian of its edge graph given as a CSR adjacency
    (adj_off [nv + 1], adj: int32 neighbour lists, both ends of every edge)."""

    def __init__(self, adj_off: torch.Tensor, adj: torch.Tensor, lam: float):
        _dev_check(adj_off, adj)
        if adj_off.dtype != torch.int32 or adj.dtype != torch.int32:
            raise DTError("Smooth: the adjacency must be int32")
        self.adj_off, self.adj, self.lam = adj_off.contiguous(), adj.contiguous(), float(lam)
        self.nv = adj_off.numel() - 1
        n = C.c_size_t()
        _check(load().dt_smooth_bytes(self.nv, C.byref(n)))
        self.ws = _bytes(n.value, adj.device)
        self.iters, self.resid = 0, 0.0

    def solve(self, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-10, max_iters: int = 1000) -> torch.Tensor:
        """Solves in place into x (float64 [nv, 3], holding the starting guess)
        and returns it; self.iters / self.resid: the iterations run and the
        final relative residual.  Raises DTError when the solve does not
        converge within max_iters."""
        b = b.contiguous()
        _dev_check(b, x)
        if b.dtype != torch.float64 or x.dtype != torch.float64 or b.shape != (self.nv, 3) or x.shape != b.shape \
                or not x.is_contiguous():
            raise DTError("Smooth.solve: b and x must be float64 [nv, 3], x contiguous")
        it, res = C.c_int32(), C.c_double()
        st = load().dt_smooth_solve(_ptr(self.adj_off), _ptr(self.adj), self.nv, self.lam, _ptr(b), _ptr(x),
                                    tol, max_iters, C.byref(it), C.byref(res), _ptr(self.ws), self.ws.numel(),
                                    _stream(x.device))
        self.iters, self.resid = it.value, res.value
        _check(st)
        return x
