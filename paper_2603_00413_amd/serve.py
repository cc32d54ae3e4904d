"""Continuous-batching render server over the device step `dt_serve_step`.

Scenes (mesh + BVH + IoR + sigma + environment map) stay resident on the
device.  Requests (render: the scene's own environment; relight: another one)
arrive over time; the host loop admits waiting requests into free slots while
the pixel pool and the ray queue have room, and runs one device step per
iteration: every live ray of every admitted request advances by one surface
interaction, and the camera rays of the requests admitted in that iteration
join the same queue.  When a request's slot has no rays left its image is
complete; it is copied out and its slot and pixels are released.

`run_fifo` serves the same stream one request at a time with the plain
tracer (`dt_trace_forward`), the baseline the server is compared against.
"""
from __future__ import annotations

import collections
import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B

MAX_SCENES, MAX_ENVS, MAX_SLOTS = 8, 8, 256


class _ServeScene(C.Structure):
    _fields_ = [("V", C.c_void_p), ("nv", C.c_int32), ("F", C.c_void_p), ("nf", C.c_int32),
                ("bvh", C.c_void_p), ("ior", C.c_void_p), ("sigma", C.c_void_p)]


class _Admit(C.Structure):
    _fields_ = [("slot", C.c_int32), ("scene", C.c_int32), ("env", C.c_int32),
                ("max_depth", C.c_int32), ("camera", B._Camera)]


def _bind(L):
    if getattr(L, "_serve_bound", False):
        return L
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.dt_serve_bytes.argtypes = [i64, C.POINTER(C.c_size_t)]
    L.dt_serve_reset.argtypes = [vp, C.c_size_t, i64, vp]
    L.dt_serve_step.argtypes = [C.POINTER(_ServeScene), i32, C.POINTER(B._Env), i32,
                                C.POINTER(_Admit), i32, i64, vp, i64, vp, vp, i64, C.c_float, vp,
                                C.c_size_t, vp]
    L._serve_bound = True
    return L


@dataclass
class Request:
    rid: int
    scene: int
    camera: object                 # synth.Camera
    max_depth: int
    env: int | None = None         # None: the scene's own environment (render)
    arrival: float = 0.0           # seconds after the start of the stream
    admitted: float | None = None
    finished: float | None = None
    image: np.ndarray | None = None
    pixel_offset: int = -1
    slot: int = -1

    @property
    def n_pixels(self):
        return self.camera.width * self.camera.height

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class _Pool:
    """First-fit allocator of pixel ranges."""

    def __init__(self, n):
        self.free = [(0, n)]

    def alloc(self, k):
        for i, (a, n) in enumerate(self.free):
            if n >= k:
                if n == k:
                    self.free.pop(i)
                else:
                    self.free[i] = (a + k, n - k)
                return a
        return None

    def release(self, a, k):
        self.free.append((a, k))
        self.free.sort()
        merged = []
        for s, n in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + n)
            else:
                merged.append((s, n))
        self.free = merged


class Server:
    def __init__(self, device=None, queue_capacity: int = 16 << 20, pixel_pool: int = 16 << 20,
                 t_eps: float = 1e-5):
        self.dev = torch.device(device or "cuda:0")
        self.L = _bind(B.load())
        self.cap = int(queue_capacity)
        sz = C.c_size_t()
        B._check(self.L.dt_serve_bytes(self.cap, C.byref(sz)))
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=self.dev)
        self.n_pixels = int(pixel_pool)
        self.pixels = torch.zeros(self.n_pixels, 3, dtype=torch.float32, device=self.dev)
        self.live = torch.zeros(MAX_SLOTS, dtype=torch.int32, device=self.dev)
        self.stats = torch.zeros(3, dtype=torch.int64, device=self.dev)
        self.t_eps = t_eps
        self.scenes, self.envs, self.scene_env = [], [], []
        self._keep = []

    # ------------------------------------------------------------ resident data
    def add_env(self, env) -> int:
        """env: equirect texels [H, W, 3] (numpy), or a binding Env (map or MLP)
        already on this device."""
        if len(self.envs) >= MAX_ENVS:
            raise B.DTError("too many environments")
        if not isinstance(env, B.Env):
            env = B.Env(torch.from_numpy(np.ascontiguousarray(env, np.float32)).to(self.dev))
        self.envs.append(env)
        return len(self.envs) - 1

    def add_scene(self, V, F, ior, sigma, env_texels) -> int:
        """env_texels: the scene's own environment, as for add_env."""
        if len(self.scenes) >= MAX_SCENES:
            raise B.DTError("too many scenes")
        mesh = B.Mesh(torch.from_numpy(np.asarray(V, np.float32)).to(self.dev),
                      torch.from_numpy(np.asarray(F, np.int32)).to(self.dev))
        ior_t = torch.tensor([float(ior)], dtype=torch.float32, device=self.dev)
        sg = np.broadcast_to(np.asarray(sigma, np.float32), (3,)).copy()
        sigma_t = torch.from_numpy(sg).to(self.dev)
        self.scenes.append((mesh, ior_t, sigma_t))
        self.scene_env.append(self.add_env(env_texels))
        return len(self.scenes) - 1

    def _tables(self):
        sc = (_ServeScene * len(self.scenes))()
        for i, (m, ior, sg) in enumerate(self.scenes):
            sc[i].V, sc[i].nv, sc[i].F, sc[i].nf = m.V.data_ptr(), m.nv, m.F.data_ptr(), m.nf
            sc[i].bvh, sc[i].ior, sc[i].sigma = m.blob.data_ptr(), ior.data_ptr(), sg.data_ptr()
        ev = (B._Env * len(self.envs))()
        for i, e in enumerate(self.envs):
            ev[i] = e.s
        return sc, ev

    # ------------------------------------------------------------ the loop
    def run(self, requests, realtime: bool = True, max_wait_s: float = 600.0):
        """Serve `requests` (arrival times relative to now).  Returns them with
        admitted / finished times and images filled in."""
        L = self.L
        stream = B._stream(self.dev)
        B._check(L.dt_serve_reset(C.c_void_p(self.ws.data_ptr()), self.ws.numel(), self.cap, stream))
        sc, ev = self._tables()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        active = {}
        free_slots = list(range(MAX_SLOTS))[::-1]
        pool = _Pool(self.n_pixels)
        live_rays = 0
        step = 0
        self.steps = 0
        t0 = time.perf_counter()
        clock = 0.0
        while pending or waiting or active:
            now = time.perf_counter() - t0 if realtime else clock
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            if not waiting and not active:
                nxt = pending[0].arrival
                if realtime:
                    time.sleep(max(0.0, min(nxt - now, 0.01)))
                else:
                    clock = nxt
                if now > max_wait_s:
                    raise B.DTError("server idle beyond max_wait_s")
                continue
            admits = []
            est = live_rays
            while waiting and free_slots:
                r = waiting[0]
                if 2 * (est + r.n_pixels) > self.cap:
                    break
                off = pool.alloc(r.n_pixels)
                if off is None:
                    break
                waiting.popleft()
                r.pixel_offset, r.slot = off, free_slots.pop()
                r.admitted = now
                est += r.n_pixels
                admits.append(r)
                active[r.slot] = r
            if not admits and not active:
                r = waiting[0]
                raise B.DTError(f"request {r.rid} ({r.n_pixels} pixels) can never be admitted: "
                                f"pixel pool {self.n_pixels}, queue capacity {self.cap}")
            arr = (_Admit * max(len(admits), 1))()
            for i, r in enumerate(admits):
                a = arr[i]
                a.slot, a.scene, a.max_depth = r.slot, r.scene, r.max_depth
                a.env = self.scene_env[r.scene] if r.env is None else r.env
                c = r.camera
                for k in range(3):
                    a.camera.eye[k], a.camera.target[k], a.camera.up[k] = c.eye[k], c.target[k], c.up[k]
                a.camera.fov_deg, a.camera.width, a.camera.height = c.fov_deg, c.width, c.height
                a.camera.pixel_offset = r.pixel_offset
            B._check(L.dt_serve_step(sc, len(self.scenes), ev, len(self.envs), arr, len(admits), step,
                                     C.c_void_p(self.pixels.data_ptr()), self.n_pixels,
                                     C.c_void_p(self.live.data_ptr()), C.c_void_p(self.stats.data_ptr()),
                                     self.cap, self.t_eps, C.c_void_p(self.ws.data_ptr()),
                                     self.ws.numel(), stream))
            step += 1
            live = self.live.cpu().numpy()          # synchronises with the step
            st = self.stats.cpu().numpy()
            live_rays = int(st[2])
            if not realtime:
                clock += 1e-4
            done_t = time.perf_counter() - t0 if realtime else clock
            for slot in list(active):
                if live[slot] == 0:
                    r = active.pop(slot)
                    a, n = r.pixel_offset, r.n_pixels
                    r.image = self.pixels[a:a + n].cpu().numpy().copy()
                    r.finished = time.perf_counter() - t0 if realtime else done_t
                    pool.release(a, n)
                    free_slots.append(slot)
        self.steps = step
        self.traced = int(self.stats.cpu()[0])
        self.dropped = int(self.stats.cpu()[1])
        return requests


def run_fifo(server: Server, requests, realtime: bool = True):
    """Baseline: the same stream served one request at a time, in arrival
    order, each traced alone with the plain tracer."""
    dev = server.dev
    reqs = sorted(requests, key=lambda r: r.arrival)
    bufs = {}
    traced = 0
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        mesh, ior, sg = server.scenes[r.scene]
        env = server.envs[server.scene_env[r.scene] if r.env is None else r.env]
        scene = B.Scene(mesh, ior, sg, env)
        rays = B.Rays(cameras=[r.camera])
        key = (r.scene, r.n_pixels)
        cap = bufs[key][0] if key in bufs else 2 * r.n_pixels
        r.admitted = time.perf_counter() - t0
        while True:
            p = B.Params(max_depth=r.max_depth, queue_capacity=cap, t_eps=server.t_eps)
            if key not in bufs or bufs[key][0] != cap:
                bufs[key] = (cap, B.Buffers(p, rays, mesh, tape=False))
            buf = bufs[key][1]
            rgb, _, _ = B.dt_trace_forward(scene, rays, p, buf, want_aux=False)
            st = buf.stats.cpu().numpy()
            if st[B.STAT_DROPPED] == 0:
                break
            cap *= 2                         # a queue overflowed: trace again, larger
        r.image = rgb.cpu().numpy()
        traced += int(st[B.STAT_TOTAL])
        r.finished = time.perf_counter() - t0
    return reqs, traced
