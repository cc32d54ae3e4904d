"""Continuous-batching render server over the device step `dt_serve_step`.

Scenes (mesh + BVH + IoR + sigma + environment map) stay resident on the
device.  Requests (render: the scene's own environment; relight: another one)
arrive over time; the host loop admits waiting requests into free slots while
the pixel pool and the ray queue have room, and runs one device step per
iteration: every live ray of every admitted request advances by one surface
interaction, and the camera rays of the requests admitted in that iteration
join the same queue.  When a request's slot has no rays left its image is
complete; it is copied out (with per-pixel flags and path signatures) and its
slot and pixels are released.  A request that lost rays to a full queue is
traced again instead.

`run_fifo` serves the same stream one request at a time with the plain
tracer (`dt_trace_forward`), the baseline the server is compared against.
"""
from __future__ import annotations

import collections
import ctypes as C
import math
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
                                C.POINTER(_Admit), i32, i64, vp, vp, vp, i64, vp, vp, vp, i64,
                                C.c_float, vp, C.c_size_t, vp]
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
    flags: np.ndarray | None = None    # per-pixel DT_FLAG_* of the served image
    sig: np.ndarray | None = None      # per-pixel path signatures (uint64)
    pixel_offset: int = -1
    slot: int = -1
    retries: int = 0                   # attempts that lost rays to a full queue
    reserved: int = 0
    admit_step: int = -1
    peak: int = 0                      # most live rays seen in one step

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
    """Resident scenes and environments, a pixel pool, one ray queue.

    Admission: a request reserves queue room for its peak number of live rays,
    its pixel count times the largest peak-to-camera-ray ratio measured so far
    on its scene (`growth`, times a margin; `default_growth` before the first
    measurement); it is admitted while a slot, a pixel range and unreserved
    queue room are free.  The device reports per slot the rays lost to a full
    queue; a request that lost any is traced again with twice the reservation,
    so a finished image is never missing radiance.

    The loop keeps the device busy: step k + 1 is queued before the host reads
    step k's per-slot counts (copied into pinned memory behind an event), so
    host bookkeeping overlaps device work; admissions and releases act one
    step later than they could.
    """

    MARGIN = 1.25

    def __init__(self, device=None, queue_capacity: int = 16 << 20, pixel_pool: int = 16 << 20,
                 t_eps: float = 1e-5, default_growth: float = 2.0):
        self.dev = torch.device(device or "cuda:0")
        self.L = _bind(B.load())
        self.cap = int(queue_capacity)
        sz = C.c_size_t()
        B._check(self.L.dt_serve_bytes(self.cap, C.byref(sz)))
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=self.dev)
        self.n_pixels = int(pixel_pool)
        self.pixels = torch.zeros(self.n_pixels, 3, dtype=torch.float32, device=self.dev)
        self.flags = torch.zeros(self.n_pixels, dtype=torch.int32, device=self.dev)
        self.sig = torch.zeros(self.n_pixels, dtype=torch.int64, device=self.dev)
        # per-step report, one buffer: live rays per slot, dropped rays per
        # slot (both uint32), then the three int64 stats
        self.info = torch.zeros(2 * MAX_SLOTS * 4 + 3 * 8, dtype=torch.uint8, device=self.dev)
        self.live = self.info[:4 * MAX_SLOTS].view(torch.int32)
        self.slot_dropped = self.info[4 * MAX_SLOTS:8 * MAX_SLOTS].view(torch.int32)
        self.stats = self.info[8 * MAX_SLOTS:].view(torch.int64)
        self._host = [torch.empty(self.info.numel(), dtype=torch.uint8).pin_memory() for _ in range(2)]
        self._ev = [torch.cuda.Event() for _ in range(2)]
        self.t_eps = t_eps
        self.default_growth = float(default_growth)
        self.growth = {}
        self.scenes, self.envs, self.scene_env = [], [], []
        self.retries = 0

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

    def reservation(self, r) -> int:
        """Queue room reserved for request r: pixels x the measured peak growth
        of its scene (x a margin), doubled per earlier attempt that lost rays."""
        g = self.growth.get(r.scene)
        f = self.default_growth if g is None else max(g * self.MARGIN, 1.0)
        return int(min(self.cap, math.ceil(r.n_pixels * f * (2 ** r.retries))))

    # ------------------------------------------------------------ the loop
    def run(self, requests, realtime: bool = True, max_wait_s: float = 600.0):
        """Serve `requests` (arrival times relative to now).  Returns them with
        admitted / finished times, images, per-pixel flags and path signatures
        filled in."""
        L = self.L
        stream = B._stream(self.dev)
        tstream = torch.cuda.current_stream(self.dev)
        B._check(L.dt_serve_reset(C.c_void_p(self.ws.data_ptr()), self.ws.numel(), self.cap, stream))
        sc, ev = self._tables()
        for r in requests:
            r.retries, r.image, r.finished = 0, None, None
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        active = {}            # slot -> request
        draining = []          # (request, image, flags, sig, event): copies in flight
        free_slots = list(range(MAX_SLOTS))[::-1]
        pool = _Pool(self.n_pixels)
        reserved = 0
        step = 0
        prev = None            # step whose report is not read yet
        self.steps, self.retries = 0, 0
        self.traced = self.dropped = 0
        t0 = time.perf_counter()
        clock = 0.0

        def now_s():
            return time.perf_counter() - t0 if realtime else clock

        def drain(block=False):
            keep = []
            for item in draining:
                r, img, fl, sg, e = item
                if block:
                    e.synchronize()
                if block or e.query():
                    r.image, r.flags, r.sig = img.numpy(), fl.numpy(), sg.numpy().view(np.uint64)
                    r.finished = now_s()
                else:
                    keep.append(item)
            draining[:] = keep

        while pending or waiting or active or prev is not None or draining:
            now = now_s()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            admits = []
            while waiting and free_slots:
                r = waiting[0]
                need = self.reservation(r)
                if r.n_pixels > self.cap:
                    raise B.DTError(f"request {r.rid} ({r.n_pixels} pixels) can never be admitted: "
                                    f"queue capacity {self.cap}")
                if reserved + need > self.cap and (active or admits):
                    break
                off = pool.alloc(r.n_pixels)
                if off is None:
                    if not active and not admits and r.n_pixels > self.n_pixels:
                        raise B.DTError(f"request {r.rid} ({r.n_pixels} pixels) can never be "
                                        f"admitted: pixel pool {self.n_pixels}")
                    break
                waiting.popleft()
                r.pixel_offset, r.slot = off, free_slots.pop()
                r.reserved, r.admit_step, r.peak = need, step, 0
                if r.retries == 0:
                    r.admitted = now
                reserved += need
                admits.append(r)
                active[r.slot] = r
            launched = None
            if admits or any(a.admit_step < step for a in active.values()):
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
                B._check(L.dt_serve_step(
                    sc, len(self.scenes), ev, len(self.envs), arr, len(admits), step,
                    C.c_void_p(self.pixels.data_ptr()), C.c_void_p(self.flags.data_ptr()),
                    C.c_void_p(self.sig.data_ptr()), self.n_pixels,
                    C.c_void_p(self.live.data_ptr()), C.c_void_p(self.slot_dropped.data_ptr()),
                    C.c_void_p(self.stats.data_ptr()), self.cap, self.t_eps,
                    C.c_void_p(self.ws.data_ptr()), self.ws.numel(), stream))
                buf = self._host[step & 1]
                buf.copy_(self.info, non_blocking=True)
                self._ev[step & 1].record(tstream)
                launched = step
                step += 1
                if not realtime:
                    clock += 1e-4
            elif prev is None:
                drain()
                if not waiting and not active and pending:
                    nxt = pending[0].arrival
                    if now > max_wait_s:
                        raise B.DTError("server idle beyond max_wait_s")
                    if realtime:
                        time.sleep(max(0.0, min(nxt - now, 0.002)))
                    else:
                        clock = max(clock, nxt)
                elif draining:
                    time.sleep(0.0)
                continue
            if prev is not None:
                # the report of the step before the one just queued
                self._ev[prev & 1].synchronize()
                rep = self._host[prev & 1]
                live = rep[:4 * MAX_SLOTS].view(torch.int32).numpy()
                lost = rep[4 * MAX_SLOTS:8 * MAX_SLOTS].view(torch.int32).numpy()
                st = rep[8 * MAX_SLOTS:].view(torch.int64).numpy()
                self.traced, self.dropped = int(st[0]), int(st[1])
                for slot in list(active):
                    r = active[slot]
                    if r.admit_step > prev:
                        continue               # admitted by a step not reported yet
                    r.peak = max(r.peak, int(live[slot]))
                    if live[slot] != 0:
                        continue
                    active.pop(slot)
                    reserved -= r.reserved
                    a, n = r.pixel_offset, r.n_pixels
                    if lost[slot] != 0:
                        # rays were lost to a full queue: trace it again with
                        # twice the room, ahead of everything still waiting
                        if r.reserved >= self.cap and len(active) == 0:
                            raise B.DTError(f"request {r.rid} loses rays even alone: queue "
                                            f"capacity {self.cap} is too small")
                        r.retries += 1
                        self.retries += 1
                        waiting.appendleft(r)
                    else:
                        g = max(r.peak, r.n_pixels) / r.n_pixels
                        self.growth[r.scene] = max(self.growth.get(r.scene, 0.0), g)
                        img = self.pixels[a:a + n].to("cpu", non_blocking=True)
                        fl = self.flags[a:a + n].to("cpu", non_blocking=True)
                        sg = self.sig[a:a + n].to("cpu", non_blocking=True)
                        e = torch.cuda.Event()
                        e.record(tstream)
                        draining.append((r, img, fl, sg, e))
                    pool.release(a, n)
                    free_slots.append(slot)
            prev = launched
            drain()
        drain(block=True)
        self.steps = step
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
