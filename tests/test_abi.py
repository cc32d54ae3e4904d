"""The C-ABI library loads, exports every entry point the header declares,
and rejects bad arguments on the host (no device work is queued)."""
import ctypes as C
import os
import re

import pytest

from paper_2603_00413_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "difftrans.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["dt_build_bvh", "dt_trace_forward", "dt_trace_backward", "dt_env_query"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = B.load()
    for name in declared():
        assert hasattr(L, name), name
    assert set(B.EXPORTS) <= set(declared())


def test_host_validation_without_device():
    L = B.load()
    a, b = C.c_size_t(), C.c_size_t()
    assert L.dt_bvh_bytes(0, 0, C.byref(a), C.byref(b)) == 1
    assert "nv >= 3" in L.dt_last_error().decode()
    assert L.dt_bvh_bytes(642, 1280, C.byref(a), C.byref(b)) == 0
    assert a.value > 1280 * 48 and b.value > 0
    p = B.Params(max_depth=17).c()
    assert L.dt_trace_bytes(C.byref(p), 100, 3, 1, C.byref(a), C.byref(b)) == 1
    p = B.Params(max_depth=6, checkpoint_stride=2).c()
    assert L.dt_trace_bytes(C.byref(p), 4096, 642, 1280, C.byref(a), C.byref(b)) == 0
    ws2, tape2 = a.value, b.value
    p = B.Params(max_depth=6, checkpoint_stride=1).c()
    assert L.dt_trace_bytes(C.byref(p), 4096, 642, 1280, C.byref(a), C.byref(b)) == 0
    assert b.value > tape2          # storing every generation costs more tape
    # a null scene is rejected before anything touches a device
    assert L.dt_trace_forward(None, None, None, None, None, None, None, None, None, 0, None, 0,
                              None) == 1
    assert L.dt_status_string(2) == b"workspace too small"
    # the reparameterisation's solve: workspace sizing and null pointers
    assert L.dt_smooth_bytes(0, C.byref(a)) == 1
    assert L.dt_smooth_bytes(1000, C.byref(a)) == 0
    assert a.value >= 3 * 3 * 1000 * 8
    assert L.dt_smooth_solve(None, None, 1000, 1.0, None, None, 1e-10, 100, None, None, None, 0, None) == 1
    assert L.dt_status_string(6) == b"not converged"


def test_queue_capacity_bounds_tape():
    L = B.load()
    a, b = C.c_size_t(), C.c_size_t()
    p = B.Params(max_depth=6, queue_capacity=0).c()
    L.dt_trace_bytes(C.byref(p), 1 << 20, 51200, 102400, C.byref(a), C.byref(b))
    worst = b.value
    p = B.Params(max_depth=6, queue_capacity=2 << 20).c()
    L.dt_trace_bytes(C.byref(p), 1 << 20, 51200, 102400, C.byref(a), C.byref(b))
    assert b.value < worst / 5


def test_unsupported_shapes_are_rejected_on_the_host():
    """An MLP with more frequencies than the matrix-core input order holds, or
    a mesh beyond the traversal's 2^26-triangle packing, is refused before any
    device work (the pointers below are never dereferenced)."""
    L = B.load()
    e = B._Env()
    e.kind = B.ENV_MLP
    e.n_freq, e.n_layers, e.hidden, e.in_pad = 8, 3, 64, 64
    e.weights, e.biases = 16, 16          # non-null, never read
    assert L.dt_env_query(C.byref(e), C.c_void_p(16), 1, C.c_void_p(16), None) == 5
    assert "n_freq <= 7" in L.dt_last_error().decode()
    e.n_freq, e.hidden = 6, 96
    assert L.dt_env_query(C.byref(e), C.c_void_p(16), 1, C.c_void_p(16), None) == 5
    a, b = C.c_size_t(), C.c_size_t()
    assert L.dt_bvh_bytes(3, (1 << 26) + 1, C.byref(a), C.byref(b)) == 1
    assert "2^26" in L.dt_last_error().decode()
    assert L.dt_bvh_bytes(3, 1 << 26, C.byref(a), C.byref(b)) == 0


def test_noalloc_build_rejects_meshes_beyond_its_array():
    """The no-allocation build refuses, on the host, a mesh whose build
    workspace exceeds the library's per-device array (about 500k faces)."""
    L = B.load()
    a, b = C.c_size_t(), C.c_size_t()
    fake = C.c_void_p(16)            # never dereferenced: rejected before any device call
    assert L.dt_build_bvh_noalloc(fake, 1 << 20, fake, 2 << 20, fake, 1 << 30, None) == 3
    msg = L.dt_last_error().decode()
    assert "dt_build_bvh_noalloc" in msg and "workspace" in msg
    assert L.dt_build_bvh_noalloc(None, 642, fake, 1280, fake, 1 << 20, None) == 1
    # the largest serving scene (500k faces) fits
    L.dt_bvh_bytes(250_000, 500_000, C.byref(a), C.byref(b))
    assert b.value <= 32 << 20


def test_bad_field_is_rejected_on_the_host():
    """A volumetric field with too few nodes, no samples, half of its
    gradient targets, or beside an MLP environment is refused before any
    device work (the pointers below are never dereferenced)."""
    L = B.load()
    fake = 16
    env = B._Env()
    env.kind, env.width, env.height, env.texels = B.ENV_EQUIRECT, 8, 4, fake
    f = B._Field()
    f.grid, f.planes, f.nx, f.ny, f.nz, f.res, f.samples = fake, fake, 3, 3, 3, 4, 4
    for k in range(3):
        f.lo[k], f.hi[k] = -1.0, 1.0
    s = B._Scene()
    s.V, s.nv, s.F, s.nf, s.bvh, s.ior, s.sigma = fake, 3, fake, 1, fake, fake, fake
    s.env, s.field = C.pointer(env), C.pointer(f)
    p = B.Params(max_depth=2).c()

    def run():
        return L.dt_trace_forward(C.byref(s), None, C.byref(p), None, None, None, None, None, None, 0,
                                  None, 0, None)

    f.nx = 1
    assert run() == 1 and "field needs 2..1024" in L.dt_last_error().decode()
    f.nx, f.samples = 3, 0
    assert run() == 1 and "samples" in L.dt_last_error().decode()
    f.samples, f.d_grid = 4, fake
    assert run() == 1 and "d_grid and d_planes" in L.dt_last_error().decode()
    f.d_grid, f.hi[1] = None, -1.0
    assert run() == 1 and "hi > lo" in L.dt_last_error().decode()
    f.hi[1] = 1.0
    env.kind, env.n_freq, env.n_layers, env.hidden, env.in_pad = B.ENV_MLP, 6, 3, 64, 64
    env.weights, env.biases = fake, fake
    assert run() == 5 and "MLP" in L.dt_last_error().decode()
