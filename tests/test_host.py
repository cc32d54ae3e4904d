"""Host-side logic that runs without a device: the server's pixel-range
allocator, the memory policy that picks the checkpoint stride, camera
marshalling and the benchmark's single-GPU guard."""
import os
import subprocess
import sys

import numpy as np

from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pixel_pool_first_fit_and_merge():
    from paper_2603_00413_amd.serve import _Pool
    p = _Pool(100)
    a = p.alloc(30)
    b = p.alloc(30)
    c = p.alloc(30)
    assert (a, b, c) == (0, 30, 60)
    assert p.alloc(20) is None            # only 10 left
    p.release(b, 30)
    assert p.alloc(40) is None            # the hole is 30 wide
    d = p.alloc(25)                       # first fit: inside the hole
    assert d == 30
    p.release(a, 30)
    p.release(d, 25)
    p.release(c, 30)
    assert p.free == [(0, 100)]           # every range merged back


def test_checkpoint_stride_follows_the_budget():
    from paper_2603_00413_amd.autograd import choose_stride
    args = dict(max_depth=6, n_rays=1 << 20, nv=51200, nf=102400, capacity=1 << 21)
    sizes = []
    for k in range(1, 8):
        ws, tape = B.dt_trace_bytes(B.Params(max_depth=6, checkpoint_stride=k,
                                             queue_capacity=args["capacity"]),
                                    args["n_rays"], args["nv"], args["nf"])
        sizes.append(ws + tape)
    assert choose_stride(budget_bytes=1 << 62, **args) == 1          # everything fits
    k_min = int(np.argmin(sizes)) + 1
    assert choose_stride(budget_bytes=1, **args) == k_min           # nothing fits: least memory
    # a budget between the two picks the smallest stride that fits
    mid = (sizes[0] + min(sizes)) // 2
    k = choose_stride(budget_bytes=mid, **args)
    assert sizes[k - 1] <= mid and all(s > mid for s in sizes[:k - 1])


def test_camera_marshalling_offsets():
    cams = [synth.look_at_camera(np.array([0.0, 0.0, 3.0]), 32, 16),
            synth.look_at_camera(np.array([3.0, 0.0, 0.0]), 8, 8)]
    r = B.Rays(cameras=cams)
    assert r.n_rays == r.n_pixels == 32 * 16 + 64
    assert r.s.n_cameras == 2
    c0, c1 = r.s.cameras[0], r.s.cameras[1]
    assert (c0.width, c0.height, c0.pixel_offset) == (32, 16, 0)
    assert (c1.width, c1.height, c1.pixel_offset) == (8, 8, 512)
    assert abs(c1.eye[0] - 3.0) < 1e-6 and abs(c0.fov_deg - cams[0].fov_deg) < 1e-6


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
