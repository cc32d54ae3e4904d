#!/usr/bin/env python
"""Throughput of the differentiable transparent-mesh tracer on one MI355X.

Workload: seeded displaced torus (102,400 triangles, genus 1), IoR 1.45,
sigma 0.3, eight 512x512 views from a sphere of radius 3, depth 6, 512x256
FP32 equirect environment.  One step = the whole hot path over the batch:
vertex normals + LBVH rebuild, camera rays, the wavefront forward (trace,
shade, compaction, environment, pixel accumulation) with its tape, the
gradient of an L2 loss, and the adjoint sweep to dV, dIoR, dsigma.

Metric: Mrays/s = ray segments intersected per step (every generation,
counted once) / step time.  Prints one JSON line.  Beside the headline it
reports the plain forward, the recompute form (stride 3), camera rays/s with
and without the tree rebuild, and further legs unless switched off: a
spatially varying absorption grid with its gradient, the texel gradient and a
volumetric exterior field with its gradient (--no-grid), the serving loop (--no-serve), the MLP-lit training step
(--no-mlp), the 2M-triangle thin shell (--no-stress) and the oracle's CPU
rate (--no-cpu-baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mrays/s fwd+bwd at depth 6 (1 GPU) vs plain tracer; p50/p99 render latency"

# algorithmic bytes per ray of each kernel (compulsory traffic; BVH node
# reads are cache-resident and counted separately)
TRACE_PER_RAY = 48 + 16 + 4          # ray record in, hit + decision out
TRACE_PER_HIT = 12 + 36 + 48         # face row, 3 vertices, 3 vertex normals
TRACE_PER_MISS = 48 + 12             # 4 texels, pixel accumulation
ADJ_PER_RAY = 48 + 16 + 4 + 8 + 12 + 48   # ray, hit, decision, children, dL/dC, adjoint out
ADJ_PER_HIT = 96 + 96 + 64 + 8       # geometry, 2 child adjoints, face record and (face, rank) key
ADJ_PER_MISS = 48                    # 4 texels

# HBM bytes per launch of the dominant kernel on this workload, measured with
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch, averaged
# over the run's launches), FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0:
# what the two counters read for a 1 GiB device-to-device copy.  Valid only
# for the kernel sources with this SHA-256; other sources report null.
MEASURED_TRAFFIC = {
    "k_trace": {
        # the traversal kernel and the tree builder whose tree it walks
        "sources": ["paper_2603_00413_amd/csrc/trace.hip", "paper_2603_00413_amd/csrc/dt_device.h",
                    "paper_2603_00413_amd/csrc/dt_internal.h", "paper_2603_00413_amd/csrc/dt_queue.h",
                    "paper_2603_00413_amd/csrc/bvh.hip"],
        "sha256": "3f81142cced588f5d14840ca135c9dcc59b1b8a4dbcf75baa9ab5206c1062c94",
        "bytes": (316911.5 * 2.0 + 79344.9) * 1024,
        # rocprofv3 --pmc SQ_INSTS_VALU SQ_THREAD_CYCLES_VALU SQ_ACTIVE_INST_VALU:
        # wave-level VALU instructions per launch, and the share of lanes active
        # in them
        "valu_insts": 2.605e8,
        "lane_utilization": 0.619,
    },
}


# VALU issue peak: 256 CUs x 4 SIMDs, a wave64 VALU instruction every 4 cycles
# per SIMD (16 lanes), 2.4 GHz = 614.4 G wave-instructions/s (the FP32 vector
# peak of 157.3 TFLOP/s counts 2 flops of an FMA on 2 packed values per lane)
VALU_ISSUE_PEAK_GIPS = 256 * 2.4


def _measured(kernel):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return m if h.hexdigest() == m["sha256"] else None


def measured_traffic(kernel):
    """Counter-measured bytes per launch of kernel, or None when the sources
    changed since the counters were taken."""
    m = _measured(kernel)
    return int(m["bytes"]) if m else None


def valu_issue(kernel, avg_launch_ms):
    """Counter-measured VALU instruction rate of kernel against the issue peak
    (None when the sources changed since the counters were taken)."""
    m = _measured(kernel)
    if not m or "valu_insts" not in m:
        return None
    rate = m["valu_insts"] / (avg_launch_ms * 1e-3) / 1e9
    return {"insts_per_launch": m["valu_insts"], "achieved": round(rate, 1),
            "peak": VALU_ISSUE_PEAK_GIPS, "unit": "G wave-instr/s",
            "frac": round(rate / VALU_ISSUE_PEAK_GIPS, 4),
            "lane_utilization": m["lane_utilization"]}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--stride", type=int, default=1, help="checkpoint stride of the backward")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=1,
                    help="oracle baseline traces every n-th pixel in x and y")
    ap.add_argument("--no-mlp", action="store_true", help="skip the MLP-lit training-step leg")
    ap.add_argument("--no-stress", action="store_true", help="skip the 2M-triangle thin-shell leg")
    ap.add_argument("--no-grid", action="store_true",
                    help="skip the absorption-grid, texel-gradient and volumetric-field legs")
    ap.add_argument("--copy-only", action="store_true",
                    help="run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load as a fraction of the measured one-at-a-time capacity")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is a design note, not a runnable configuration", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2603_00413_amd import binding as B
    from paper_2603_00413_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    if args.copy_only:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n}))
        return

    wl = synth.torus_scene(n_views=args.views, res=args.res)
    log(f"scene {wl.name}: nv={len(wl.V)} nf={len(wl.F)} views={len(wl.cameras)} res={args.res}")
    V = torch.from_numpy(wl.V.astype(np.float32)).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    mesh = B.Mesh(V, F)
    env = B.Env(torch.from_numpy(wl.env).to(dev))
    ior = torch.tensor([wl.ior], dtype=torch.float32, device=dev)
    sigma = torch.tensor(wl.sigma, dtype=torch.float32, device=dev)
    scene = B.Scene(mesh, ior, sigma, env)
    rays = B.Rays(cameras=wl.cameras)
    N = rays.n_rays

    # queue capacity: grow until nothing is dropped, then size to the
    # largest generation with 5 % headroom
    cap = 2 * N
    while True:
        p = B.Params(max_depth=wl.max_depth, queue_capacity=cap)
        buf = B.Buffers(p, rays, mesh, tape=False)
        B.dt_trace_forward(scene, rays, p, buf, want_aux=False)
        st = buf.stats.cpu().numpy()
        if st[B.STAT_DROPPED] == 0:
            break
        cap *= 2
    counts = st[:wl.max_depth + 1].astype(np.int64)
    hits = st[B.STAT_HITS:B.STAT_HITS + wl.max_depth + 1].astype(np.int64)
    cap = int(max(counts[1:].max() * 1.05, 2048))
    del buf
    segs = int(counts.sum())
    log(f"rays per generation {counts.tolist()} hits {hits.tolist()} total {segs} capacity {cap}")

    params = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=args.stride)
    buf = B.Buffers(params, rays, mesh, tape=True)
    log(f"workspace {buf.ws_bytes / 2**30:.2f} GiB tape {buf.tape_bytes / 2**30:.2f} GiB")

    # L2 loss against a target rendered with other material parameters
    tscene = B.Scene(mesh, torch.tensor([1.5], device=dev), torch.tensor([0.25, 0.3, 0.35], device=dev), env)
    target, _, _ = B.dt_trace_forward(tscene, rays, params, buf, want_aux=False)
    target = target.clone()

    def step():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        grad = (rgb - target) * (2.0 / rgb.numel())
        return B.dt_trace_backward(scene, rays, params, buf, grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the timed steps traced the whole workload, nothing dropped
    st = buf.stats.cpu().numpy()
    assert st[B.STAT_DROPPED] == 0 and int(st[B.STAT_TOTAL]) == segs
    ms_step = 1e3 * elapsed / args.steps
    mrays = segs / (elapsed / args.steps) / 1e6

    # forward-only plain tracer on the same batch (context)
    pf = B.Params(max_depth=wl.max_depth, queue_capacity=cap)
    buf_f = B.Buffers(pf, rays, mesh, tape=False)
    for _ in range(2):
        B.dt_trace_forward(scene, rays, pf, buf_f, want_aux=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nf_steps = max(args.steps, 3)
    for _ in range(nf_steps):
        B.dt_trace_forward(scene, rays, pf, buf_f, want_aux=False)
    torch.cuda.synchronize()
    fwd_ms = 1e3 * (time.perf_counter() - t1) / nf_steps
    del buf_f

    def timed(fn, n):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / n

    # the same step without the per-step tree rebuild (the mesh unchanged)
    def step_no_rebuild():
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        return B.dt_trace_backward(scene, rays, params, buf, (rgb - target) * (2.0 / rgb.numel()))
    norebuild_ms = timed(step_no_rebuild, max(args.steps, 3))
    # the recompute form: every third generation on the tape, the others
    # traced again during the backward
    p3 = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=3)
    buf3 = B.Buffers(p3, rays, mesh, tape=True)

    def step_recompute():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, p3, buf3, want_aux=False)
        return B.dt_trace_backward(scene, rays, p3, buf3, (rgb - target) * (2.0 / rgb.numel()))
    recompute_ms = timed(step_recompute, max(args.steps, 3))
    recompute_mem = (buf3.ws_bytes + buf3.tape_bytes) / 2**30
    del buf3
    log(f"without rebuild {norebuild_ms:.2f} ms; recompute (stride 3) {recompute_ms:.2f} ms, "
        f"{recompute_mem:.2f} GiB workspace + tape")

    # per-kernel durations of the instrumented steps, on the library's stream
    timer = B.KernelTimer(wl.max_depth)
    params_t = B.Params(max_depth=wl.max_depth, queue_capacity=cap,
                        checkpoint_stride=args.stride, timing=timer)
    G = wl.max_depth + 1
    tr_ms, ad_ms = np.zeros(G), np.zeros(G)
    reps = 3
    for _ in range(reps):
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params_t, buf, want_aux=False)
        grad = (rgb - target) * (2.0 / rgb.numel())
        B.dt_trace_backward(scene, rays, params_t, buf, grad)
        torch.cuda.synchronize()
        tr_ms += np.array(timer.trace_ms(G)) / reps
        ad_ms += np.array(timer.adjoint_ms(G)) / reps
    miss = counts - hits
    tr_bytes = counts * TRACE_PER_RAY + hits * TRACE_PER_HIT + miss * TRACE_PER_MISS
    ad_bytes = counts * ADJ_PER_RAY + hits * ADJ_PER_HIT + miss * ADJ_PER_MISS
    kernels = {
        "k_trace": (tr_ms, tr_bytes),
        "k_adjoint": (ad_ms, ad_bytes),
    }
    dom = max(kernels, key=lambda k: kernels[k][0].sum())
    kms, kb = kernels[dom]
    launches = int((counts > 0).sum())
    avg_ms = float(kms.sum() / launches)
    bytes_per_launch = float(kb.sum() / launches)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    log(f"step {ms_step:.2f} ms; forward-only {fwd_ms:.2f} ms; k_trace per gen ms {np.round(tr_ms, 3).tolist()}; "
        f"k_adjoint per gen ms {np.round(ad_ms, 3).tolist()}")

    grid = None
    if not args.no_grid:
        grid = grid_bench(args, dev, mesh, rays, env, ior, sigma, wl, cap, target, segs)
        grid["env_texel_gradient"] = texel_grad_bench(args, dev, mesh, rays, ior, sigma, wl, cap,
                                                      target, segs)
        grid["volumetric_field"] = field_bench(args, dev, mesh, rays, env, ior, sigma, wl, cap, target, segs)
    buf_bytes = buf.ws_bytes + buf.tape_bytes
    del buf
    torch.cuda.empty_cache()
    serving = None
    if not args.no_serve:
        serving = serving_bench(args, dev)
    training = trainer = None
    if not args.no_mlp:
        training = training_step_bench(args, dev)
        trainer = trainer_bench(args, dev)
    stress = None
    if not args.no_stress:
        stress = stress_bench(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_stride)

    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": round(mrays, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded displaced torus, seeded sky map, seeded views)",
        "config": {
            "workload": "torus-102k fwd+bwd: 102,400 tris, 8 views x 512x512, depth 6, "
                        "IoR 1.45, sigma 0.3, env 512x256 f32, LBVH rebuilt every step",
            "camera_rays": N,
            "segments_per_step": segs,
            "checkpoint_stride": args.stride,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic(dom),
            "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": int(bytes_per_launch),
            # what actually bounds the traversal: VALU issue
            "valu_issue": valu_issue(dom, avg_ms),
        },
        "step_latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                            "p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "serving": serving,
        "training_step_mlp": training,
        "trainer_step_training_shape": trainer,
        "stress_thin_shell": stress,
        "absorption_grid": grid,
        "plain_forward": {"ms": round(fwd_ms, 3), "Mrays/s": round(segs / fwd_ms / 1e3, 3)},
        "recompute_stride3": {"ms_per_step": round(recompute_ms, 3),
                              "Mrays/s": round(segs / recompute_ms / 1e3, 3),
                              "workspace_plus_tape_GiB": round(recompute_mem, 3),
                              "store_all_GiB": round((buf_bytes) / 2**30, 3)},
        "camera_rays_per_s": {"with_rebuild": round(N / (ms_step * 1e-3)),
                              "without_rebuild": round(N / (norebuild_ms * 1e-3))},
        "kernel_ms_per_generation": {"k_trace": np.round(tr_ms, 4).tolist(),
                                     "k_adjoint": np.round(ad_ms, 4).tolist()},
        "cpu_baseline": cpu,
        "paper_timings": PAPER_TIMINGS,
    }
    print(json.dumps(out), flush=True)


def grid_bench(args, dev, mesh, rays, env, ior, sigma, wl, cap, target, segs):
    """The torus fwd+bwd step with a spatially varying absorption rate: a
    seeded 32^3 RGB grid over the object's box (values 0.1-0.5), 16 midpoint
    samples per interior segment; the grid gradient is written every step."""
    import torch

    from paper_2603_00413_amd import binding as B
    n, S = 32, 16
    rng = np.random.default_rng(7)
    mu = torch.from_numpy(rng.uniform(0.1, 0.5, (n, n, n, 3)).astype(np.float32)).to(dev)
    lo, hi = wl.V.min(0) - 0.01, wl.V.max(0) + 0.01
    ab = B.Absorption(mu, lo, hi, S)
    scene = B.Scene(mesh, ior, sigma, env, absorb=ab)
    params = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=args.stride)
    buf = B.Buffers(params, rays, mesh, tape=True)

    def step():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        grad = (rgb - target) * (2.0 / rgb.numel())
        return B.dt_trace_backward(scene, rays, params, buf, grad)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    st = buf.stats.cpu().numpy()
    assert st[B.STAT_DROPPED] == 0 and int(st[B.STAT_TOTAL]) == segs
    timer = B.KernelTimer(wl.max_depth)
    pt = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=args.stride,
                  timing=timer)
    mesh.build()
    rgb, _, _ = B.dt_trace_forward(scene, rays, pt, buf, want_aux=False)
    B.dt_trace_backward(scene, rays, pt, buf, (rgb - target) * (2.0 / rgb.numel()))
    torch.cuda.synchronize()
    G = wl.max_depth + 1
    tr, ad = np.array(timer.trace_ms(G)), np.array(timer.adjoint_ms(G))
    assert torch.isfinite(ab.d_mu).all() and float(ab.d_mu.abs().sum()) > 0
    log(f"absorption grid {n}^3 x {S} samples: step {ms:.2f} ms; k_trace per gen ms "
        f"{np.round(tr, 3).tolist()}; k_adjoint per gen ms {np.round(ad, 3).tolist()}")
    del buf
    return {"workload": f"torus-102k fwd+bwd as above with a {n}^3 RGB absorption grid, "
                        f"{S} samples per interior segment, grid gradient written",
            "ms_per_step": round(ms, 3), "Mrays/s": round(segs / ms / 1e3, 3),
            "k_trace_ms_per_generation": np.round(tr, 4).tolist(),
            "k_adjoint_ms_per_generation": np.round(ad, 4).tolist()}


def field_bench(args, dev, mesh, rays, env, ior, sigma, wl, cap, target, segs):
    """The torus fwd+bwd step with a volumetric exterior field: a seeded 32^3
    grid plus three 64^2 planes (4 channels: density before the softplus,
    colour) over a box 0.3 wider than the object on every side, 8 midpoint
    samples per exterior segment inside the box; the field's gradient is
    written every step."""
    import torch

    from paper_2603_00413_amd import binding as B
    n, res, S = 32, 64, 8
    rng = np.random.default_rng(11)
    grid = np.empty((n, n, n, 4), np.float32)
    grid[..., 0] = -1.5 + rng.normal(0.0, 0.6, (n, n, n))
    grid[..., 1:] = rng.uniform(0.0, 0.5, (n, n, n, 3))
    planes = np.empty((3, res, res, 4), np.float32)
    planes[..., 0] = rng.normal(0.0, 0.4, (3, res, res))
    planes[..., 1:] = rng.uniform(-0.1, 0.2, (3, res, res, 3))
    lo, hi = wl.V.min(0) - 0.3, wl.V.max(0) + 0.3
    field = B.Field(torch.from_numpy(grid).to(dev), torch.from_numpy(planes).to(dev), lo, hi, S)
    scene = B.Scene(mesh, ior, sigma, env, field=field)
    params = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=args.stride)
    buf = B.Buffers(params, rays, mesh, tape=True)

    def step():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        return B.dt_trace_backward(scene, rays, params, buf, (rgb - target) * (2.0 / rgb.numel()))

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    st = buf.stats.cpu().numpy()
    assert st[B.STAT_DROPPED] == 0 and int(st[B.STAT_TOTAL]) == segs
    timer = B.KernelTimer(wl.max_depth)
    pt = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=args.stride,
                  timing=timer)
    mesh.build()
    rgb, _, _ = B.dt_trace_forward(scene, rays, pt, buf, want_aux=False)
    B.dt_trace_backward(scene, rays, pt, buf, (rgb - target) * (2.0 / rgb.numel()))
    torch.cuda.synchronize()
    G = wl.max_depth + 1
    tr, ad = np.array(timer.trace_ms(G)), np.array(timer.adjoint_ms(G))
    assert torch.isfinite(field.d_grid).all() and float(field.d_grid.abs().sum()) > 0
    assert torch.isfinite(field.d_planes).all() and float(field.d_planes.abs().sum()) > 0
    log(f"volumetric field {n}^3 + 3 x {res}^2 x {S} samples: step {ms:.2f} ms; k_trace per gen ms "
        f"{np.round(tr, 3).tolist()}; k_adjoint per gen ms {np.round(ad, 3).tolist()}")
    del buf
    return {"workload": f"torus-102k fwd+bwd as above with a volumetric exterior field ({n}^3 grid + "
                        f"3 x {res}^2 planes, 4 channels, {S} samples per exterior segment in a box "
                        f"0.3 wider than the object), field gradient written",
            "ms_per_step": round(ms, 3), "Mrays/s": round(segs / ms / 1e3, 3),
            "k_trace_ms_per_generation": np.round(tr, 4).tolist(),
            "k_adjoint_ms_per_generation": np.round(ad, 4).tolist()}


def texel_grad_bench(args, dev, mesh, rays, ior, sigma, wl, cap, target, segs):
    """The torus fwd+bwd step with the gradient with respect to the 512x256
    equirect map's texels written as well."""
    import torch

    from paper_2603_00413_amd import binding as B
    env = B.Env(torch.from_numpy(wl.env).to(dev), want_grad=True)
    scene = B.Scene(mesh, ior, sigma, env)
    params = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=args.stride)
    buf = B.Buffers(params, rays, mesh, tape=True)

    def step():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        return B.dt_trace_backward(scene, rays, params, buf, (rgb - target) * (2.0 / rgb.numel()))

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    assert torch.isfinite(env.d_texels).all() and float(env.d_texels.abs().sum()) > 0
    log(f"texel gradient: step {ms:.2f} ms")
    del buf
    return {"workload": "torus-102k fwd+bwd with dLoss/dtexel of the 512x256 map",
            "ms_per_step": round(ms, 3), "Mrays/s": round(segs / ms / 1e3, 3)}


def mlp_flops(width, layers, in_dim=39):
    """Multiply-adds x 2 of one evaluation of the environment network:
    encoding (in_dim) -> layers x width (ReLU) -> 3."""
    return 2 * (in_dim * width + (layers - 1) * width * width + width * 3)


def training_step_bench(args, dev):
    """The training-step shape: SDF union (~300k triangles), 8 views x 800^2,
    depth 6, lit by the 3 x 64 environment MLP on bf16 MFMA; forward with tape,
    L2 loss gradient, adjoint.  Reports Mrays/s and the MLP kernels' achieved
    rate against the bf16 dense MFMA peak."""
    import torch

    from paper_2603_00413_amd import binding as B
    from paper_2603_00413_amd import synth
    wl = synth.sdf_union_scene()
    Ws, Bs, n_freq = wl.mlp
    layers, width = len(Ws) - 1, Ws[0].shape[0]
    V = torch.from_numpy(wl.V.astype(np.float32)).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    mesh = B.Mesh(V, F)
    env = B.Env.mlp(Ws, Bs, n_freq, dev)
    scene = B.Scene(mesh, torch.tensor([wl.ior], dtype=torch.float32, device=dev),
                    torch.tensor(wl.sigma, dtype=torch.float32, device=dev), env)
    rays = B.Rays(cameras=wl.cameras)
    cap = int(1.3 * rays.n_rays)
    while True:
        p = B.Params(max_depth=wl.max_depth, queue_capacity=cap)
        buf = B.Buffers(p, rays, mesh, tape=False)
        B.dt_trace_forward(scene, rays, p, buf, want_aux=False)
        st = buf.stats.cpu().numpy()
        if st[B.STAT_DROPPED] == 0:
            break
        cap *= 2
    del buf
    G = wl.max_depth + 1
    counts = st[:G].astype(np.int64)
    hits = st[B.STAT_HITS:B.STAT_HITS + G].astype(np.int64)
    segs = int(counts.sum())
    cap = int(max(counts[1:].max() * 1.05, 2048))
    timer = B.KernelTimer(wl.max_depth)
    params = B.Params(max_depth=wl.max_depth, queue_capacity=cap, timing=timer)
    buf = B.Buffers(params, rays, mesh, tape=True)
    tscene = B.Scene(mesh, torch.tensor([1.5], device=dev), torch.tensor([0.4, 0.25, 0.1], device=dev), env)
    target, _, _ = B.dt_trace_forward(tscene, rays, params, buf, want_aux=False)
    target = target.clone()

    def step():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        grad = (rgb - target) * (2.0 / rgb.numel())
        return B.dt_trace_backward(scene, rays, params, buf, grad)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    steps = max(3, args.steps // 2)
    fwd_ms, bwd_ms = np.zeros(G), np.zeros(G)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        torch.cuda.synchronize()
        fwd_ms += np.array(timer.mlp_ms(G)) / steps
        bwd_ms += np.array(timer.mlp_adjoint_ms(G)) / steps
    ms = 1e3 * (time.perf_counter() - t0) / steps
    st = buf.stats.cpu().numpy()
    assert st[B.STAT_DROPPED] == 0 and int(st[B.STAT_TOTAL]) == segs
    misses = counts - hits
    fl = mlp_flops(width, layers)
    # the forward kernel runs the network once per miss; the backward kernel
    # replays it and runs the transposed chain (about twice the multiply-adds)
    fwd_tf = misses.sum() * fl / (fwd_ms.sum() * 1e-3) / 1e12
    bwd_tf = misses.sum() * 2 * fl / (bwd_ms.sum() * 1e-3) / 1e12
    log(f"training step (MLP): {ms:.2f} ms, {segs / ms / 1e3:.1f} Mrays/s; MLP fwd kernels "
        f"{fwd_ms.sum():.3f} ms ({fwd_tf:.1f} TFLOP/s), bwd {bwd_ms.sum():.3f} ms ({bwd_tf:.1f} TFLOP/s)")
    return {
        "workload": "SDF union %d tris, %d views x %d^2, depth %d, env MLP %d x %d bf16 MFMA, fwd+bwd"
                    % (len(wl.F), len(wl.cameras), wl.cameras[0].width, wl.max_depth, layers, width),
        "ms_per_step": round(ms, 3),
        "Mrays/s": round(segs / ms / 1e3, 3),
        "segments_per_step": segs,
        "env_lookups_per_step": int(misses.sum()),
        "mlp_mfma": {
            "kernel": "k_mlp_trace_fwd",
            "achieved": round(float(fwd_tf), 2),
            "peak": 2500.0,
            "unit": "TFLOP/s",
            "frac": round(float(fwd_tf) / 2500.0, 5),
            "flops_per_lookup": fl,
            "ms_per_step": round(float(fwd_ms.sum()), 4),
            "backward_kernel_TFLOP/s": round(float(bwd_tf), 2),
            "backward_ms_per_step": round(float(bwd_ms.sum()), 4),
        },
    }


def trainer_bench(args, dev):
    """The ray-tracing stage's optimisation step at the training-step shape
    (`train.Trainer`): SDF union (~300k triangles), 8 views x 800^2, depth 6,
    lit by the 3 x 64 environment MLP whose weights are trained too (bf16
    MFMA forward, MFMA weight gradient); L_color + 0.1 L_tone against a target
    rendered with other material parameters (eta 1.5, sigma (0.4, 0.25, 0.1)),
    AdamUniform on the Laplacian reparameterisation of the vertices (lambda
    20), Adam on IoR, sigma and the network; every 10th step adds the
    periodic L_mask (outline gradient), L_edge and L_lap.  The BVH is rebuilt
    from the updated vertices every step."""
    import torch

    from paper_2603_00413_amd import autograd as A
    from paper_2603_00413_amd import binding as B
    from paper_2603_00413_amd import synth
    from paper_2603_00413_amd import train as T
    wl = synth.sdf_union_scene()
    Ws, Bs, n_freq = wl.mlp
    V0 = torch.from_numpy(wl.V.astype(np.float32)).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    env = B.Env.mlp(Ws, Bs, n_freq, dev, want_grad=True)
    tr = A.Tracer(F, env, wl.cameras, max_depth=wl.max_depth)
    w0 = torch.cat([torch.as_tensor(x).reshape(-1) for x in Ws]).to(dev)
    b0 = torch.cat([torch.as_tensor(x).reshape(-1) for x in Bs]).to(dev)
    with torch.no_grad():
        gt = A.render_mlp(V0, torch.tensor([1.5], device=dev), torch.tensor([0.4, 0.25, 0.1], device=dev),
                          w0, b0, tr).clone()
        gt_mask = A.render_mask(V0, tr).clone()
    V = V0.clone().requires_grad_(True)
    ior = torch.tensor([wl.ior], device=dev, requires_grad=True)
    sigma = torch.tensor(wl.sigma, dtype=torch.float32, device=dev, requires_grad=True)
    w = w0.clone().requires_grad_(True)
    b = b0.clone().requires_grad_(True)
    trainer = T.Trainer(tr, V, ior, sigma=sigma, lr=1e-3, l_color=1.0, l_tone=0.1, l_edge=0.01,
                        l_mask=0.1, l_lap=0.01, period=10, large_steps=20.0, lr_mesh=1e-3,
                        mlp=(w, b))
    for _ in range(2):
        trainer.step(gt, gt_mask)
    torch.cuda.synchronize()
    steps = 20
    t0 = time.perf_counter()
    for _ in range(steps):
        out = trainer.step(gt, gt_mask)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    st = tr.last_stats.numpy()
    segs = int(st[B.STAT_TOTAL])
    log(f"trainer step (training-step shape, MLP trained): {ms:.2f} ms, {segs / ms / 1e3:.1f} Mrays/s, "
        f"loss terms {out}")
    return {
        "workload": "Trainer: SDF union %d tris, %d views x %d^2, depth %d, env MLP 3 x 64 trained, "
                    "AdamUniform (lambda 20) on V, Adam on IoR / sigma / MLP, periodic L_mask + L_edge "
                    "+ L_lap every 10 steps, BVH rebuilt every step"
                    % (len(wl.F), len(wl.cameras), wl.cameras[0].width, wl.max_depth),
        "ms_per_step": round(ms, 3),
        "Mrays/s": round(segs / ms / 1e3, 3),
        "segments_per_step": segs,
        "checkpoint_stride": tr.stride,
    }


def stress_bench(args, dev):
    """The stress shape: thin-shell SDF mesh (~2M triangles, frequent TIR),
    one 2048^2 view, depth 8, environment MLP 4 x 128; forward with a tape
    every 2 generations, L2 loss gradient, adjoint recomputing the generations
    in between.  Reports Mrays/s, the ray queue's compaction efficiency (live
    rays over allocated slots, per generation) and the traversal kernel's
    achieved HBM rate."""
    import torch

    from paper_2603_00413_amd import binding as B
    from paper_2603_00413_amd import synth
    wl = synth.thin_shell_scene()
    Ws, Bs, n_freq = wl.mlp
    V = torch.from_numpy(wl.V.astype(np.float32)).to(dev)
    F = torch.from_numpy(wl.F).to(dev)
    mesh = B.Mesh(V, F)
    env = B.Env.mlp(Ws, Bs, n_freq, dev)
    scene = B.Scene(mesh, torch.tensor([wl.ior], dtype=torch.float32, device=dev),
                    torch.tensor(wl.sigma, dtype=torch.float32, device=dev), env)
    rays = B.Rays(cameras=wl.cameras)
    cap = int(1.3 * rays.n_rays)
    while True:
        p = B.Params(max_depth=wl.max_depth, queue_capacity=cap)
        buf = B.Buffers(p, rays, mesh, tape=False)
        B.dt_trace_forward(scene, rays, p, buf, want_aux=False)
        st = buf.stats.cpu().numpy()
        if st[B.STAT_DROPPED] == 0:
            break
        cap *= 2
    del buf
    G = wl.max_depth + 1
    counts = st[:G].astype(np.int64)
    hits = st[B.STAT_HITS:B.STAT_HITS + G].astype(np.int64)
    segs = int(counts.sum())
    cap = int(max(counts[1:].max() * 1.05, 2048))
    stride = 2
    timer = B.KernelTimer(wl.max_depth)
    params = B.Params(max_depth=wl.max_depth, queue_capacity=cap, checkpoint_stride=stride,
                      timing=timer)
    buf = B.Buffers(params, rays, mesh, tape=True)
    tscene = B.Scene(mesh, torch.tensor([1.55], device=dev), torch.tensor([0.2, 0.3, 0.4], device=dev),
                     env)
    target, _, _ = B.dt_trace_forward(tscene, rays, params, buf, want_aux=False)
    target = target.clone()

    def step():
        mesh.build()
        rgb, _, _ = B.dt_trace_forward(scene, rays, params, buf, want_aux=False)
        grad = (rgb - target) * (2.0 / rgb.numel())
        return B.dt_trace_backward(scene, rays, params, buf, grad)

    step()
    torch.cuda.synchronize()
    steps = 3
    tr_ms = np.zeros(G)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        torch.cuda.synchronize()
        tr_ms += np.array(timer.trace_ms(G)) / steps
    ms = 1e3 * (time.perf_counter() - t0) / steps
    st = buf.stats.cpu().numpy()
    assert st[B.STAT_DROPPED] == 0 and int(st[B.STAT_TOTAL]) == segs
    miss = counts - hits
    tr_bytes = counts * TRACE_PER_RAY + hits * TRACE_PER_HIT + miss * TRACE_PER_MISS
    gbs = float(tr_bytes.sum() / (tr_ms.sum() * 1e-3) / 1e9)
    # the queue of a generation is dense (stable compaction leaves no holes);
    # its allocation is the camera rays for generation 0, else the smaller of
    # the capacity and the worst case 2^g camera rays
    alloc = [rays.n_rays if g == 0 else min(cap, rays.n_rays << g) for g in range(G)]
    eff = [round(float(counts[g]) / alloc[g], 4) for g in range(G)]
    log(f"stress (thin shell): {len(wl.F)} tris, {ms:.2f} ms per step, {segs / ms / 1e3:.1f} Mrays/s; "
        f"live per generation {counts.tolist()} of capacity {cap}; k_trace {gbs:.1f} GB/s")
    return {
        "workload": "thin-shell SDF %d tris, 1 view x %d^2, depth %d, IoR %.2f, env MLP %d x %d bf16, "
                    "fwd+bwd with a tape every %d generations"
                    % (len(wl.F), wl.cameras[0].width, wl.max_depth, wl.ior, len(Ws) - 1, Ws[0].shape[0],
                       stride),
        "ms_per_step": round(ms, 3),
        "Mrays/s": round(segs / ms / 1e3, 3),
        "segments_per_step": segs,
        "queue": {"capacity": cap, "allocated_per_generation": alloc,
                  "live_per_generation": counts.tolist(), "compaction_efficiency": eff,
                  "hits_per_generation": hits.tolist()},
        "k_trace": {"ms_per_generation": np.round(tr_ms, 4).tolist(),
                    "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 5)},
    }


def serving_bench(args, dev):
    """Render server on four resident scenes under a Poisson request stream,
    against one-request-at-a-time plain tracing of the same stream: at
    saturation (every request waiting at t = 0) and at offered loads of 0.3,
    0.5, 0.7 and 0.9 of the one-at-a-time capacity."""
    from paper_2603_00413_amd import binding as B
    from paper_2603_00413_amd import synth
    from paper_2603_00413_amd.serve import Request, Server, run_fifo
    rng = np.random.default_rng(4)
    srv = Server(dev, queue_capacity=24 << 20, pixel_pool=24 << 20)
    sizes = (50_000, 150_000, 300_000, 500_000)
    nf = []
    for k, target in enumerate(sizes):
        V, F = synth.sdf_union_faces(target, seed=41 + k)
        nf.append(len(F))
        srv.add_scene(V, F, float(rng.uniform(1.37, 1.6)), tuple(rng.uniform(0.05, 0.5, 3)),
                      synth.env_equirect(512, 256, seed=100 + k))
    # relight targets: two maps and two environment MLPs
    relight = [srv.add_env(synth.env_equirect(512, 256, seed=200 + k)) for k in range(2)]
    for k, (layers, width) in enumerate([(3, 64), (2, 128)]):
        Wm, Bm = synth.env_mlp_weights(seed=210 + k, n_layers=layers, width=width)
        relight.append(srv.add_env(B.Env.mlp(Wm, Bm, 6, dev)))
    n_req = args.serve_requests
    eyes = synth.views_on_sphere(n_req, 3.0, seed=5)

    def make_stream(times):
        r2 = np.random.default_rng(6)
        out = []
        for i in range(n_req):
            res = int(r2.choice([128, 256, 512, 1024]))
            sc = int(r2.integers(0, 4))
            env = None if r2.uniform() < 0.7 else relight[int(r2.integers(0, 4))]
            out.append(Request(i, sc, synth.look_at_camera(eyes[i], res, res),
                               int(r2.integers(4, 9)), env, arrival=float(times[i])))
        return out

    def pct(reqs, q):
        return round(float(np.percentile(np.array([r.latency for r in reqs]) * 1e3, q)), 3)

    # one-at-a-time capacity: the same requests back to back
    warm = make_stream(np.zeros(n_req))[:16]
    run_fifo(srv, warm, realtime=False)
    srv.run(make_stream(np.zeros(n_req))[:16], realtime=True)
    t = time.perf_counter()
    _, traced_solo = run_fifo(srv, make_stream(np.zeros(n_req)), realtime=False)
    solo_s = time.perf_counter() - t
    mu = n_req / solo_s
    # saturation: the whole stream waiting at t = 0
    t = time.perf_counter()
    sat = srv.run(make_stream(np.zeros(n_req)), realtime=True)
    sat_s = time.perf_counter() - t
    assert all(r.image is not None for r in sat)
    saturation = {"server_Mrays/s": round(srv.traced / sat_s / 1e6, 2),
                  "server_requests_per_s": round(n_req / sat_s, 2),
                  "server_retries": srv.retries,
                  "fifo_Mrays/s": round(traced_solo / solo_s / 1e6, 2),
                  "fifo_requests_per_s": round(mu, 2)}
    log(f"serving: scenes {nf} faces; saturation: server {saturation['server_Mrays/s']} Mrays/s "
        f"({saturation['server_requests_per_s']} req/s), one at a time {saturation['fifo_Mrays/s']} "
        f"Mrays/s ({mu:.1f} req/s)")
    sweep = []
    for load in (0.3, 0.5, 0.7, 0.9):
        lam = load * mu
        arrivals = np.cumsum(np.random.default_rng(7).exponential(1.0 / lam, n_req))
        t = time.perf_counter()
        served = srv.run(make_stream(arrivals), realtime=True)
        span = time.perf_counter() - t
        t = time.perf_counter()
        fifo, traced_fifo = run_fifo(srv, make_stream(arrivals), realtime=True)
        span_f = time.perf_counter() - t
        row = {"load": load, "requests_per_s_offered": round(lam, 2),
               "p50_ms": pct(served, 50), "p99_ms": pct(served, 99),
               "Mrays/s": round(srv.traced / span / 1e6, 2), "device_steps": srv.steps,
               "retries": srv.retries,
               "fifo_p50_ms": pct(fifo, 50), "fifo_p99_ms": pct(fifo, 99),
               "fifo_Mrays/s": round(traced_fifo / span_f / 1e6, 2)}
        sweep.append(row)
        log(f"serving load {load}: p50 {row['p50_ms']} / p99 {row['p99_ms']} ms, {row['Mrays/s']} Mrays/s; "
            f"fifo p50 {row['fifo_p50_ms']} / p99 {row['fifo_p99_ms']} ms")
    head = next(r for r in sweep if r["load"] == args.serve_load) if args.serve_load in (0.3, 0.5, 0.7, 0.9) \
        else sweep[2]
    return {
        "workload": "4 resident SDF-union scenes (%s tris), Poisson stream of %d requests "
                    "(70%% render / 30%% relight on 2 maps and 2 MLPs, 128^2-1024^2, depth 4-8)"
                    % ("/".join(str(x) for x in nf), n_req),
        "load": head["load"],
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "Mrays/s": head["Mrays/s"],
        "fifo_plain_tracer": {"p50_ms": head["fifo_p50_ms"], "p99_ms": head["fifo_p99_ms"],
                              "Mrays/s": head["fifo_Mrays/s"]},
        "saturation": saturation,
        "load_sweep": sweep,
    }


def host_cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own timings, with the hardware they were taken on (its appendix
# on computational and training efficiency, and on implementation details):
# one NVIDIA RTX 3090 (24 GB) beside an Intel Core i7-10700K; training a scene
# takes 1-2 hours with batches of 5,000 rays and at most 4 bounces (8 at
# inference), using about 20 GB of GPU memory.  It states no rays-per-second
# figure, so there is no number for vs_baseline.
PAPER_TIMINGS = {
    "hardware": "1x NVIDIA RTX 3090 (24 GB), Intel Core i7-10700K, 64 GB RAM",
    "training_time_per_scene_h": [1, 2],
    "rays_per_batch": 5000,
    "max_bounces_training": 4,
    "max_bounces_inference": 8,
    "training_gpu_memory_GB": 20,
    "rays_per_second": None,
}


def cpu_baseline(wl, stride):
    """The FP64 oracle (forward + reverse-mode gradient) on a stratified
    sample of the same workload: every `stride`-th pixel in x and y of
    every view."""
    import oracle
    sc = oracle.Scene(wl.V, wl.F, wl.ior, wl.sigma, oracle.Env(tex=wl.env), wl.max_depth)
    o, d = [], []
    for cam in wl.cameras:
        oo, dd = oracle.camera_rays(cam)
        W, H = cam.width, cam.height
        sel = (np.arange(H)[:, None] % stride == 0) & (np.arange(W)[None, :] % stride == 0)
        sel = sel.reshape(-1)
        o.append(oo[sel])
        d.append(dd[sel])
    o, d = np.concatenate(o), np.concatenate(d)
    g = np.random.default_rng(0).normal(size=o.shape)
    segs = int(sc.trace(o, d)["nseg"].sum())     # segment count (not timed)
    t = time.perf_counter()
    sc.trace_grad(o, d, g)                        # forward + gradient on the tape
    el = time.perf_counter() - t
    log(f"cpu baseline: {len(o)} camera rays, {segs} segments, {el:.1f} s")
    return {"value": round(segs / el / 1e6, 4), "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": (f"every pixel of all {len(wl.cameras)} views" if stride == 1 else
                       f"every {stride}th pixel in x and y of all {len(wl.cameras)} views")
                      + f" ({len(o)} camera rays, {segs} segments); FP64 forward + reverse-mode "
                      f"gradient in one pass per camera ray",
            "seconds": round(el, 2)}


if __name__ == "__main__":
    main()
