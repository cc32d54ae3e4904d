"""The continuous-batching server.  Every served image matches the FP64
oracle per pixel (the tracer's bars, with the same flag, path-signature and
conditioning classification as the plain tracer's parity tests), and equals
the plain tracer's and its own render alone within 1e-6 relative, in a mix of
overlapping requests (scenes, environments, resolutions and depths differ);
admission waits for memory instead of failing, and a request that loses rays
to a full queue is traced again."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from paper_2603_00413_amd.serve import Request, Server, run_fifo
from tests.gpu_helpers import check_radiance, device

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _server(pool=1 << 20, cap=1 << 20):
    device()
    srv = Server(queue_capacity=cap, pixel_pool=pool)
    V1, F1 = synth.icosphere(3)
    V2, F2 = synth.displaced_torus(seed=5, nu=120, nv=60)
    srv.add_scene(V1, F1, 1.5, (0.5, 0.2, 0.1), synth.env_equirect(64, 32, seed=1))
    srv.add_scene(V2, F2, 1.45, 0.3, synth.env_equirect(128, 64, seed=2))
    relight = srv.add_env(synth.env_equirect(96, 48, seed=9))
    return srv, relight


def _requests(relight):
    eyes = synth.views_on_sphere(6, 3.0, seed=11)
    spec = [(0, 32, 4, None), (1, 48, 6, None), (0, 64, 5, relight), (1, 40, 3, relight),
            (1, 64, 7, None), (0, 24, 8, None)]
    out = []
    for k, (sc, res, dep, env) in enumerate(spec):
        out.append(Request(k, sc, synth.look_at_camera(eyes[k], res, res), dep, env,
                           arrival=1e-4 * (k // 2)))
    return out


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def test_alone_vs_mix_vs_plain_tracer():
    srv, relight = _server()
    mixed = srv.run(_requests(relight), realtime=False)
    assert srv.dropped == 0
    traced_mixed = srv.traced
    # the requests' device work overlapped
    overlap = any(a.admitted < b.finished and b.admitted < a.finished
                  for a in mixed for b in mixed if a is not b)
    assert overlap
    for r in _requests(relight):
        alone = srv.run([r], realtime=False)[0]
        m = mixed[r.rid]
        _print("request", r.rid, "alone vs mix", _rel(alone.image, m.image))
        assert _rel(alone.image, m.image) <= 1e-6
    fifo, traced = run_fifo(srv, _requests(relight), realtime=False)
    for f in fifo:
        _print("request", f.rid, "plain vs server", _rel(f.image, mixed[f.rid].image))
        assert _rel(f.image, mixed[f.rid].image) <= 1e-6
    # the same rays were intersected, one request at a time or all together
    assert traced == traced_mixed


def test_admission_waits_for_memory():
    """A pool that holds one 64x64 image at a time still serves everything."""
    srv, relight = _server(pool=64 * 64 + 10)
    reqs = srv.run(_requests(relight), realtime=False)
    assert all(r.finished is not None for r in reqs)
    order = sorted(reqs, key=lambda r: r.admitted)
    # never two 64x64 requests resident together
    big = [r for r in reqs if r.n_pixels == 64 * 64]
    assert not (big[0].admitted < big[1].finished and big[1].admitted < big[0].finished)
    ref = srv.run([_requests(relight)[2]], realtime=False)[0]
    assert _rel(ref.image, reqs[2].image) <= 1e-6


def test_mlp_environment_requests():
    """Requests lit by MLP environments (a scene's own and a relight target)
    mixed with map-lit ones: each image equals the plain tracer's and its own
    render alone, within 1e-6 relative."""
    dev = device()
    srv = Server(queue_capacity=1 << 20, pixel_pool=1 << 20)
    V1, F1 = synth.icosphere(3)
    V2, F2 = synth.displaced_torus(seed=5, nu=120, nv=60)
    W64, B64 = synth.env_mlp_weights(seed=3, n_layers=3, width=64)
    W128, B128 = synth.env_mlp_weights(seed=5, n_layers=2, width=128)
    srv.add_scene(V1, F1, 1.5, (0.5, 0.2, 0.1), B.Env.mlp(W64, B64, 6, dev))
    srv.add_scene(V2, F2, 1.45, 0.3, synth.env_equirect(128, 64, seed=2))
    relight = srv.add_env(B.Env.mlp(W128, B128, 6, dev))
    eyes = synth.views_on_sphere(5, 3.0, seed=13)
    spec = [(0, 40, 5, None), (1, 48, 6, relight), (0, 32, 4, relight), (1, 56, 7, None),
            (0, 24, 3, None)]

    def reqs():
        return [Request(k, sc, synth.look_at_camera(eyes[k], res, res), dep, env,
                        arrival=1e-4 * (k // 2))
                for k, (sc, res, dep, env) in enumerate(spec)]

    mixed = srv.run(reqs(), realtime=False)
    assert srv.dropped == 0
    for m in mixed:
        assert np.isfinite(m.image).all() and np.abs(m.image).max() > 0
    for r in reqs():
        alone = srv.run([r], realtime=False)[0]
        _print("mlp request", r.rid, "alone vs mix", _rel(alone.image, mixed[r.rid].image))
        assert _rel(alone.image, mixed[r.rid].image) <= 1e-6
    fifo, _ = run_fifo(srv, reqs(), realtime=False)
    for f in fifo:
        _print("mlp request", f.rid, "plain vs server", _rel(f.image, mixed[f.rid].image))
        assert _rel(f.image, mixed[f.rid].image) <= 1e-6


# ---------------------------------------------------------------- oracle parity of served images
def _oracle_env(spec):
    kind, data = spec
    if kind == "map":
        return oracle.Env(tex=data)
    Ws, Bs = data
    return oracle.Env(mlp=([w.astype(np.float64) for w in Ws], [b.astype(np.float64) for b in Bs], 6))


def check_served(r, scene, env_spec, pix=None, label=""):
    """One served request against the oracle, with the plain tracer's bars
    and classification (check_radiance).  scene = (V32, F, ior, sigma);
    env_spec = ("map", texels) or ("mlp", (weights, biases)).  pix: optional
    sample of the request's pixels."""
    V32, F, ior, sigma = scene
    orc = oracle.Scene(V32.astype(np.float64), F, float(np.float32(ior)),
                       np.broadcast_to(np.asarray(sigma, np.float32), (3,)).astype(np.float64),
                       _oracle_env(env_spec), r.max_depth)
    o, d = oracle.camera_rays(r.camera)
    img, fl, sig = r.image, r.flags, r.sig
    if pix is not None:
        o, d, img, fl, sig = o[pix], d[pix], img[pix], fl[pix], sig[pix]
    return check_radiance(orc, o, d, img, fl, sig, mlp=env_spec[0] == "mlp", label=f"served {label}")


def test_served_images_match_the_oracle():
    """Map- and MLP-lit scenes, render and relight requests, depths 3-8, all
    in one stream; each served image against the oracle."""
    dev = device()
    srv = Server(queue_capacity=1 << 20, pixel_pool=1 << 20)
    V1, F1 = synth.icosphere(3)
    V2, F2 = synth.displaced_torus(seed=5, nu=120, nv=60)
    W64, B64 = synth.env_mlp_weights(seed=3, n_layers=3, width=64)
    W128, B128 = synth.env_mlp_weights(seed=5, n_layers=2, width=128)
    map1, map2, map3 = (synth.env_equirect(64, 32, seed=1), synth.env_equirect(128, 64, seed=2),
                        synth.env_equirect(96, 48, seed=9))
    scenes = [(V1.astype(np.float32), F1, 1.5, (0.5, 0.2, 0.1)),
              (V2.astype(np.float32), F2, 1.45, 0.3),
              (V1.astype(np.float32), F1, 1.4, (0.1, 0.3, 0.2))]
    srv.add_scene(*scenes[0], map1)
    srv.add_scene(*scenes[1], map2)
    srv.add_scene(*scenes[2], B.Env.mlp(W64, B64, 6, dev))
    env_map = srv.add_env(map3)
    env_mlp = srv.add_env(B.Env.mlp(W128, B128, 6, dev))
    specs = {0: ("map", map1), 1: ("map", map2), 2: ("mlp", (W64, B64)), env_map: ("map", map3),
             env_mlp: ("mlp", (W128, B128))}
    own = {0: 0, 1: 1, 2: 2}
    eyes = synth.views_on_sphere(9, 3.0, seed=21)
    plan = [(0, 48, 3, None), (1, 40, 8, None), (2, 32, 5, None), (0, 40, 6, env_mlp),
            (1, 32, 4, env_map), (2, 24, 7, env_map), (1, 48, 6, env_mlp), (0, 24, 8, None),
            (2, 40, 4, env_mlp)]
    reqs = [Request(k, sc, synth.look_at_camera(eyes[k], res, res), dep, env, arrival=2e-4 * (k // 3))
            for k, (sc, res, dep, env) in enumerate(plan)]
    served = srv.run(reqs, realtime=False)
    assert all(r.retries == 0 for r in served) and srv.dropped == 0
    for r in served:
        e = srv.scene_env[r.scene] if r.env is None else r.env
        check_served(r, scenes[r.scene], specs[e],
                     label=f"req {r.rid} scene {r.scene} env {e} depth {r.max_depth}")


def test_served_images_at_stream_shape_sampled():
    """The benchmark's serving shape: four resident SDF-union scenes of 50k,
    150k, 300k and 500k faces, requests of 128^2-1024^2 at depths 4-8, render
    and relight with map and MLP environments, served together; 1,500 pixels
    of each image checked against the oracle one by one."""
    dev = device()
    rng = np.random.default_rng(4)
    srv = Server(queue_capacity=12 << 20, pixel_pool=8 << 20)
    scenes, specs = [], {}
    for k, target in enumerate((50_000, 150_000, 300_000, 500_000)):
        V, F = synth.sdf_union_faces(target, seed=41 + k)
        sc = (V.astype(np.float32), F, float(rng.uniform(1.37, 1.6)), tuple(rng.uniform(0.05, 0.5, 3)))
        scenes.append(sc)
        tex = synth.env_equirect(512, 256, seed=100 + k)
        srv.add_scene(*sc, tex)
        specs[k] = ("map", tex)
    tex = synth.env_equirect(512, 256, seed=200)
    specs[srv.add_env(tex)] = ("map", tex)
    Wm, Bm = synth.env_mlp_weights(seed=201, n_layers=3, width=64)
    specs[srv.add_env(B.Env.mlp(Wm, Bm, 6, dev))] = ("mlp", (Wm, Bm))
    eyes = synth.views_on_sphere(8, 3.0, seed=5)
    plan = [(0, 128, 4, None), (1, 256, 8, 4), (2, 512, 6, None), (3, 1024, 5, 5),
            (3, 256, 7, None), (2, 128, 8, 5), (1, 512, 4, None), (0, 1024, 6, 4)]
    reqs = [Request(k, sc, synth.look_at_camera(eyes[k], res, res), dep, env, arrival=0.0)
            for k, (sc, res, dep, env) in enumerate(plan)]
    served = srv.run(reqs, realtime=False)
    ps = np.random.default_rng(9)
    for r in served:
        e = srv.scene_env[r.scene] if r.env is None else r.env
        pix = np.sort(ps.choice(r.n_pixels, min(1500, r.n_pixels), replace=False))
        check_served(r, scenes[r.scene], specs[e], pix=pix,
                     label=f"req {r.rid} {r.camera.width}^2 scene {r.scene} env {e} depth {r.max_depth}")


def test_lost_rays_are_traced_again():
    """A queue too small for the mix: rays are lost, the requests that lost
    them are traced again, and every returned image equals the request's
    render alone in a roomy queue."""
    device()
    srv, relight = _server(cap=9000)
    srv.default_growth = 1.0           # reserve too little at first
    reqs = srv.run(_requests(relight), realtime=False)
    assert srv.retries > 0
    big, _ = _server()
    for r in _requests(relight):
        ref = big.run([r], realtime=False)[0]
        assert _rel(ref.image, reqs[r.rid].image) <= 1e-6
        assert not (reqs[r.rid].flags & B.FLAG_OVERFLOW).any()
