"""The continuous-batching server: every request's image equals the plain
tracer's, alone and in a mix of overlapping requests (scenes, environments,
resolutions and depths differ), within 1e-6 relative; admission waits for
memory instead of failing."""
import numpy as np
import pytest
import torch

from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import synth
from paper_2603_00413_amd.serve import Request, Server, run_fifo
from tests.gpu_helpers import device

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
