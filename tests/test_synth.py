"""Seeded input generators: determinism, closed oriented meshes, sizes."""
import numpy as np

from paper_2603_00413_amd import synth


def test_icosphere_counts_and_topology():
    V, F = synth.icosphere(3)
    assert V.shape == (642, 3) and F.shape == (1280, 3)
    st = synth.mesh_stats(V, F)
    assert st["closed_manifold"] and st["consistently_oriented"] and st["euler"] == 2
    np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-15)


def test_torus_counts_genus_and_bounds():
    V, F = synth.displaced_torus(seed=2)
    assert V.shape == (51200, 3) and F.shape == (102400, 3)
    st = synth.mesh_stats(V, F)
    assert st["closed_manifold"] and st["consistently_oriented"] and st["euler"] == 0
    assert np.linalg.norm(V, axis=1).max() < 1.0
    V2, F2 = synth.displaced_torus(seed=2)
    assert np.array_equal(V, V2) and np.array_equal(F, F2)


def test_outward_orientation_positive_volume():
    for V, F in [synth.icosphere(2), synth.displaced_torus(seed=3, nu=40, nv=20),
                 synth.sdf_union_mesh(seed=3, res=40)]:
        a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
        vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
        assert vol > 0


def test_sdf_union_closed_genus():
    V, F = synth.sdf_union_mesh(seed=3, res=64)
    st = synth.mesh_stats(V, F)
    assert st["closed_manifold"] and st["consistently_oriented"]
    assert st["genus_if_connected"] >= 3 or st["euler"] <= -4
    assert np.linalg.norm(V, axis=1).max() < 1.0
    V2, F2 = synth.sdf_union_mesh(seed=3, res=64)
    assert np.array_equal(V, V2) and np.array_equal(F, F2)


def test_env_and_cameras():
    e = synth.env_equirect(64, 32, seed=1)
    assert e.shape == (32, 64, 3) and e.dtype == np.float32 and (e > 0).all()
    assert np.array_equal(e, synth.env_equirect(64, 32, seed=1))
    eyes = synth.views_on_sphere(8, 3.0, seed=2)
    np.testing.assert_allclose(np.linalg.norm(eyes, axis=1), 3.0)
    cam = synth.look_at_camera((0.0, 3.0, 0.0), 8, 8)
    assert cam.up == (0.0, 0.0, 1.0)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 1e-3], np.float32)
    r = synth.round_to_bf16(x)
    assert (r.view(np.uint32) & 0xFFFF == 0).all()
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert r[1] == 1.0
    assert abs(r[3] - x[3]) <= 2 ** -8 * abs(x[3])
