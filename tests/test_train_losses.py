"""The training-step losses (Sec. 3.3 "Optimization" and the appendix's
regularizers) against their definitions written out in numpy, and the
torch vertex normals against the oracle's (an independent implementation of
Eq. 12-13)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_00413_amd import synth
from paper_2603_00413_amd import train as T


def test_color_and_tone_losses():
    rng = np.random.default_rng(0)
    p, g = rng.uniform(0.01, 1, (50, 3)), rng.uniform(0.01, 1, (50, 3))
    col = np.mean(np.sum(((p - g) * g) ** 2, axis=1))
    cos = np.sum(p * g, 1) / (np.linalg.norm(p, axis=1) * np.linalg.norm(g, axis=1))
    tone = np.mean((1 - cos) ** 2 - np.var(g, axis=1))
    pt, gt = torch.from_numpy(p), torch.from_numpy(g)
    assert abs(float(T.color_loss(pt, gt)) - col) < 1e-14
    assert abs(float(T.tone_loss(pt, gt)) - tone) < 1e-14
    assert abs(float(T.tone_loss(gt * 3.0, gt)) + np.mean(np.var(g, axis=1))) < 1e-14  # same tone


def test_grid_rate_reproduces_linear_fields_and_clamps():
    lo, hi, n = (-1.0, -0.5, -2.0), (1.0, 1.5, 0.0), (5, 4, 3)
    xs = [np.linspace(lo[a], hi[a], n[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    lin = lambda x, y, z: np.stack([0.3 + 0.2 * x - 0.1 * z, 0.5 * y, 0.7 + 0 * x], -1)
    mu = torch.from_numpy(lin(X, Y, Z))
    pts = np.random.default_rng(1).uniform([-1, -0.5, -2], [1, 1.5, 0], (200, 3))
    got = T.grid_rate(mu, lo, hi, torch.from_numpy(pts)).numpy()
    np.testing.assert_allclose(got, lin(pts[:, 0], pts[:, 1], pts[:, 2]), atol=1e-14)
    out = np.array([[5.0, 0.2, -1.0]])                     # beyond hi in x: clamped
    edge = np.array([[1.0, 0.2, -1.0]])
    np.testing.assert_allclose(T.grid_rate(mu, lo, hi, torch.from_numpy(out)).numpy(),
                               T.grid_rate(mu, lo, hi, torch.from_numpy(edge)).numpy(), atol=1e-15)


def test_material_regularizers_on_constant_grids():
    mu = torch.full((3, 4, 5, 3), 0.25, dtype=torch.float64) * torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64)
    pts = torch.rand(100, 3, dtype=torch.float64) * 2 - 1
    xi = torch.rand(100, 3, dtype=torch.float64) * 0.1
    lo, hi = (-1, -1, -1), (1, 1, 1)
    assert float(T.mat_smooth_loss(mu, lo, hi, pts, xi)) < 1e-15   # weights sum to 1 up to rounding
    assert abs(float(T.vol_loss(mu, lo, hi, pts)) - 100 * 0.0625 * 14) < 1e-12


def test_vertex_normals_match_the_oracle_and_edge_loss():
    V, F = synth.icosphere(2)
    n = T.vertex_normals(torch.from_numpy(V), torch.from_numpy(F)).numpy()
    np.testing.assert_allclose(n, oracle.vertex_normals(V, F), atol=1e-13)
    assert float(T.edge_loss(torch.from_numpy(V), torch.from_numpy(F))) > 0.0
    # a flat sheet: every normal is +z, the edge term vanishes
    g = np.stack(np.meshgrid(np.arange(4.0), np.arange(4.0), indexing="ij"), -1).reshape(-1, 2)
    Vp = np.concatenate([g, np.zeros((16, 1))], 1)
    Fp = np.array([[i * 4 + j, (i + 1) * 4 + j, i * 4 + j + 1] for i in range(3) for j in range(3)] +
                  [[(i + 1) * 4 + j, (i + 1) * 4 + j + 1, i * 4 + j + 1] for i in range(3) for j in range(3)])
    assert float(T.edge_loss(torch.from_numpy(Vp), torch.from_numpy(Fp))) < 1e-28


def test_laplacian_and_large_steps_roundtrip():
    V, F = synth.icosphere(2)
    Ft = torch.from_numpy(F)
    L = T.laplacian(len(V), Ft).to_dense().numpy()
    assert np.allclose(L, L.T) and np.abs(L.sum(1)).max() == 0.0
    deg = np.diag(L)
    assert deg.min() >= 5 and deg.max() <= 6          # icosphere valences
    # the CSR adjacency the device solve takes: the off-diagonal pattern of L,
    # neighbours ascending, degrees the diagonal
    off, adj = T.adjacency_csr(len(V), Ft)
    assert off.dtype == torch.int32 and adj.dtype == torch.int32
    off, adj = off.numpy(), adj.numpy()
    assert off[0] == 0 and off[-1] == len(adj) and np.array_equal(np.diff(off), deg.astype(np.int64))
    A = np.zeros_like(L)
    for i in range(len(V)):
        nb = adj[off[i]:off[i + 1]]
        assert np.all(np.diff(nb) > 0)
        A[i, nb] = 1.0
    np.testing.assert_array_equal(np.diag(deg) - A, L)
    # the solve is device-only: no host fallback
    with pytest.raises(ValueError, match="device"):
        T.LargeSteps(len(V), Ft, lam=10.0)


def test_adam_uniform_step_matches_its_definition():
    g = torch.tensor([[0.5, -2.0], [1.0, 0.25]], dtype=torch.float64)
    p = torch.zeros(2, 2, dtype=torch.float64, requires_grad=True)
    opt = T.AdamUniform([p], lr=0.1)
    for t in (1, 2):
        p.grad = g.clone()
        opt.step()
    # two identical gradients: m_hat = g, v_hat = g^2, step = lr g / max|g| each time
    expect = -2 * 0.1 * g.numpy() / (np.abs(g.numpy()).max() + 1e-8)
    np.testing.assert_allclose(p.detach().numpy(), expect, rtol=1e-12)


def test_uniform_laplacian_loss():
    """(L V)_i = V_i - mean of its neighbours: zero at the centre of a regular
    hexagon fan, the same for a translated mesh (rows sum to zero), and the
    loss scales with the square of a scaling of the mesh."""
    ang = np.arange(6) * np.pi / 3
    V = np.concatenate([[[0.0, 0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang), 0 * ang], 1)])
    F = np.array([[0, 1 + k, 1 + (k + 1) % 6] for k in range(6)], np.int32)
    Vt = torch.tensor(V, dtype=torch.float32)
    Ft = torch.from_numpy(F)
    Lu = T.uniform_laplacian(7, Ft)
    LV = torch.sparse.mm(Lu, Vt)
    assert torch.abs(LV[0]).max() < 1e-7
    # a rim vertex: neighbours are the centre and its two rim neighbours
    np.testing.assert_allclose(LV[1].numpy(), V[1] - (V[0] + V[2] + V[6]) / 3, atol=1e-6)
    l0 = T.lap_loss(Vt, Lu)
    assert abs(float(T.lap_loss(Vt + torch.tensor([0.3, -2.0, 5.0]), Lu)) - float(l0)) < 1e-5
    assert abs(float(T.lap_loss(3.0 * Vt, Lu)) - 9.0 * float(l0)) < 1e-5 * float(l0) * 9
