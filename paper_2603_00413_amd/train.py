"""Training-step pieces around the tracer (Sec. 3.3 "Optimization", and the
regularizers of the appendix on the ray tracer's optimization).

The tracer returns pixel colours and, through `autograd.render` /
`autograd.render_grid`, their gradients; this module holds the losses the
paper puts on those colours and on the parameters, and a step that renders,
adds the losses up and updates the parameters:

* L_color: per pixel the squared norm of (c_hat - c) * c (the error weighted
  by the ground-truth colour, so over-absorbed dark pixels weigh less),
  averaged over the batch;
* L_tone: (1 - cos(c_hat, c))^2 - var(c) per pixel, var the variance of c's
  three channels (a constant: it shifts the loss, not its gradient);
* L_mat-smooth: mean over sample points of |mu(v) - mu(v + xi)| (L1 over the
  channels) for the absorption grid;
* L_vol: sum over sample points of ||mu(x)||^2;
* L_edge: mean over mesh edges of (1 - n_i . n_j)^2 with the unit vertex
  normals;
* L_lap: mean over vertices of ||(L V)_i||^2 with the uniform Laplacian
  (L V)_i = V_i - mean of V_i's neighbours (the uniformity term of the large-
  steps paper the appendix cites);
* L_mask: mean over pixels of (M_p - M*_p)^2, M the object's coverage with
  the outline (silhouette) gradient of `autograd.render_mask`.
L_mask, L_edge and L_lap are the periodic regularization of the appendix
("Periodical Regularization"): added every `period`-th step.

The vertices are optimised either with plain Adam or, as in the paper, with
AdamUniform on the Laplacian reparameterisation u = (I + lambda L) V (below);
the other parameters with Adam, the environment MLP's float32 parameters
included when given.
"""
from __future__ import annotations

import torch

from . import autograd as A
from . import binding as B


def color_loss(pred: torch.Tensor, gt: torch.Tensor) -> torch.Tensor:
    """mean_i ||(c_hat_i - c_i) * c_i||^2 over pixels [n, 3]."""
    return (((pred - gt) * gt) ** 2).sum(-1).mean()


def tone_loss(pred: torch.Tensor, gt: torch.Tensor, eps: float = 1e-12) -> torch.Tensor:
    """mean_i (1 - cos(c_hat_i, c_i))^2 - var(c_i), var over the 3 channels."""
    cos = (pred * gt).sum(-1) / (pred.norm(dim=-1) * gt.norm(dim=-1)).clamp_min(eps)
    return ((1.0 - cos) ** 2 - gt.var(dim=-1, unbiased=False)).mean()


def grid_rate(mu: torch.Tensor, lo, hi, x: torch.Tensor) -> torch.Tensor:
    """The absorption grid's rate at points x [n, 3]: trilinear over mu
    [nz, ny, nx, 3] on the box [lo, hi], x clamped into the box (the same
    definition the tracer uses)."""
    nz, ny, nx, _ = mu.shape
    n = torch.tensor([nx, ny, nz], dtype=x.dtype, device=x.device)
    lo_t = torch.as_tensor(lo, dtype=x.dtype, device=x.device)
    hi_t = torch.as_tensor(hi, dtype=x.dtype, device=x.device)
    u = ((x - lo_t) * (n - 1) / (hi_t - lo_t)).clamp(min=0.0)
    u = torch.minimum(u, n - 1)
    i = torch.minimum(u.floor(), n - 2).long()
    f = u - i.to(x.dtype)
    out = torch.zeros(x.shape[0], 3, dtype=mu.dtype, device=x.device)
    for c in range(8):
        dx, dy, dz = c & 1, (c >> 1) & 1, c >> 2
        w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) *
             (f[:, 2] if dz else 1 - f[:, 2]))
        out = out + w[:, None] * mu[i[:, 2] + dz, i[:, 1] + dy, i[:, 0] + dx]
    return out


def mat_smooth_loss(mu, lo, hi, pts: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
    """mean_i |mu(v_i) - mu(v_i + xi_i)| (L1 over the channels)."""
    return (grid_rate(mu, lo, hi, pts) - grid_rate(mu, lo, hi, pts + xi)).abs().sum(-1).mean()


def vol_loss(mu, lo, hi, pts: torch.Tensor) -> torch.Tensor:
    """sum_i ||mu(x_i)||^2."""
    return (grid_rate(mu, lo, hi, pts) ** 2).sum()


def vertex_normals(V: torch.Tensor, F: torch.Tensor) -> torch.Tensor:
    """One third of the sum of the unit normals of the faces around each
    vertex (Eq. 13, the vertex normals the tracer blends), differentiable in
    V."""
    F = F.long()
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    fn = torch.cross(e1, e2, dim=-1)
    fn = fn / fn.norm(dim=-1, keepdim=True).clamp_min(1e-30)
    acc = torch.zeros_like(V)
    for k in range(3):
        acc = acc.index_add(0, F[:, k], fn)
    return acc / 3.0


def mesh_edges(F: torch.Tensor) -> torch.Tensor:
    """Unique undirected edges [m, 2] of a triangle list."""
    F = F.long()
    e = torch.cat([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = torch.sort(e, dim=1).values
    return torch.unique(e, dim=0)


def edge_loss(V: torch.Tensor, F: torch.Tensor, edges: torch.Tensor | None = None) -> torch.Tensor:
    """mean over edges (i, j) of (1 - n_i . n_j)^2, n the unit vertex normals
    (the direction of Eq. 13's normal, so the dot product is a cosine)."""
    if edges is None:
        edges = mesh_edges(F)
    n = vertex_normals(V, F)
    n = n / n.norm(dim=-1, keepdim=True).clamp_min(1e-30)
    return ((1.0 - (n[edges[:, 0]] * n[edges[:, 1]]).sum(-1)) ** 2).mean()


def uniform_laplacian(nv: int, F: torch.Tensor) -> torch.Tensor:
    """I - D^-1 A of the mesh's edge graph, sparse [nv, nv] float32."""
    e = mesh_edges(F)
    i = torch.cat([e[:, 0], e[:, 1]])
    j = torch.cat([e[:, 1], e[:, 0]])
    ones = torch.ones(i.shape[0], dtype=torch.float32, device=F.device)
    deg = torch.zeros(nv, dtype=torch.float32, device=F.device).index_add(0, i, ones)
    d = torch.arange(nv, device=F.device)
    idx = torch.cat([torch.stack([i, j]), torch.stack([d, d])], 1)
    val = torch.cat([-ones / deg[i], torch.ones(nv, dtype=torch.float32, device=F.device)])
    return torch.sparse_coo_tensor(idx, val, (nv, nv)).coalesce()


def lap_loss(V: torch.Tensor, Lu: torch.Tensor) -> torch.Tensor:
    """mean_i ||(L V)_i||^2 with the uniform Laplacian Lu."""
    return (torch.sparse.mm(Lu, V) ** 2).sum(-1).mean()


def mask_loss(pred: torch.Tensor, gt: torch.Tensor) -> torch.Tensor:
    """mean_p (M_p - M*_p)^2."""
    return ((pred - gt) ** 2).mean()


class Trainer:
    """One optimisation step of the paper's ray-tracing stage: render with the
    current parameters, L_total = l_color L_color + l_tone L_tone (+ l_smooth
    L_mat-smooth + l_vol L_vol with an absorption grid) + l_edge L_edge, and
    update every parameter given as a tensor with requires_grad: Adam, or for
    the vertices with large_steps = lambda, AdamUniform on u = (I + lambda L) V
    at learning rate lr_mesh."""

    def __init__(self, tracer: A.Tracer, V: torch.Tensor, ior: torch.Tensor,
                 sigma: torch.Tensor | None = None, grid=None, lr: float = 1e-3,
                 l_color: float = 1.0, l_tone: float = 0.0, l_smooth: float = 0.0,
                 l_vol: float = 0.0, l_edge: float = 0.0, n_points: int = 4096, seed: int = 0,
                 large_steps: float | None = None, lr_mesh: float = 1e-3, mlp=None,
                 l_mask: float = 0.0, l_lap: float = 0.0, period: int = 1, mask_rho: float = 2.0):
        """grid: (mu, lo, hi, samples) with mu a leaf tensor [nz, ny, nx, 3].
        mlp: (weights, biases) float32 leaf tensors of the tracer's MLP
        environment (made with want_grad=True).  L_mask, L_edge and L_lap are
        added on every `period`-th step (counting from the first)."""
        self.tracer, self.V, self.ior, self.sigma, self.grid = tracer, V, ior, sigma, grid
        self.mlp = mlp
        self.period, self.mask_rho, self.t = max(int(period), 1), mask_rho, 0
        self.w = dict(color=l_color, tone=l_tone, smooth=l_smooth, vol=l_vol, edge=l_edge,
                      mask=l_mask, lap=l_lap)
        self.Lu = uniform_laplacian(V.shape[0], tracer.F) if l_lap else None
        self.ls, self.u, self.opt_mesh = None, None, None
        if large_steps is not None and V.requires_grad:
            self.ls = LargeSteps(V.shape[0], tracer.F, large_steps)
            self.u = self.ls.to_u(V.detach()).requires_grad_(True)
            self.opt_mesh = AdamUniform([self.u], lr=lr_mesh)
        params = [p for p in (None if self.ls else V, ior, sigma, grid[0] if grid else None,
                              *(mlp or ()))
                  if p is not None and p.requires_grad]
        self.opt = torch.optim.Adam(params, lr=lr) if params else None
        self.n_points = n_points
        self.gen = torch.Generator(device=V.device).manual_seed(seed)
        self.edges = mesh_edges(tracer.F) if l_edge else None

    def _points(self, lo, hi):
        lo_t = torch.as_tensor(lo, dtype=torch.float32, device=self.V.device)
        hi_t = torch.as_tensor(hi, dtype=torch.float32, device=self.V.device)
        r = torch.rand(self.n_points, 3, generator=self.gen, device=self.V.device)
        return lo_t + r * (hi_t - lo_t), (hi_t - lo_t)

    def step(self, gt: torch.Tensor, gt_mask: torch.Tensor | None = None) -> dict:
        """One step against target colours gt [n_pixels, 3] (and, for L_mask,
        the target coverage gt_mask [n_pixels])."""
        for o in (self.opt, self.opt_mesh):
            if o is not None:
                o.zero_grad(set_to_none=True)
        if self.ls is not None:
            self.V = _FromU.apply(self.u, self.ls)
        periodic = self.t % self.period == 0
        self.t += 1
        terms = {}
        if periodic and self.w["mask"]:
            if gt_mask is None:
                raise ValueError("L_mask needs the target mask")
            terms["mask"] = mask_loss(A.render_mask(self.V, self.tracer, self.mask_rho), gt_mask)
        if self.grid is not None:
            mu, lo, hi, samples = self.grid
            pred = A.render_grid(self.V, self.ior, mu, self.tracer, lo, hi, samples)
        elif self.mlp is not None:
            sg = self.sigma.expand(3) if self.sigma.numel() == 1 else self.sigma
            pred = A.render_mlp(self.V, self.ior, sg, self.mlp[0], self.mlp[1], self.tracer)
        else:
            pred = A.render(self.V, self.ior, self.sigma, self.tracer)
        terms["color"] = color_loss(pred, gt)
        if self.w["tone"]:
            terms["tone"] = tone_loss(pred, gt)
        if self.grid is not None and (self.w["smooth"] or self.w["vol"]):
            pts, ext = self._points(lo, hi)
            if self.w["smooth"]:
                xi = (torch.rand(pts.shape, generator=self.gen, device=pts.device) - 0.5) * 0.02 * ext
                terms["smooth"] = mat_smooth_loss(mu, lo, hi, pts, xi)
            if self.w["vol"]:
                terms["vol"] = vol_loss(mu, lo, hi, pts)
        if periodic and self.w["edge"]:
            terms["edge"] = edge_loss(self.V, self.tracer.F, self.edges)
        if periodic and self.w["lap"]:
            terms["lap"] = lap_loss(self.V, self.Lu)
        total = sum(self.w[k] * v for k, v in terms.items())
        total.backward()
        for o in (self.opt, self.opt_mesh):
            if o is not None:
                o.step()
        if self.ls is not None:
            # the mesh the next render will see, so that self.V never lags u
            with torch.no_grad():
                self.V = self.ls.to_v(self.u.detach())
        out = {k: float(v.detach()) for k, v in terms.items()}
        out["total"] = float(total.detach())
        return out


# ---------------------------------------------------------------- AdamUniform
# The mesh optimiser the paper adopts (Nicolet, Jacobson and Jakob, "Large
# Steps in Inverse Rendering of Geometry", SIGGRAPH Asia 2021): the vertices
# are reparameterised as u = (I + lambda L) V with L the combinatorial graph
# Laplacian of the mesh, u is updated by Adam whose step is scaled uniformly
# (the second-moment estimate is replaced by its maximum over the whole
# parameter, so every entry moves at the same rate), and V is recovered by
# solving (I + lambda L) V = u.


def laplacian(nv: int, F: torch.Tensor) -> torch.Tensor:
    """Combinatorial Laplacian D - A of the mesh's edge graph, sparse [nv, nv]."""
    e = mesh_edges(F)
    i = torch.cat([e[:, 0], e[:, 1]])
    j = torch.cat([e[:, 1], e[:, 0]])
    ones = torch.ones(i.shape[0], dtype=torch.float64, device=F.device)
    deg = torch.zeros(nv, dtype=torch.float64, device=F.device).index_add(0, i, ones)
    d = torch.arange(nv, device=F.device)
    idx = torch.cat([torch.stack([i, j]), torch.stack([d, d])], 1)
    val = torch.cat([-ones, deg])
    return torch.sparse_coo_tensor(idx, val, (nv, nv)).coalesce()


def adjacency_csr(nv: int, F: torch.Tensor) -> tuple[torch.Tensor, torch.Tensor]:
    """The edge graph as int32 CSR: off [nv + 1], adj [2 m] with vertex i's
    neighbours (ascending) in adj[off[i]:off[i + 1]], every edge from both ends."""
    e = mesh_edges(F)
    i = torch.cat([e[:, 0], e[:, 1]])
    j = torch.cat([e[:, 1], e[:, 0]])
    order = torch.argsort(i * nv + j)
    off = torch.zeros(nv + 1, dtype=torch.int64, device=F.device)
    off[1:] = torch.cumsum(torch.bincount(i, minlength=nv), 0)
    return off.to(torch.int32), j[order].to(torch.int32)


class LargeSteps:
    """u = (I + lam L) V and back, for one mesh on the device; the solve runs
    in the library's Chebyshev-iteration kernels (float64, to a relative
    residual of 1e-10 per coordinate column), each from the previous solve of
    its kind: vertices from the last vertices, a gradient from the last
    gradient."""

    def __init__(self, nv: int, F: torch.Tensor, lam: float, tol: float = 1e-10, max_iters: int = 1000):
        if not F.is_cuda:
            raise ValueError("LargeSteps solves on the device: F must be a device tensor")
        self.L = laplacian(nv, F)
        self.lam, self.tol, self.max_iters = lam, tol, max_iters
        self.solver = B.Smooth(*adjacency_csr(nv, F), lam)
        self._last = {}        # the previous solve of each kind: the next one starts there

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        return x + self.lam * torch.sparse.mm(self.L, x)

    def to_u(self, V: torch.Tensor) -> torch.Tensor:
        return self.matvec(V.double()).to(V.dtype)

    def to_v(self, u: torch.Tensor, slot: str | None = "v") -> torch.Tensor:
        """(I + lam L)^-1 u, started from the last solution kept under `slot`
        (None: from zero, nothing kept)."""
        b = u.detach().double().contiguous()
        x0 = self._last.get(slot) if slot is not None else None
        x = x0.clone() if x0 is not None and x0.shape == b.shape else torch.zeros_like(b)
        self.solver.solve(b, x, tol=self.tol, max_iters=self.max_iters)
        if slot is not None:
            self._last[slot] = x
        return x.to(u.dtype)


class AdamUniform(torch.optim.Optimizer):
    """Adam with a uniform step: the bias-corrected second moment is replaced
    by its maximum over each parameter tensor."""

    def __init__(self, params, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8):
        super().__init__(params, dict(lr=lr, betas=betas, eps=eps))

    @torch.no_grad()
    def step(self, closure=None):
        for group in self.param_groups:
            b1, b2 = group["betas"]
            for p in group["params"]:
                if p.grad is None:
                    continue
                st = self.state[p]
                if not st:
                    st["t"] = 0
                    st["m"] = torch.zeros_like(p)
                    st["v"] = torch.zeros_like(p)
                st["t"] += 1
                t = st["t"]
                st["m"].mul_(b1).add_(p.grad, alpha=1 - b1)
                st["v"].mul_(b2).addcmul_(p.grad, p.grad, value=1 - b2)
                m_hat = st["m"] / (1 - b1 ** t)
                v_max = (st["v"] / (1 - b2 ** t)).max()
                p.add_(m_hat / (v_max.sqrt() + group["eps"]), alpha=-group["lr"])


class _FromU(torch.autograd.Function):
    """V = (I + lambda L)^-1 u; the matrix is symmetric, so the backward is
    the same solve applied to the incoming gradient."""

    @staticmethod
    def forward(ctx, u, ls):
        ctx.ls = ls
        return ls.to_v(u)

    @staticmethod
    def backward(ctx, g):
        return ctx.ls.to_v(g.contiguous(), slot="g"), None
