"""Differentiable rendering as a torch.autograd.Function.

`render(V, ior, sigma)` traces every camera ray of a `Tracer` through the
mesh (V, F) and returns pixel colours; its backward runs the device adjoint
and returns dLoss/dV, dLoss/dIoR and dLoss/dsigma (paper Sec. 3.3: vertex
positions, index of refraction and absorption rate are optimised jointly).
`render_grid(V, ior, mu, ...)` does the same with a spatially varying
absorption rate, an RGB grid mu, and returns dLoss/dmu for it (Sec. 3.2).

Memory policy: the forward keeps the per-generation ray state the adjoint
needs.  When storing every generation fits the memory budget it does so;
otherwise it stores every k-th generation and the backward recomputes the
others, with k the smallest stride whose tape + workspace fit the budget.
"""
from __future__ import annotations

import torch

from . import binding as B


def choose_stride(max_depth: int, n_rays: int, nv: int, nf: int, capacity: int,
                  budget_bytes: int) -> int:
    """Smallest checkpoint stride k (1 = store every generation) whose tape
    plus workspace fit in budget_bytes; the stride of least memory if none fits."""
    best_k, best_bytes = 1, None
    for k in range(1, max_depth + 2):
        p = B.Params(max_depth=max_depth, checkpoint_stride=k, queue_capacity=capacity)
        ws, tape = B.dt_trace_bytes(p, n_rays, nv, nf)
        if ws + tape <= budget_bytes:
            return k
        if best_bytes is None or ws + tape < best_bytes:
            best_k, best_bytes = k, ws + tape
    return best_k


class Tracer:
    """Fixed part of a differentiable render: faces, environment, cameras and
    trace parameters.  Reuses its buffers between calls."""

    def __init__(self, F: torch.Tensor, env: B.Env, cameras, max_depth: int = 6,
                 memory_budget: int | None = None, queue_capacity: int | None = None,
                 terminal_env: bool = False, t_eps: float = 1e-5):
        self.F = F
        self.env = env
        self.rays = B.Rays(cameras=cameras)
        self.max_depth = max_depth
        self.terminal_env = terminal_env
        self.t_eps = t_eps
        self.memory_budget = memory_budget
        self.capacity = queue_capacity or 2 * self.rays.n_rays
        self.stride = None
        self.last_stats = None
        self._mesh = None
        self._buf = None
        self._key = None
        self.version = 0     # bumped by every forward: the tape holds only the last one
        self._mask_grad = None
        self._mask_grad_key = None

    def _params(self, stride=None, timing=None) -> B.Params:
        return B.Params(max_depth=self.max_depth, terminal_env=self.terminal_env, t_eps=self.t_eps,
                        checkpoint_stride=stride or self.stride or 1,
                        queue_capacity=self.capacity, timing=timing)

    def _budget(self, device) -> int:
        if self.memory_budget is not None:
            return int(self.memory_budget)
        free, _ = torch.cuda.mem_get_info(device)
        return int(0.5 * free)

    def _prepare(self, V: torch.Tensor):
        nv, nf = V.shape[0], self.F.shape[0]
        if self._mesh is None or self._mesh.nv != nv or self._mesh.V.device != V.device:
            self._mesh = B.Mesh(V, self.F)
        else:
            self._mesh.V = V
            self._mesh.build()
        key = (self.capacity, nv, nf)
        if self._buf is None or self._key != key:
            self.stride = choose_stride(self.max_depth, self.rays.n_rays, nv, nf, self.capacity,
                                        self._budget(V.device))
            self._buf = B.Buffers(self._params(), self.rays, self._mesh, tape=True)
            self._key = key
        return self._mesh, self._buf

    def forward(self, V: torch.Tensor, ior: torch.Tensor, sigma: torch.Tensor,
                absorb: B.Absorption | None = None):
        V = V.detach().contiguous().float()
        while True:
            mesh, buf = self._prepare(V)
            scene = B.Scene(mesh, ior.detach().contiguous().float(),
                            sigma.detach().contiguous().float(), self.env, absorb=absorb)
            rgb, _, _ = B.dt_trace_forward(scene, self.rays, self._params(), buf, want_aux=False)
            stats = buf.stats.cpu()          # one small read: did a ray queue overflow?
            self.last_stats = stats
            if int(stats[B.STAT_DROPPED]) == 0:
                self.version += 1
                return rgb, scene, buf
            self.capacity *= 2               # grow and trace again

    def backward(self, scene, buf, grad_rgb: torch.Tensor, version: int):
        if version != self.version:
            raise B.DTError("this Tracer ran another forward since; its tape holds only the "
                            "latest one (use one Tracer per outstanding graph)")
        return B.dt_trace_backward(scene, self.rays, self._params(), buf,
                                   grad_rgb.contiguous().float())


class DTTrace(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, ior, sigma, tracer: Tracer):
        rgb, scene, buf = tracer.forward(V, ior, sigma)
        ctx.tracer, ctx.scene, ctx.buf, ctx.version = tracer, scene, buf, tracer.version
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        dV, d_ior, d_sigma = ctx.tracer.backward(ctx.scene, ctx.buf, grad_rgb, ctx.version)
        return dV, d_ior.reshape(1), d_sigma.reshape(3), None


def render(V: torch.Tensor, ior: torch.Tensor, sigma: torch.Tensor, tracer: Tracer):
    """Pixel colours [n_pixels, 3], differentiable in V, ior and sigma.
    sigma may be [3] (RGB) or [1] (one rate for all channels)."""
    if sigma.numel() == 1:
        return _BroadcastSigma.apply(V, ior, sigma, tracer)
    return DTTrace.apply(V, ior, sigma, tracer)


class _BroadcastSigma(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, ior, sigma, tracer):
        rgb, scene, buf = tracer.forward(V, ior, sigma.expand(3))
        ctx.tracer, ctx.scene, ctx.buf, ctx.version = tracer, scene, buf, tracer.version
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        dV, d_ior, d_sigma = ctx.tracer.backward(ctx.scene, ctx.buf, grad_rgb, ctx.version)
        return dV, d_ior.reshape(1), d_sigma.sum().reshape(1), None


class _DTTraceGrid(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, ior, mu, tracer, lo, hi, samples):
        ab = B.Absorption(mu.detach().contiguous().float(), lo, hi, samples)
        unused = torch.zeros(3, dtype=torch.float32, device=V.device)   # sigma: replaced by the grid
        rgb, scene, buf = tracer.forward(V, ior, unused, absorb=ab)
        ctx.tracer, ctx.scene, ctx.buf, ctx.version, ctx.ab = tracer, scene, buf, tracer.version, ab
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        dV, d_ior, _ = ctx.tracer.backward(ctx.scene, ctx.buf, grad_rgb, ctx.version)
        return dV, d_ior.reshape(1), ctx.ab.d_mu.clone(), None, None, None, None


def render_grid(V: torch.Tensor, ior: torch.Tensor, mu: torch.Tensor, tracer: Tracer, lo, hi,
                samples: int = 16):
    """Pixel colours [n_pixels, 3] with a spatially varying absorption rate:
    mu is an RGB grid [nz, ny, nx, 3] over the box [lo, hi], trilinear,
    `samples` midpoint samples per interior segment.  Differentiable in V,
    ior and mu."""
    return _DTTraceGrid.apply(V, ior, mu, tracer, lo, hi, samples)


# ------------------------------------------------------------------ environment MLP parameters
class _DTTraceMLP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, ior, sigma, w, b, tracer):
        env = tracer.env
        with torch.no_grad():
            # the device evaluates bf16 weights: round the float32 parameters
            env.weights.copy_(w.detach().to(torch.bfloat16).view(torch.int16))
            env.biases.copy_(b.detach())
        rgb, scene, buf = tracer.forward(V, ior, sigma)
        ctx.tracer, ctx.scene, ctx.buf, ctx.version = tracer, scene, buf, tracer.version
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        dV, d_ior, d_sigma = ctx.tracer.backward(ctx.scene, ctx.buf, grad_rgb, ctx.version)
        env = ctx.tracer.env
        # the gradient with respect to the bf16 weights is passed to the
        # float32 parameters unchanged (straight through the rounding)
        return (dV, d_ior.reshape(1), d_sigma.reshape(3), env.d_weights.clone(), env.d_biases.clone(),
                None)


def render_mlp(V: torch.Tensor, ior: torch.Tensor, sigma: torch.Tensor, weights: torch.Tensor,
               biases: torch.Tensor, tracer: Tracer):
    """Pixel colours lit by the tracer's MLP environment (an Env made with
    want_grad=True), differentiable in V, ior, sigma [3] and the network's
    float32 parameters (flat weights of every layer, flat biases; the device
    runs them rounded to bf16)."""
    env = tracer.env
    if getattr(env, "d_weights", None) is None:
        raise B.DTError("render_mlp needs an MLP environment made with want_grad=True")
    return _DTTraceMLP.apply(V, ior, sigma, weights, biases, tracer)


# ------------------------------------------------------------------ silhouette (mask) term
class _MaskFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, tracer, rho):
        mesh, _ = tracer._prepare(V.detach().contiguous().float())
        mask = B.dt_mask_forward(mesh, tracer.rays, tracer.t_eps)
        ctx.tracer, ctx.mesh, ctx.rho, ctx.version = tracer, mesh, rho, tracer.version
        return mask

    @staticmethod
    def backward(ctx, grad_mask):
        tr = ctx.tracer
        if tr._mask_grad is None or tr._mask_grad_key != (ctx.mesh.nv, ctx.mesh.nf):
            tr._mask_grad = B.MaskGrad(ctx.mesh)
            tr._mask_grad_key = (ctx.mesh.nv, ctx.mesh.nf)
        dV = tr._mask_grad(ctx.mesh, tr.rays, grad_mask.contiguous().float(), ctx.rho)
        return dV, None, None


def render_mask(V: torch.Tensor, tracer: Tracer, rho: float = 2.0):
    """Centre-sample coverage [n_pixels] of the tracer's cameras; its
    gradient with respect to V is the outline (edge-sampling) gradient of the
    pixels' area coverage, rho quadrature points per pixel of edge length.
    Builds the mesh's BVH from V; call it before render() in a step if both
    are used, or after render()'s backward (the tracer keeps one mesh)."""
    return _MaskFn.apply(V, tracer, float(rho))
