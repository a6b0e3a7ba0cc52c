"""Differentiable time march: u(T) as a function of (u0, kx, ky) (and kz on a
three-dimensional plan).

Forward: m implicit steps through rsfde_step, keeping checkpoints every s
steps (s = ceil(sqrt(m)) by default).  Backward: for each checkpoint segment
from the last to the first, recompute the segment's states with rsfde_step,
then run rsfde_adjoint_step from the segment end down to its start.  Every
arithmetic step runs in the HIP library; this module only schedules calls
and holds device buffers.

The adjoint of one step M u^k = u^{k-1} + dt mask f(u^{k-1}) (M symmetric):
  mu^k = M^{-1} lam^k,  lam^{k-1} = mu^k + dt mask f'(u^{k-1}) mu^k,
  dL/dkx += <mu^k, (I (x) A_x/kx) u^k>,  dL/dky += <mu^k, (A_y/ky (x) I) u^k>,
  (3-D: dL/dkz += <mu^k, (A_z/kz (x) I (x) I) u^k>)
with lam^m = dL/du^m and dL/du0 = lam^0.
"""

from __future__ import annotations

import math
from typing import List, Tuple

import torch

from ._lib import make_opts


def checkpoint_schedule(m: int, every: int = 0) -> List[Tuple[int, int]]:
    """Segments (start, end) covering steps 1..m; a checkpoint holds the state at
    `start` (and start-1) and the segment recomputes steps start+1..end."""
    if m < 1:
        return []
    s = every if every and every > 0 else max(1, math.ceil(math.sqrt(m)))
    segs = []
    c = 0
    while c < m:
        segs.append((c, min(c + s, m)))
        c += s
    return segs


def _march_forward(ctx, u0, ks, plan, m, f_kind, opts, every, adj_opts):
    opts = make_opts() if opts is None else opts
    kf = tuple(float(k) for k in ks)
    plan.set_coeffs(*kf)
    segs = checkpoint_schedule(m, every)
    u0c = u0.detach().contiguous()
    ckpt = {0: (u0c.clone(), None)}
    prev, cur = None, u0c.clone()
    iters = []
    for k in range(1, m + 1):
        nxt, st = plan.step(cur, prev, f_kind, opts)
        iters.append(st.iters)
        prev, cur = cur, nxt
        if any(k == a for a, _ in segs):
            ckpt[k] = (cur.clone(), prev.clone())
    ctx.plan, ctx.m, ctx.f_kind = plan, m, f_kind
    ctx.opts = opts
    ctx.adj_opts = opts if adj_opts is None else adj_opts
    ctx.segs, ctx.ckpt, ctx.k = segs, ckpt, kf
    ctx.k_is_tensor = tuple(isinstance(k, torch.Tensor) for k in ks)
    ctx.forward_iters = iters
    return cur


def _march_backward(ctx, grad_out):
    """Reverse sweep over the checkpoint segments; returns (dL/du0, dL/dk...)."""
    plan, f_kind = ctx.plan, ctx.f_kind
    plan.set_coeffs(*ctx.k)
    lam = grad_out.detach().contiguous().clone()
    lam_prev = torch.empty_like(lam)
    mu = torch.zeros_like(lam)  # previous mu: initial guess of the next adjoint solve
    dk = torch.zeros(len(ctx.k), dtype=torch.float64, device=lam.device)
    for (a, b) in reversed(ctx.segs):
        ua, ua_prev = ctx.ckpt[a]
        states = [ua]
        prev, cur = ua_prev, ua
        for _ in range(a + 1, b + 1):
            nxt, _ = plan.step(cur, prev, f_kind, ctx.opts)
            prev, cur = cur, nxt
            states.append(cur)
        for k in range(b, a, -1):
            plan.adjoint_step(states[k - a - 1], states[k - a], lam, f_kind, ctx.adj_opts,
                              lam_prev, dk, mu)
            lam, lam_prev = lam_prev, lam
    grads = tuple(dk[i].clone() if t else None for i, t in enumerate(ctx.k_is_tensor))
    return (lam,) + grads


class RsfdeMarch(torch.autograd.Function):
    """u_T = RsfdeMarch.apply(u0, kx, ky, plan, m, f_kind, opts, every, adj_opts)

    u0: FP64 CUDA tensor with plan.N elements; kx, ky: 0-d FP64 tensors (or
    floats).  opts / adj_opts: rsfde_solver_opts for the forward and adjoint
    solves (adj_opts defaults to opts).  Gradients are returned for u0, kx, ky.
    """

    @staticmethod
    def forward(ctx, u0, kx, ky, plan, m, f_kind, opts=None, every=0, adj_opts=None):
        return _march_forward(ctx, u0, (kx, ky), plan, m, f_kind, opts, every, adj_opts)

    @staticmethod
    def backward(ctx, grad_out):
        return _march_backward(ctx, grad_out) + (None,) * 6


class RsfdeMarch3(torch.autograd.Function):
    """u_T = RsfdeMarch3.apply(u0, kx, ky, kz, plan, m, f_kind, opts, every,
    adj_opts) on a three-dimensional plan; gradients for u0, kx, ky, kz."""

    @staticmethod
    def forward(ctx, u0, kx, ky, kz, plan, m, f_kind, opts=None, every=0, adj_opts=None):
        if not plan.is3d:
            raise ValueError("RsfdeMarch3 needs a three-dimensional plan")
        return _march_forward(ctx, u0, (kx, ky, kz), plan, m, f_kind, opts, every, adj_opts)

    @staticmethod
    def backward(ctx, grad_out):
        return _march_backward(ctx, grad_out) + (None,) * 6


def march(u0, kx, ky, plan, m, f_kind, opts=None, every=0, adj_opts=None):
    """Functional form of RsfdeMarch."""
    return RsfdeMarch.apply(u0, kx, ky, plan, m, f_kind, opts, every, adj_opts)


def march3(u0, kx, ky, kz, plan, m, f_kind, opts=None, every=0, adj_opts=None):
    """Functional form of RsfdeMarch3."""
    return RsfdeMarch3.apply(u0, kx, ky, kz, plan, m, f_kind, opts, every, adj_opts)
