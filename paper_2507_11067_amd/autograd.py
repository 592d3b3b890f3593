"""Differentiable acoustic modelling on top of the library's forward and
adjoint wave kernels (torch.autograd.Function), with checkpoint/recompute.

WavePropagate.apply(m, u0, u1, problem) -> traces [nt, ny, nx]
    m = v^2 on the padded grid (FP32); u0, u1 = the first two wavefield levels.
    Backward returns dJ/dm, dJ/du0, dJ/du1 for any loss J of the traces, from
    the exact discrete adjoint, not from a self-adjoint shortcut.  By default
    the adjoint runs in mu = C2 G lam (mms_wave_adjoint_mu: the forward step's
    form, one fewer field stream per step, and the more accurate of the two in
    the dot-product test), which needs m > 0 on the whole interior (true for
    m = v^2); adjoint_form="lam" runs mms_wave_adjoint for any m, and "auto"
    checks m on the device and picks one (a host synchronisation).

Memory plan: the forward pass keeps the pair (u^k, u^{k+1}) at every level
k = 0, K, 2K, ... .  The backward pass walks the segments [k, k+K) from the
last to the first: it restores the pair, recomputes u^{k+2} .. u^{k+K-1} into
a K-level buffer, then runs the adjoint steps k+K-1 .. k, which read u^n from
that buffer and accumulate the FP64 gradient.  Extra cost: one more forward
sweep; extra memory: 2 nt/K + K grids.  With Problem.store_all the forward
pass writes every level into a grid of its own instead (nt + 1 grids, 74 GB
for 256^3 x 1000 steps, within one MI355X's 288 GB) and the backward pass
runs the adjoint over all steps in one call with no recompute.

Misfit.apply(traces, d_obs) -> J = 0.5 sum (d - d_obs)^2 (FP64, one element),
computed by the library's reduction kernel; its backward scales the residual by
the upstream derivative in the library (mms_flat_scale_f32), with no host sync.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import Grid, Wave, dense_to_grid, flat_misfit, flat_scale


@dataclass
class Problem:
    grid: Grid
    lap: tuple                 # per-axis weights at unit spacing: centre, k = 1..r
    nt: int                    # time levels 0..nt-1
    h: float
    dt: float
    src: tuple = (0, 0, 0)
    src_dt2f: torch.Tensor | None = None   # device [nt] FP32
    sponge_width: int = 0
    sponge_alpha: float = 0.0
    sponge_faces: int = 0
    checkpoint_every: int = 50
    grad_block: int = 8        # adjoint steps whose gradient terms are summed in FP32
    adjoint_form: str = "mu"   # "mu" (needs m > 0 on the interior), "lam", or "auto"
    store_all: bool = False    # keep every forward level resident (nt + 1 grids), no recompute
    stats: dict = field(default_factory=dict)

    @property
    def c2_scale(self) -> float:
        return (self.dt / self.h) ** 2

    def wave(self, m: torch.Tensor, traces=None, source=True) -> Wave:
        return Wave(self.grid, m, self.lap, self.nt, c2_scale=self.c2_scale,
                    sponge_width=self.sponge_width, sponge_alpha=self.sponge_alpha,
                    sponge_faces=self.sponge_faces, src=self.src,
                    src_dt2f=self.src_dt2f if source else None, traces=traces)


class WavePropagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, u0, u1, prob: Problem):
        g = prob.grid
        K = max(1, int(prob.checkpoint_every))
        nt = prob.nt
        m = m.detach().contiguous()
        traces = torch.zeros((nt, g.ny, g.nx), dtype=torch.float32, device=m.device)
        w = prob.wave(m, traces)
        ckpts, levels = [], None
        if prob.store_all:
            # level n in levels[n]; step nt-1 writes u^nt, which nothing reads
            levels = [g.zeros(m.device) for _ in range(nt + 1)]
            levels[0].copy_(u0.detach())
            if nt > 0:
                levels[1].copy_(u1.detach())
                w.record(0, levels[0])
            if nt > 1:
                w.forward(1, nt, levels)
        else:
            bufs = [u0.detach().clone(), u1.detach().clone(), g.zeros(m.device)]
            if nt > 0:
                w.record(0, bufs[0])
            for k in range(0, nt, K):
                ckpts.append((bufs[k % 3].clone(), bufs[(k + 1) % 3].clone()))
                n_end = min(k + K + 1, nt)
                if n_end > k + 1:
                    w.forward(k + 1, n_end, [bufs[(k + i) % 3] for i in range(n_end - k + 1)])
        ctx.prob = prob
        ctx.ckpts = ckpts
        ctx.levels = levels
        ctx.save_for_backward(m)
        prob.stats["forward_steps"] = max(nt - 1, 0)
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        (m,) = ctx.saved_tensors
        prob = ctx.prob
        g = prob.grid
        K = max(1, int(prob.checkpoint_every))
        nt = prob.nt
        dev = m.device
        resid = grad_traces.detach().to(torch.float32).contiguous()
        wa = prob.wave(m, source=False)    # adjoint: geometry, C2 and sponge
        H = g.halo
        if prob.adjoint_form not in ("auto", "mu", "lam"):
            raise ValueError(f"adjoint_form {prob.adjoint_form!r}")
        if prob.adjoint_form == "auto":
            # the one host synchronisation of a backward pass, only when asked for
            mu_form = bool((m[H:H + g.nz, H:H + g.ny, H:H + g.nx] > 0).all())
        else:
            mu_form = prob.adjoint_form == "mu"
        adjoint = wa.adjoint_mu if mu_form else wa.adjoint
        lam = [g.zeros(dev) for _ in range(3)]   # lam^n (or mu^n) lives in lam[n % 3]
        seg = [] if ctx.levels is not None else [g.zeros(dev) for _ in range(min(K, max(nt, 1)))]
        grad = torch.zeros((g.nz, g.ny, g.nx), dtype=torch.float64, device=dev)
        if prob.grad_block > 1:
            # each block of grad_block adjoint steps is summed in FP32, then added in FP64
            wa.set_accumulation(torch.empty((g.nz, g.ny, g.nx), device=dev), prob.grad_block)
        recomputed = 0
        w_src = prob.wave(m)               # recompute: same source, no receivers
        if ctx.levels is not None and nt > 0:
            # every level is resident: the whole adjoint in one call
            adjoint(nt - 1, 0, [lam[i % 3] for i in range(nt + 2)], us=ctx.levels[0:nt],
                    resid=resid, grad=grad)
        for si in range(len(ctx.ckpts) - 1, -1, -1):
            k = si * K
            hi = min(k + K, nt) - 1
            seg[0].copy_(ctx.ckpts[si][0])
            if hi >= k + 1:
                seg[1].copy_(ctx.ckpts[si][1])
            if hi >= k + 2:
                w_src.forward(k + 1, hi, seg[0:hi - k + 1])
                recomputed += hi - k - 1
            adjoint(hi, k, [lam[(k + i) % 3] for i in range(hi - k + 3)],
                    us=seg[0:hi - k + 1], resid=resid, grad=grad)
        if mu_form:
            for b in lam[:2]:
                wa.scale_mu(b, b, -1)      # mu^0, mu^1 -> lam^0, lam^1
        grad_m = dense_to_grid(grad, g.zeros(dev), g)
        grad_u0 = lam[0].clone() if nt > 0 else g.zeros(dev)
        grad_u1 = lam[1 % 3].clone() if nt > 1 else g.zeros(dev)
        prob.stats["recomputed_steps"] = recomputed
        ctx.levels = None
        prob.stats["adjoint_form"] = "mu" if mu_form else "lam"
        ctx.ckpts = None
        return grad_m, grad_u0, grad_u1, None


class Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, traces, d_obs):
        t = traces.detach().contiguous()
        resid = torch.empty_like(t)
        pair = flat_misfit(t, d_obs.detach().contiguous(), resid=resid)
        ctx.save_for_backward(resid)
        return pair[:1].clone()    # J; pair[1] counts non-finite terms

    @staticmethod
    def backward(ctx, gJ):
        (resid,) = ctx.saved_tensors
        # dJ/dd = resid times the upstream derivative, read on the device by the library
        scale = gJ.detach().to(torch.float64).reshape(1).contiguous()
        return flat_scale(resid, scale, torch.empty_like(resid)), None


def propagate(m, u0, u1, prob: Problem):
    return WavePropagate.apply(m, u0, u1, prob)


def misfit(traces, d_obs):
    return Misfit.apply(traces, d_obs)
