"""torch.autograd bindings of the operators and of unrolled Algorithm 1 iterations.

Every forward and backward step runs in the library's kernels; torch provides device
memory and the autograd graph.

* phi(plan, x):        y = Phi x, backward x_bar = Re Phi^dagger y_bar (Eq. 3 on real images)
* phi_adj(plan, y):    x = Re Phi^dagger y, backward y_bar = Phi x_bar
* psi(sara, s):        x = Psi s, backward s_bar = Psi^dagger x_bar
* psi_adj(sara, x):    s = Psi^dagger x, backward x_bar = Psi s_bar
* unrolled_pd(...):    x^(T) of T iterations of Algorithm 1 from the zero start with fixed
  active sets, differentiable with respect to (tau, sigma); the backward pass re-runs
  each segment of `checkpoint` iterations from a stored state and sweeps it in reverse
  with ri_pd_step_vjp.

Complex tensors follow torch's convention for gradients of real losses (the gradient
of L with respect to z = a + ib is dL/da + i dL/db), which for the real-linear map
x -> Phi x makes the vector-Jacobian product Re Phi^dagger.
"""
import numpy as np
import torch

from . import _lib as L
from .ops import PD


class _Phi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan, mask):
        ctx.plan, ctx.mask = plan, mask
        return plan.phi(x.detach().contiguous(), mask=mask)

    @staticmethod
    def backward(ctx, gy):
        return ctx.plan.phi_adj(gy.contiguous(), mask=ctx.mask), None, None


class _PhiAdj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, plan, mask):
        ctx.plan, ctx.mask = plan, mask
        return plan.phi_adj(y.detach().contiguous(), mask=mask)

    @staticmethod
    def backward(ctx, gx):
        return ctx.plan.phi(gx.contiguous(), mask=ctx.mask), None, None


class _Psi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, sara):
        ctx.sara = sara
        return sara.psi(s.detach().contiguous())

    @staticmethod
    def backward(ctx, gx):
        return ctx.sara.psi_adj(gx.contiguous()), None


class _PsiAdj(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, sara):
        ctx.sara = sara
        return sara.psi_adj(x.detach().contiguous())

    @staticmethod
    def backward(ctx, gs):
        return ctx.sara.psi(gs.contiguous()), None


def phi(plan, x, mask=None):
    return _Phi.apply(x, plan, mask)


def phi_adj(plan, y, mask=None):
    return _PhiAdj.apply(y, plan, mask)


def psi(sara, s):
    return _Psi.apply(s, sara)


def psi_adj(sara, x):
    return _PsiAdj.apply(x, sara)


class _UnrolledPD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, plan, sara, y, eps, varsigma, kappa, psi_norm, phi_norm, masks, checkpoint):
        tau, sigma = (float(v) for v in params.detach().cpu().tolist())
        pd = PD(plan, sara, y, eps, tau, sigma, varsigma, kappa, psi_norm, phi_norm)
        T = masks.shape[0]
        saved = {}
        for t in range(T):
            if t % checkpoint == 0:
                pd.refresh()  # the segment re-run starts from the same running sum
                saved[t] = [pd.get(w).clone() for w in (L.RI_PD_X, L.RI_PD_XTILDE, L.RI_PD_S, L.RI_PD_V)]
            pd.step(masks[t])
        ctx.pd, ctx.saved, ctx.masks, ctx.checkpoint = pd, saved, masks, checkpoint
        ctx.params_device, ctx.params_dtype = params.device, params.dtype
        return pd.get(L.RI_PD_X).clone()

    @staticmethod
    def backward(ctx, gx):
        pd, masks, C = ctx.pd, ctx.masks, ctx.checkpoint
        T, d = masks.shape
        xbar = gx.detach().to(torch.float32).contiguous().clone()
        xtbar = torch.zeros_like(xbar)
        sbar = torch.zeros_like(ctx.saved[0][2])
        vbar = torch.zeros_like(ctx.saved[0][3])
        pgrad = torch.zeros(2, dtype=torch.float64, device="cuda")
        stats = torch.empty(d, 2, dtype=torch.float64, device="cuda")
        for t0 in sorted(ctx.saved, reverse=True):
            for w, v in zip((L.RI_PD_X, L.RI_PD_XTILDE, L.RI_PD_S, L.RI_PD_V), ctx.saved[t0]):
                pd.set(w, v)
            tape = []
            for t in range(t0, min(t0 + C, T)):
                pd.step(masks[t], stats)
                tape.append((masks[t], pd.get(L.RI_PD_X).clone(), pd.get(L.RI_PD_S).clone(),
                             pd.get(L.RI_PD_V).clone(), pd.get(L.RI_PD_E).clone(), stats.clone()))
            for rec in reversed(tape):
                pd.step_vjp(*rec, xbar, xtbar, sbar, vbar, pgrad)
        grad = pgrad.to(device=ctx.params_device, dtype=ctx.params_dtype)
        return (grad,) + (None,) * 10


def unrolled_pd(params, plan, sara, y, eps, varsigma, kappa, psi_norm, phi_norm, masks, checkpoint=5):
    """x^(T) after T = len(masks) iterations; params = tensor([tau, sigma]) (requires_grad
    for d/d(tau, sigma)); masks: (T, d) uint8 CUDA tensor of fixed active sets."""
    masks = masks if isinstance(masks, torch.Tensor) else torch.tensor(np.asarray(masks, np.uint8))
    masks = masks.to(device="cuda", dtype=torch.uint8).contiguous()
    return _UnrolledPD.apply(params, plan, sara, y, eps, varsigma, kappa, psi_norm, phi_norm, masks, int(checkpoint))
