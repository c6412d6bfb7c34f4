"""torch.autograd.Function over the library's forward and adjoint.

theta = [R_1..R_J, Lim_1..Lim_J, OccR, OccL, AggR, AggL] (float64) maps to
(mean annual loss, TVaR_p) of one layer.  The forward runs ara_run_layers
with ARA_CHECKPOINT_S and ara_risk_metrics; the backward calls ara_backward,
whose partials are integer counts over the strict-subgradient convention, and
scales them by the incoming gradients.  Everything runs on the device;
torch supplies the memory and the stream.
"""

from __future__ import annotations

import numpy as np
import torch

from . import ara


class ARAFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, tables: "ara.Tables", spec: "ara.LayerSpec", tvar_p: float):
        th = theta.detach().to("cpu", torch.float64).numpy()
        s = spec.with_theta(th)
        dev = torch.device("cuda", torch.cuda.current_device())
        ylt = torch.empty(s.trial_count, dtype=torch.float64, device=dev)
        ara.run_layers(tables, [s], out=ylt, flags=ara.ARA_CHECKPOINT_S)
        res = torch.empty(3, dtype=torch.float64, device=dev)
        ara.risk_metrics(ylt, [tvar_p], outputs=res)
        ctx.tables = tables
        ctx.spec = s
        ctx.tvar_p = float(tvar_p)
        ctx.theta_device = theta.device
        ctx.mark_non_differentiable(ylt)
        return res[0].clone(), res[2].clone(), ylt

    @staticmethod
    def backward(ctx, g_mean, g_tvar, g_ylt):
        P = 2 * ctx.spec.n_elts + 4
        dev = torch.device("cuda", torch.cuda.current_device())
        gm = torch.empty(P, dtype=torch.float64, device=dev)
        gt = torch.empty(P, dtype=torch.float64, device=dev)
        ara.backward(ctx.tables, ctx.spec, ctx.tvar_p, grad_mean=gm, grad_tvar=gt)
        grad = torch.zeros(P, dtype=torch.float64, device=dev)
        if g_mean is not None:
            grad = grad + g_mean.to(dev, torch.float64) * gm
        if g_tvar is not None:
            grad = grad + g_tvar.to(dev, torch.float64) * gt
        return grad.to(ctx.theta_device), None, None, None


def mean_and_tvar(theta: torch.Tensor, tables: "ara.Tables", spec: "ara.LayerSpec", tvar_p: float = 0.99):
    """(mean, TVaR_p, YLT) as differentiable functions of theta (YLT is not)."""
    return ARAFunction.apply(theta, tables, spec, tvar_p)


def theta_of(spec: "ara.LayerSpec", device=None) -> torch.Tensor:
    return torch.tensor(np.asarray(spec.theta()), dtype=torch.float64, device=device)
