"""The pseudo-fermion (and gauge) action as a ``torch.autograd.Function`` whose backward is the
library's hand-written force kernels.

The gauge field is parametrised around a fixed field U0 by Lie-algebra coordinates omega
(whmc algebra layout, float64 on the GPU):  U(omega) = exp(omega) U0.  ``forward`` sets the
context's gauge field to U(omega) (T-step kernel) and returns
    S(omega) = S~_PF(U(omega), phi)  [+ S~_G(U(omega)) if include_gauge]
(Sec. 1 eq. WePe_action, Sec. 2 eq. ModPF / ModGauge).  ``backward`` evaluates the force
F = dS/d(omega') at U(omega) (defined by (omega', F) = delta_omega' S for delta U = omega' U,
Sec. 1) with the force kernels and maps it to the omega coordinates with the transpose of the
exponential's differential, so gradients are exact for any omega (they equal F at omega = 0).
"""
import torch

from . import whmc


class GaugeChart:
    """a whmc context plus the base field U0 of the chart U(omega) = exp(omega) U0."""

    def __init__(self, ctx, U0, phi, k=0, n_t=0, n_max=0, kappa=0.156, beta=5.6, solver=None,
                 include_gauge=False):
        self.ctx = ctx
        self.U0 = U0.clone()
        self.phi = phi
        self.filter = (k, n_t, n_max)
        self.kappa = kappa
        self.beta = beta
        self.solver = solver or whmc.cg_params(tol=1e-12)
        self.include_gauge = include_gauge

    def set_field(self, omega):
        self.ctx.load_gauge(self.U0, unitarity_tol=0.0)
        self.ctx.update_links(omega, 1.0)


class PFAction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, omega, chart):
        chart.set_field(omega.detach())
        k, n_t, n_max = chart.filter
        sg, spf = chart.ctx.action(chart.phi, k, n_t, n_max, chart.kappa, chart.beta, solver=chart.solver)
        fctx.chart = chart
        fctx.save_for_backward(omega.detach())
        S = spf + (sg if chart.include_gauge else 0.0)
        return torch.tensor(S, dtype=torch.float64, device=omega.device)

    @staticmethod
    def backward(fctx, grad_S):
        (omega,) = fctx.saved_tensors
        chart = fctx.chart
        chart.set_field(omega)
        k, n_t, n_max = chart.filter
        flags = whmc.FORCE_PF | (whmc.FORCE_GAUGE if chart.include_gauge else 0)
        F = chart.ctx.force(chart.phi, k, n_t, n_max, chart.kappa, chart.beta, flags=flags, solver=chart.solver)
        g = chart.ctx.dexp_transpose(omega.contiguous(), F)
        return grad_S * g, None


def pf_action(omega, chart):
    return PFAction.apply(omega, chart)
