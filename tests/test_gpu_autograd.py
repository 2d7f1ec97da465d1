"""The pseudo-fermion action as torch.autograd.Function: its backward (the force kernels plus the
exponential-chart chain rule) against central finite differences of S along random algebra
directions, at omega = 0 and away from it, and against the oracle force at omega = 0."""
import numpy as np
import pytest
import torch

from oracle import hpe
from oracle.lattice import Lattice
from paper_1805_03560_amd import synth, whmc
from paper_1805_03560_amd.autograd import GaugeChart, pf_action

from gpu_util import algebra_to_numpy, make_ctx, pack_half, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _chart(k, n_t, n_max, include_gauge=False):
    dims = (4, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 6000)
    phi = synth.gaussian_spinor(lat.Vh, 6001)
    ctx = make_ctx(dims, U)
    chart = GaugeChart(ctx, to_dev(U), pack_half(ctx, phi), k=k, n_t=n_t, n_max=n_max, kappa=0.156, beta=5.6,
                       solver=whmc.cg_params(tol=1e-14, check_every=4), include_gauge=include_gauge)
    return lat, U, phi, ctx, chart


@pytest.mark.parametrize("k,n_t,include_gauge", [(0, 0, False), (2, 6, True)])
@pytest.mark.parametrize("omega_scale", [0.0, 0.2])
def test_autograd_gradient_matches_finite_differences(k, n_t, include_gauge, omega_scale):
    lat, U, phi, ctx, chart = _chart(k, n_t, n_t, include_gauge)
    dims = lat.dims
    omega0 = ctx.pack_algebra(to_dev(synth.random_algebra(dims, 6002, scale=omega_scale)))
    omega = omega0.clone().requires_grad_(True)
    S = pf_action(omega, chart)
    S.backward()
    grad = omega.grad.clone()
    for seed in (6003, 6004):
        eta = ctx.pack_algebra(to_dev(synth.random_algebra(dims, seed)))
        eps = 1e-4
        f = lambda e: float(pf_action(omega0 + e * eta, chart))
        fd = (8 * (f(eps) - f(-eps)) - (f(2 * eps) - f(-2 * eps))) / (12 * eps)
        assert float(torch.dot(grad, eta)) == pytest.approx(fd, rel=1e-7)


def test_autograd_gradient_at_zero_is_the_oracle_force():
    lat, U, phi, ctx, chart = _chart(2, 5, 5)
    omega = ctx.algebra().requires_grad_(True)
    S = pf_action(omega, chart)
    assert float(S.detach()) == pytest.approx(hpe.filtered_action(lat, U, phi, 0.156, 2, 5, tol=1e-14), rel=1e-11)
    S.backward()
    ref = hpe.filtered_force(lat, U, phi, 0.156, 2, 5, tol=1e-14)
    assert rel_err(algebra_to_numpy(ctx, omega.grad), ref) < 1e-12
