"""Failure handling with non-finite inputs: a NaN or infinity in a pseudo-fermion field makes every
solver, force and trajectory entry point return WHMC_ENONFINITE (never a silent result), and a NaN
link is rejected by the SU(3) check of the gauge import."""
import numpy as np
import pytest

from oracle.lattice import Lattice
from paper_1805_03560_amd import synth, whmc

from gpu_util import make_ctx, pack_full, pack_half, to_dev

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 8)
ENONFINITE = 7


def _bad(lat, seed, value, n=None):
    b = synth.gaussian_spinor(lat.Vh if n is None else n, seed)
    b[min(17, len(b) - 1), 2, 1] = value
    return b


@pytest.fixture(scope="module")
def case():
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, 8000)
    return lat, U, make_ctx(DIMS, U)


def _expect_nonfinite(fn):
    with pytest.raises(whmc.WhmcError) as e:
        fn()
    assert e.value.status == ENONFINITE, str(e.value)


@pytest.mark.parametrize("value", [np.nan, np.inf])
def test_solvers_reject_non_finite_sources(case, value):
    lat, U, ctx = case
    b = pack_half(ctx, _bad(lat, 8001, value))
    _expect_nonfinite(lambda: ctx.cg_solve(b, [0.156], whmc.cg_params()))
    _expect_nonfinite(lambda: ctx.cg_solve(b, [0.156], whmc.cg_params(prec=whmc.F16, links=whmc.L12, delta=0.01)))
    _expect_nonfinite(lambda: ctx.cg_solve(b, [0.156], whmc.cg_params(prec=whmc.F32, links=whmc.L12, delta=0.01)))
    _expect_nonfinite(lambda: ctx.bicgstab_solve(b, 0.12))
    two = pack_half(ctx, np.stack([synth.gaussian_spinor(lat.Vh, 8002), _bad(lat, 8003, value)]))
    _expect_nonfinite(lambda: ctx.cg_solve(two, [0.15, 0.156], whmc.cg_params()))
    full = pack_full(ctx, _bad(lat, 8004, value, n=lat.V))
    _expect_nonfinite(lambda: ctx.cg_solve_full(full, 0.12))


def test_force_and_trajectory_reject_a_nan_field(case):
    lat, U, ctx = case
    phi = pack_half(ctx, _bad(lat, 8010, np.nan))
    _expect_nonfinite(lambda: ctx.force(phi, 2, 15, 29, 0.156, 5.6))
    _expect_nonfinite(lambda: ctx.action(phi, 0, 0, 0, 0.156, 5.6))
    pi0 = ctx.pack_algebra(to_dev(synth.gaussian_momenta(DIMS, 8011)))
    p = whmc.hmc_params(beta=5.6, kappa=0.15, k=2, n_t=6, n_max=12, m=2, m0=1, tau=0.2)
    _expect_nonfinite(lambda: ctx.hmc_trajectory(p, pi0, phi, 0.5))
    # the gauge field is left as it was
    assert np.array_equal(ctx.export_gauge().cpu().numpy(), U)
    # and a clean trajectory still runs afterwards
    res = ctx.hmc_trajectory(p, pi0, pack_half(ctx, synth.gaussian_spinor(lat.Vh, 8012)), 0.5)
    assert np.isfinite(res["dH"])


def test_nan_link_is_rejected():
    dims = (4, 4, 4, 4)
    U = synth.haar_links(dims, 8020)
    U[1, 2, 3, 0, 2, 1, 1] = np.nan
    ctx = whmc.Context(dims)
    with pytest.raises(whmc.WhmcError) as e:
        ctx.load_gauge(to_dev(U), unitarity_tol=1e-11)
    assert e.value.status == 5   # ENOTSU3
