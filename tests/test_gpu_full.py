"""GPU parity of the full-lattice fermion matrix M = 1 - kappa H (Sec. 1, no even/odd reduction):
M, M^dag, M^dag M, the FP64 CG on M^dag M, and the unfiltered full-lattice pseudo-fermion action
and force, against the oracle on 4^4 Haar links at kappa = 0.156 with phi seed 0, and on lattices
that take the per-XCD slice schedule."""
import numpy as np
import pytest

from oracle import dirac, force
from oracle.lattice import Lattice
from oracle.solve import cg
from paper_1805_03560_amd import synth, whmc

from gpu_util import algebra_to_numpy, make_ctx, pack_full, rel_err, to_dev, unpack_full

pytestmark = pytest.mark.gpu

KAPPA = 0.156


def _case(dims, gen):
    lat = Lattice(dims)
    U = synth.haar_links(dims, 1000) if gen == "haar" else synth.smooth_links(dims, 1000)
    phi = synth.gaussian_spinor(lat.V, 0).reshape(dims + (4, 3))
    return lat, U, phi


@pytest.mark.parametrize("dims,gen", [((4, 4, 4, 4), "haar"), ((4, 8, 16, 16), "smooth"), ((4, 12, 16, 16), "smooth")])
def test_full_M_and_MdagM_parity(dims, gen):
    lat, U, phi = _case(dims, gen)
    ctx = make_ctx(dims, U)
    pb = pack_full(ctx, phi)
    assert rel_err(unpack_full(ctx, ctx.apply_M(pb, KAPPA)), dirac.apply_M(lat, U, phi, KAPPA)) < 1e-12
    assert rel_err(unpack_full(ctx, ctx.apply_M(pb, KAPPA, dagger=True)), dirac.apply_Mdag(lat, U, phi, KAPPA)) < 1e-12
    ref = dirac.apply_Mdag(lat, U, dirac.apply_M(lat, U, phi, KAPPA), KAPPA)
    assert rel_err(unpack_full(ctx, ctx.apply_MdagM(pb, [KAPPA], eo=False)), ref) < 1e-12
    # two right-hand sides with their own kappa in one call
    two = np.stack([phi.reshape(-1, 4, 3), 0.5 * phi.reshape(-1, 4, 3)])
    out = ctx.apply_MdagM(ctx.pack_spinor(to_dev(two), -1), [KAPPA, 0.12], eo=False)
    got = ctx.unpack_spinor(out, -1, 2).cpu().numpy()
    ref2 = dirac.apply_Mdag(lat, U, dirac.apply_M(lat, U, 0.5 * phi, 0.12), 0.12)
    assert rel_err(got[0].reshape(ref.shape), ref) < 1e-12
    assert rel_err(got[1].reshape(ref.shape), ref2) < 1e-12


@pytest.mark.parametrize("dims,gen", [((4, 4, 4, 4), "haar"), ((4, 8, 16, 16), "smooth")])
def test_full_cg_parity(dims, gen):
    lat, U, phi = _case(dims, gen)
    A = lambda v: dirac.apply_Mdag(lat, U, dirac.apply_M(lat, U, v, KAPPA), KAPPA)
    ref, _, _ = cg(A, phi, tol=1e-14)
    ctx = make_ctx(dims, U)
    for links in (whmc.L18, whmc.L12):
        x, st = ctx.cg_solve_full(pack_full(ctx, phi), KAPPA, whmc.cg_params(tol=1e-13, check_every=4, links=links))
        assert st["converged"] and st["true_residual"] <= 1e-13
        assert rel_err(unpack_full(ctx, x), ref) < 1e-11
    # the workload tolerance of 1e-10: error bounded by cond x 1e-10
    x, st = ctx.cg_solve_full(pack_full(ctx, phi), KAPPA, whmc.cg_params(tol=1e-10))
    assert st["true_residual"] <= 1e-10 and rel_err(unpack_full(ctx, x), ref) < 1e-8


def test_full_cg_limits_and_zero_source():
    dims = (4, 4, 4, 4)
    lat, U, phi = _case(dims, "haar")
    ctx = make_ctx(dims, U)
    x, st = ctx.cg_solve_full(pack_full(ctx, np.zeros_like(phi)), KAPPA)
    assert st["converged"] and st["true_residual"] == 0.0 and not unpack_full(ctx, x).any()
    with pytest.raises(whmc.WhmcError) as e:
        ctx.cg_solve_full(pack_full(ctx, phi), KAPPA, whmc.cg_params(tol=1e-12, maxiter=3, check_every=1))
    assert e.value.status == 3   # ENOCONV
    with pytest.raises(whmc.WhmcError) as e:
        ctx.cg_solve_full(pack_full(ctx, phi), KAPPA, whmc.cg_params(prec=whmc.F32, links=whmc.L12))
    assert e.value.status == 4   # EUNSUP: FP64 only


@pytest.mark.parametrize("dims,gen", [((4, 4, 4, 4), "haar"), ((4, 12, 16, 16), "smooth")])
def test_full_action_and_force_parity(dims, gen):
    lat, U, phi = _case(dims, gen)
    ctx = make_ctx(dims, U)
    solver = whmc.cg_params(tol=1e-14, check_every=4)
    pb = pack_full(ctx, phi)
    S = ctx.action_full(pb, KAPPA, solver=solver)
    assert S == pytest.approx(force.pf_action_full(lat, U, phi, KAPPA, tol=1e-14), rel=1e-12)
    F = ctx.force_full(pb, KAPPA, solver=solver)
    ref = force.pf_force_full(lat, U, phi, KAPPA, tol=1e-14)
    assert rel_err(algebra_to_numpy(ctx, F), ref) < 1e-12
