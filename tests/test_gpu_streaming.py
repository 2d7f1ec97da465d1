"""GPU parity with the non-temporal (streaming) link loads forced on.

Streaming link loads switch on by themselves only when a link array exceeds the context's stream
threshold (128 MiB by default), i.e. on the 24^3 x 48 and 32^3 x 64 lattices, where every solver,
multi-RHS and force kernel then runs its streaming variant.  Setting the threshold to 0 selects
those variants on small lattices, so that they are compared with the oracle element by element.
The lattice (4, 8, 16, 16) has time slices of 8 x 128 sites: the per-XCD slice schedule of the
large lattices as well."""
import numpy as np
import pytest

from oracle import dirac, hpe, rooted
from oracle.lattice import Lattice
from oracle.solve import cg
from paper_1805_03560_amd import synth, whmc

from gpu_util import algebra_to_numpy, make_ctx, oracle_cached, pack_full, pack_half, rel_err, unpack_full, unpack_half

pytestmark = pytest.mark.gpu

DIMS = (4, 8, 16, 16)
KAPPA = 0.1575


def _ctx(U):
    ctx = make_ctx(DIMS, U)
    ctx.set_option(whmc.OPT_STREAM_THRESHOLD, 0)
    assert ctx.get_option(whmc.OPT_STREAM_THRESHOLD) == 0
    return ctx


def test_stream_threshold_option():
    ctx = make_ctx((4, 4, 4, 4), synth.haar_links((4, 4, 4, 4), 7000))
    assert ctx.get_option(whmc.OPT_STREAM_THRESHOLD) == 128 << 20
    ctx.set_option(whmc.OPT_STREAM_THRESHOLD, -1)
    assert ctx.get_option(whmc.OPT_STREAM_THRESHOLD) == -1
    for bad in [(whmc.OPT_STREAM_THRESHOLD, -2), (99, 0)]:
        with pytest.raises(whmc.WhmcError) as e:
            ctx.set_option(*bad)
        assert e.value.status == 1   # EARG


def test_streamed_hops_and_operators():
    lat = Lattice(DIMS)
    U = synth.haar_links(DIMS, 7001)
    x = synth.gaussian_spinor(lat.Vh, 7002)
    ctx = _ctx(U)
    for links in (whmc.L18, whmc.L12):
        for par, dag in [(0, 0), (1, 1)]:
            out = ctx.apply_H(pack_half(ctx, x), par, dagger=dag, links=links)
            assert rel_err(unpack_half(ctx, out), dirac.apply_Hblock(lat, U, x, par, dagger=bool(dag))) < 1e-12
    psi = synth.gaussian_spinor(lat.V, 7003).reshape(DIMS + (4, 3))
    assert rel_err(unpack_full(ctx, ctx.apply_H(pack_full(ctx, psi), -1)), dirac.apply_H(lat, U, psi)) < 1e-12
    assert rel_err(unpack_full(ctx, ctx.apply_M(pack_full(ctx, psi), KAPPA)), dirac.apply_M(lat, U, psi, KAPPA)) < 1e-12
    assert rel_err(unpack_half(ctx, ctx.apply_MdagM(pack_half(ctx, x), [KAPPA])),
                   dirac.apply_MooDagMoo(lat, U, x, KAPPA)) < 1e-12


def _solution(seed=7010):
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, seed)
    b = synth.gaussian_spinor(lat.Vh, seed + 1)
    ref, _, _ = cg(lambda v: dirac.apply_MooDagMoo(lat, U, v, KAPPA), b, tol=1e-14)
    return lat, U, b, ref


def test_streamed_cg_fp64_and_mixed():
    lat, U, b, ref = _solution()
    ctx = _ctx(U)
    for links in (whmc.L18, whmc.L12):
        x, st = ctx.cg_solve(pack_half(ctx, b), [KAPPA], whmc.cg_params(tol=1e-13, check_every=4, links=links))
        assert st[0]["converged"] and rel_err(unpack_half(ctx, x), ref) < 1e-11
    for prec, links in [(whmc.F32, whmc.L12), (whmc.F32, whmc.L18), (whmc.F16, whmc.L12)]:
        x, st = ctx.cg_solve(pack_half(ctx, b), [KAPPA], whmc.cg_params(tol=1e-10, prec=prec, links=links, delta=0.1))
        assert st[0]["converged"] and st[0]["true_residual"] <= 1e-10 and st[0]["reliable_updates"] >= 1
        assert rel_err(unpack_half(ctx, x), ref) < 1e-8


# multi-RHS kernels stream their links only where a launch reads each link once: one rhs group
# (lanes x rhs per thread = 4) or group-major order; block-major order with several groups keeps
# them cached whatever the threshold
@pytest.mark.parametrize("prec,links,lanes,order", [(whmc.F64, whmc.L18, 2, 0), (whmc.F64, whmc.L18, 2, 1),
                                                    (whmc.F64, whmc.L12, 4, 0), (whmc.F32, whmc.L12, 2, 1),
                                                    (whmc.F16, whmc.L12, 1, 1)])
def test_streamed_masked_multi_rhs_cg(prec, links, lanes, order):
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, 7020)
    kappas = [0.150, 0.153, 0.156, 0.1575]
    bs = np.stack([synth.gaussian_spinor(lat.Vh, 7021 + r) for r in range(4)])
    ctx = _ctx(U)
    nb = 2 if prec == whmc.F16 else 1
    prm = whmc.cg_params(tol=1e-12 if prec == whmc.F64 else 1e-10, prec=prec, links=links, delta=0.1, rhs_block=nb,
                         rhs_lanes=lanes, rhs_order=order)
    x, st = ctx.cg_solve(pack_half(ctx, bs), kappas, prm)
    got = unpack_half(ctx, x, 4)
    for r, k in enumerate(kappas):
        ref = oracle_cached(("moo_cg", DIMS, "smooth", 7020, 7021 + r, k),
                            lambda: cg(lambda v: dirac.apply_MooDagMoo(lat, U, v, k), bs[r], tol=1e-14)[0])
        assert st[r]["converged"]
        assert rel_err(got[r], ref) < (1e-9 if prec == whmc.F64 else 1e-7), r


def test_streamed_bicgstab():
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, 7030, width=0.55)
    b = synth.gaussian_spinor(lat.Vh, 7031)
    ref, _, _ = cg(lambda v: dirac.apply_MooDagMoo(lat, U, v, KAPPA), dirac.apply_Moo_dag(lat, U, b, KAPPA), tol=1e-14)
    ctx = _ctx(U)
    for links in (whmc.L18, whmc.L12):
        x, st = ctx.bicgstab_solve(pack_half(ctx, b), KAPPA, params=whmc.cg_params(tol=1e-13, links=links,
                                                                                   check_every=4))
        assert st["converged"] and rel_err(unpack_half(ctx, x), ref) < 1e-10


def test_streamed_filtered_force_and_full_cg():
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, 7040)
    phi = synth.gaussian_spinor(lat.Vh, 7041)
    ctx = _ctx(U)
    solver = whmc.cg_params(tol=1e-14, check_every=4)
    F = ctx.force(pack_half(ctx, phi), 2, 15, 29, KAPPA, 5.6, solver=solver)
    ref = hpe.filtered_force(lat, U, phi, KAPPA, 2, 15, tol=1e-14)
    assert rel_err(algebra_to_numpy(ctx, F), ref) < 1e-12
    psi = synth.gaussian_spinor(lat.V, 7042).reshape(DIMS + (4, 3))
    A = lambda v: dirac.apply_Mdag(lat, U, dirac.apply_M(lat, U, v, 0.12), 0.12)
    xr, _, _ = cg(A, psi, tol=1e-14)
    x, st = ctx.cg_solve_full(pack_full(ctx, psi), 0.12, whmc.cg_params(tol=1e-13))
    assert st["converged"] and rel_err(unpack_full(ctx, x), xr) < 1e-11


def test_streamed_rooted_force_over_several_pair_launches():
    """a remainder series at n_t = 60 gives 61 (X, Y) pairs, three launches of the pair kernel
    (24 pairs each), the later two accumulating"""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 7050)
    kappa = 0.156
    phi = synth.gaussian_spinor(lat.Vh, 7051)
    ctx = make_ctx(dims, U)
    ctx.set_option(whmc.OPT_STREAM_THRESHOLD, 0)
    r = whmc.rooted(2, (4,), k=0, n_t=60, n_max=60)
    ps, b, al = rooted.coefficients_f64(2, (4,), 0, 60)
    phis = np.stack([synth.gaussian_spinor(lat.Vh, 7052 + f) for f in range(2)] + [phi])
    F = ctx.rooted_force(pack_half(ctx, phis), r, kappa, term=2, solver=whmc.cg_params(tol=1e-14, check_every=4))
    ref = rooted.series_force(lat, U, phi, b[:61], al, kappa, tol=1e-14)
    assert rel_err(algebra_to_numpy(ctx, F), ref) < 1e-12
