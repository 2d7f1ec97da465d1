"""The single-RHS stencil schedules (WHMC_OPT_HOP_SCHEDULE), the occupancy cap
(WHMC_OPT_HOP_WG_PER_CU) and their autotuner: every schedule, chunk and cap gives the same hop bit
for bit (a site's arithmetic does not depend on which workgroup does it or how many share a compute
unit), solvers on the time-slab schedule with a cap match the oracle, and the tuner keeps a valid
choice."""
import numpy as np
import pytest

from oracle import dirac
from oracle.lattice import Lattice
from oracle.solve import cg
from paper_1805_03560_amd import synth, whmc

from gpu_util import make_ctx, pack_half, rel_err, to_dev, unpack_half

pytestmark = pytest.mark.gpu

# L_t = 8 and 16: one and two slices per XCD; time slices of 8 blocks of 128 sites
DIMS = [(8, 8, 16, 16), (16, 8, 16, 16)]


@pytest.mark.parametrize("dims", DIMS)
def test_schedules_give_identical_hops(dims):
    lat = Lattice(dims)
    U = synth.haar_links(dims, 9100)
    x = synth.gaussian_spinor(lat.Vh, 9101)
    ctx = make_ctx(dims, U)
    xb = pack_half(ctx, x)
    ref = dirac.apply_Hblock(lat, U, x, 0)
    base = ctx.apply_H(xb, 0).clone()
    assert rel_err(unpack_half(ctx, base), ref) < 1e-12
    for cap in (2, 4):
        ctx.set_option(whmc.OPT_HOP_WG_PER_CU, cap)
        assert ctx.get_option(whmc.OPT_HOP_WG_PER_CU) == cap
        assert bool((ctx.apply_H(xb, 0) == base).all())
    for chunk, cap in [(1, 0), (3, 2), (8, 8)]:   # 3: the last chunk of a slice is ragged (padding workgroups)
        ctx.set_option(whmc.OPT_HOP_WG_PER_CU, cap)
        ctx.set_option(whmc.OPT_HOP_CHUNK, chunk)
        ctx.set_option(whmc.OPT_HOP_SCHEDULE, 1)
        assert ctx.get_option(whmc.OPT_HOP_SCHEDULE) == 1 and ctx.get_option(whmc.OPT_HOP_CHUNK) == chunk
        for par, dag in [(0, 0), (1, 1)]:
            out = ctx.apply_H(xb, par, dagger=dag)
            if (par, dag) == (0, 0):
                assert bool((out == base).all())
            assert rel_err(unpack_half(ctx, out), dirac.apply_Hblock(lat, U, x, par, dagger=bool(dag))) < 1e-12


@pytest.mark.parametrize("dims", DIMS)
def test_solvers_on_the_slab_schedule(dims):
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 9110)
    b = synth.gaussian_spinor(lat.Vh, 9111)
    kappa = 0.1575
    ref, _, _ = cg(lambda v: dirac.apply_MooDagMoo(lat, U, v, kappa), b, tol=1e-14)
    ctx = make_ctx(dims, U)
    ctx.set_option(whmc.OPT_HOP_CHUNK, 3)
    ctx.set_option(whmc.OPT_HOP_SCHEDULE, 1)
    ctx.set_option(whmc.OPT_HOP_WG_PER_CU, 2)
    x, st = ctx.cg_solve(pack_half(ctx, b), [kappa], whmc.cg_params(tol=1e-13, check_every=4))
    assert st[0]["converged"] and rel_err(unpack_half(ctx, x), ref) < 1e-11
    x, st = ctx.cg_solve(pack_half(ctx, b), [kappa], whmc.cg_params(tol=1e-10, prec=whmc.F16, links=whmc.L12,
                                                                     delta=0.1))
    assert st[0]["converged"] and rel_err(unpack_half(ctx, x), ref) < 1e-8
    if dims != DIMS[0]:
        return   # the oracle's reference for BiCGstab (CG on the normal equations) is slow beyond 8 x 8 x 16 x 16
    U2 = synth.smooth_links(dims, 9112, width=0.55)
    ctx.load_gauge(to_dev(U2))
    ref2, _, _ = cg(lambda v: dirac.apply_MooDagMoo(lat, U2, v, kappa), dirac.apply_Moo_dag(lat, U2, b, kappa),
                    tol=1e-14)
    x, st = ctx.bicgstab_solve(pack_half(ctx, b), kappa, params=whmc.cg_params(tol=1e-13, check_every=4))
    assert st["converged"] and rel_err(unpack_half(ctx, x), ref2) < 1e-10


def test_schedule_autotuner_and_limits():
    dims = (16, 8, 16, 16)
    ctx = make_ctx(dims, synth.smooth_links(dims, 9120))
    sched, chunk, us = ctx.autotune_hop()
    assert sched in (0, 1) and 1 <= chunk <= 8 and us > 0
    assert ctx.get_option(whmc.OPT_HOP_SCHEDULE) == sched
    assert ctx.get_option(whmc.OPT_HOP_WG_PER_CU) in (0, 2)
    for bad in (1, 9, -1):
        with pytest.raises(whmc.WhmcError) as e:
            ctx.set_option(whmc.OPT_HOP_WG_PER_CU, bad)
        assert e.value.status == 1
    # lattices without the slab schedule: L_t not divisible by 8, or slices not whole blocks
    for bad_dims in [(6, 8, 16, 16), (8, 4, 4, 4)]:
        c2 = make_ctx(bad_dims, synth.haar_links(bad_dims, 9121))
        with pytest.raises(whmc.WhmcError) as e:
            c2.set_option(whmc.OPT_HOP_SCHEDULE, 1)
        assert e.value.status == 1
        assert c2.autotune_hop()[0] == 0
    with pytest.raises(whmc.WhmcError):
        ctx.set_option(whmc.OPT_HOP_CHUNK, 9)
