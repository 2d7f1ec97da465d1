"""The 8-real link format (U01, U02, one of U10 / U20 and two phases, rebuilt from unitarity and
det U = 1) against the oracle: FP64 hops and solves to the FP64 bar, FP32 / FP16 hops within their
rounding, mixed-precision solves to the FP64 residual, and fields the format cannot represent."""
import numpy as np
import pytest

from oracle import dirac
from oracle.lattice import Lattice
from oracle.solve import cg
from paper_1805_03560_amd import synth, whmc

from gpu_util import make_ctx, pack_full, pack_half, rel_err, to_dev, unpack_full, unpack_half

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (4, 4, 6, 6), (8, 6, 4, 12), (6, 8, 16, 16), (4, 12, 16, 16)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("gen", ["haar", "smooth"])
def test_hop_fp64_8real_parity(dims, gen):
    lat = Lattice(dims)
    U = synth.haar_links(dims, 9200) if gen == "haar" else synth.smooth_links(dims, 9200, width=0.3)
    x = synth.gaussian_spinor(lat.Vh, 9201)
    ctx = make_ctx(dims, U)
    for stream in (False, True):
        ctx.set_option(whmc.OPT_STREAM_THRESHOLD, 0 if stream else -1)
        for par, dag in [(0, 0), (1, 0), (0, 1), (1, 1)]:
            out = ctx.apply_H(pack_half(ctx, x), par, dagger=dag, links=whmc.L8)
            assert rel_err(unpack_half(ctx, out), dirac.apply_Hblock(lat, U, x, par, dagger=bool(dag))) < 1e-12


def test_full_H_8real_parity():
    dims = (4, 4, 6, 6)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 9210)
    psi = synth.gaussian_spinor(lat.V, 9211).reshape(dims + (4, 3))
    ctx = make_ctx(dims, U)
    out = ctx.apply_H(pack_full(ctx, psi), -1, links=whmc.L8)
    assert rel_err(unpack_full(ctx, out), dirac.apply_H(lat, U, psi)) < 1e-12


# FP16 8-real links keep the phases as theta / pi in half precision (|d theta| <= pi 2^-12) and rebuild
# four entries from products of three stored ones: a few 1e-3 per link on Haar links, hence 1e-2
@pytest.mark.parametrize("prec,tol,gen", [(whmc.F32, 2e-6, "smooth"), (whmc.F16, 4e-3, "smooth"),
                                          (whmc.F32, 2e-6, "haar"), (whmc.F16, 1e-2, "haar")])
def test_hop_low_precision_8real(prec, tol, gen):
    dims = (4, 4, 6, 6)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 9220) if gen == "smooth" else synth.haar_links(dims, 9220)
    x = synth.gaussian_spinor(lat.Vh, 9221)
    ref = dirac.apply_Hblock(lat, U, x, 1)
    ctx = make_ctx(dims, U)
    xin = ctx.convert_spinor(pack_half(ctx, x), whmc.F64, prec)
    out = ctx.apply_H(xin, 1, prec=prec, links=whmc.L8)
    assert rel_err(unpack_half(ctx, ctx.convert_spinor(out, prec, whmc.F64)), ref) < tol


@pytest.mark.parametrize("dims", [(8, 4, 4, 8), (4, 8, 16, 16)])
def test_cg_8real_fp64_and_mixed(dims):
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 9230)
    b = synth.gaussian_spinor(lat.Vh, 9231)
    kappa = 0.1575
    ref, _, _ = cg(lambda v: dirac.apply_MooDagMoo(lat, U, v, kappa), b, tol=1e-14)
    ctx = make_ctx(dims, U)
    x, st = ctx.cg_solve(pack_half(ctx, b), [kappa], whmc.cg_params(tol=1e-13, links=whmc.L8, check_every=4))
    assert st[0]["converged"] and rel_err(unpack_half(ctx, x), ref) < 1e-11
    for prec in (whmc.F32, whmc.F16):
        x, st = ctx.cg_solve(pack_half(ctx, b), [kappa], whmc.cg_params(tol=1e-10, prec=prec, links=whmc.L8,
                                                                         delta=0.1))
        assert st[0]["converged"] and st[0]["true_residual"] <= 1e-10 and st[0]["reliable_updates"] >= 1
        assert rel_err(unpack_half(ctx, x), ref) < 1e-8
    # several right-hand sides with 8-real links: solved one after the other
    bs = np.stack([b, synth.gaussian_spinor(lat.Vh, 9232)])
    x, st = ctx.cg_solve(pack_half(ctx, bs), [kappa, 0.15], whmc.cg_params(tol=1e-12, links=whmc.L8))
    assert all(s["converged"] for s in st)
    assert rel_err(unpack_half(ctx, x, 2)[0], ref) < 1e-10


def test_8real_rejects_fields_it_cannot_represent():
    dims = (4, 4, 4, 4)
    ctx = make_ctx(dims, synth.unit_links(dims))
    for prec in (whmc.F64, whmc.F32, whmc.F16):
        xin = ctx.half_spinor(prec)
        with pytest.raises(whmc.WhmcError) as e:
            ctx.apply_H(xin, 0, prec=prec, links=whmc.L8)
        assert e.value.status == 4   # EUNSUP
    # links a tiny rotation away from the identity (|U01|^2 + |U02|^2 ~ 1e-10): FP64 represents
    # them to the FP64 bar, FP16 rejects them
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 9240, width=2e-5)
    ctx = make_ctx(dims, U)
    x = synth.gaussian_spinor(lat.Vh, 9241)
    out = ctx.apply_H(pack_half(ctx, x), 0, links=whmc.L8)
    assert rel_err(unpack_half(ctx, out), dirac.apply_Hblock(lat, U, x, 0)) < 1e-12
    with pytest.raises(whmc.WhmcError) as e:
        ctx.apply_H(ctx.half_spinor(whmc.F16), 0, prec=whmc.F16, links=whmc.L8)
    assert e.value.status == 4
