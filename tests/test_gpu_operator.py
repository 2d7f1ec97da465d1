"""GPU parity of the hopping matrix, M_oo and M_oo^dag M_oo against the oracle (element by
element, FP64 to 1e-12 relative), low-precision formats within their rounding, and sampled
outputs at the full 32^3 x 64 size."""
import numpy as np
import pytest

from oracle import dirac
from oracle.lattice import Lattice
from paper_1805_03560_amd import synth, whmc

from gpu_util import (make_ctx, pack_full, pack_half, rel_err, to_dev, unpack_full, unpack_half)

pytestmark = pytest.mark.gpu

# several tiles and a ragged tail (Vh = 288, 1728 are not multiples of 256), the degenerate 2^4;
# (6, 8, 16, 16) has time slices of 1024 = 8 x 128 sites, so the stencil kernels give each XCD one
# eighth of every slice (the schedule used at 32^3 x 64) instead of one eighth of the lattice;
# (4, 12, 16, 16) has slices of 12 blocks, cut 1/2/1/2/... per XCD with idle padding workgroups
# (the schedule used at 24^3 x 48)
SLICED = (6, 8, 16, 16)
PADDED = (4, 12, 16, 16)
DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 4, 6, 6), (6, 4, 6, 8), (8, 6, 4, 12), SLICED, PADDED]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("out_parity", [0, 1])
@pytest.mark.parametrize("dagger", [0, 1])
def test_hop_eo_fp64_parity(dims, out_parity, dagger):
    lat = Lattice(dims)
    U = synth.haar_links(dims, 1000)
    x = synth.gaussian_spinor(lat.Vh, 1001)
    ref = dirac.apply_Hblock(lat, U, x, out_parity, dagger=bool(dagger))
    ctx = make_ctx(dims, U)
    for links in (whmc.L18, whmc.L12):
        out = ctx.apply_H(pack_half(ctx, x), out_parity, dagger=dagger, prec=whmc.F64, links=links)
        assert rel_err(unpack_half(ctx, out), ref) < 1e-12, links


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 6, 8), SLICED, PADDED])
def test_full_H_parity(dims):
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 1010)
    psi = synth.gaussian_spinor(lat.V, 1011).reshape(dims + (4, 3))
    ctx = make_ctx(dims, U)
    for dagger in (0, 1):
        ref = dirac.apply_Hdag(lat, U, psi) if dagger else dirac.apply_H(lat, U, psi)
        out = ctx.apply_H(pack_full(ctx, psi), -1, dagger=dagger)
        assert rel_err(unpack_full(ctx, out), ref) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 4, 6, 6), SLICED, PADDED])
def test_Moo_and_MdagM_parity(dims):
    lat = Lattice(dims)
    U = synth.haar_links(dims, 1020)
    x = synth.gaussian_spinor(lat.Vh, 1021)
    kappa = 0.156
    ctx = make_ctx(dims, U)
    xb = pack_half(ctx, x)
    assert rel_err(unpack_half(ctx, ctx.apply_Moo(xb, kappa)), dirac.apply_Moo(lat, U, x, kappa)) < 1e-12
    assert rel_err(unpack_half(ctx, ctx.apply_Moo(xb, kappa, dagger=True)),
                   dirac.apply_Moo_dag(lat, U, x, kappa)) < 1e-12
    assert rel_err(unpack_half(ctx, ctx.apply_MdagM(xb, [kappa])), dirac.apply_MooDagMoo(lat, U, x, kappa)) < 1e-12


def test_layout_round_trips():
    dims = (4, 4, 6, 6)
    lat = Lattice(dims)
    ctx = make_ctx(dims, synth.haar_links(dims, 1030))
    x = synth.gaussian_spinor(lat.Vh, 1031)
    assert np.array_equal(unpack_half(ctx, pack_half(ctx, x)), x)
    full = synth.gaussian_spinor(lat.V, 1032).reshape(dims + (4, 3))
    assert np.array_equal(unpack_full(ctx, pack_full(ctx, full)), full)
    U = synth.haar_links(dims, 1030)
    assert np.array_equal(ctx.export_gauge().cpu().numpy(), U)
    a = synth.random_algebra(dims, 1033)
    assert np.array_equal(ctx.unpack_algebra(ctx.pack_algebra(to_dev(a))).cpu().numpy(), a)


def test_non_su3_field_rejected():
    dims = (2, 2, 2, 4)
    U = synth.haar_links(dims, 1040)
    U[0, 0, 0, 1, 2] *= 1.001
    ctx = whmc.Context(dims)
    with pytest.raises(whmc.WhmcError) as e:
        ctx.load_gauge(to_dev(U), unitarity_tol=1e-10)
    assert e.value.status == 5


def test_bad_arguments_raise():
    with pytest.raises(whmc.WhmcError):
        whmc.Context((3, 4, 4, 4))
    ctx = whmc.Context((4, 4, 4, 4))
    with pytest.raises(whmc.WhmcError) as e:
        ctx.apply_H(ctx.half_spinor(), 0)      # no gauge field yet
    assert e.value.status == 6


@pytest.mark.parametrize("prec,links,tol", [(whmc.F32, whmc.L18, 2e-6), (whmc.F32, whmc.L12, 2e-6),
                                            (whmc.F16, whmc.L12, 4e-3)])
def test_hop_low_precision(prec, links, tol):
    dims = (4, 4, 6, 6)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 1050)
    x = synth.gaussian_spinor(lat.Vh, 1051)
    ref = dirac.apply_Hblock(lat, U, x, 1)
    ctx = make_ctx(dims, U)
    xin = ctx.convert_spinor(pack_half(ctx, x), whmc.F64, prec)
    out = ctx.apply_H(xin, 1, prec=prec, links=links)
    got = unpack_half(ctx, ctx.convert_spinor(out, prec, whmc.F64))
    assert rel_err(got, ref) < tol


def test_full_size_hop_sampled_sites():
    """32^3 x 64 (the mixed-precision workload's lattice): sampled outputs against the oracle's
    per-site evaluation, in the launch configuration the benchmark times."""
    dims = (64, 32, 32, 32)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 3000)
    x = synth.gaussian_spinor(lat.Vh, 3001)
    ctx = make_ctx(dims, U)
    out = unpack_half(ctx, ctx.apply_H(pack_half(ctx, x), 0))
    full_in = np.zeros((lat.V, 4, 3), dtype=np.complex128)
    full_in[lat.sites_of_parity(1)] = x
    even_sites = lat.sites_of_parity(0)
    pick = np.random.default_rng(7).choice(lat.Vh, 256, replace=False)
    pick = np.concatenate([pick, [0, lat.Vh - 1]])
    ref = dirac.hop_at_sites(lat, U.reshape(lat.V, 4, 3, 3), full_in, even_sites[pick])
    assert rel_err(out[pick], ref) < 1e-12
