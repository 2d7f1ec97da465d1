"""The entry point that allocates nothing, whmc_apply_MdagM_noalloc, against whmc_apply_MdagM:
two calls in a row, the second on a smaller lattice, for the even/odd and the full-lattice
operator; lattices whose intermediates exceed the static scratch are rejected."""
import numpy as np
import pytest
import torch

from paper_1805_03560_amd import synth, whmc

from gpu_util import make_ctx, to_dev

pytestmark = pytest.mark.gpu


def _apply_both(dims, kappas, eo, seed):
    U = synth.smooth_links(dims, seed)
    ctx = make_ctx(dims, U)
    n_sites = ctx.Vh if eo else ctx.V
    x = np.stack([synth.gaussian_spinor(n_sites, seed + 1 + r) for r in range(len(kappas))])
    xb = ctx.pack_spinor(to_dev(x), 0 if eo else -1)
    ref = ctx.apply_MdagM(xb, kappas, eo=eo)
    out = torch.full_like(ref, float("nan"))
    ctx.apply_MdagM_noalloc(xb, kappas, out, eo=eo)
    return ctx, ref, out


@pytest.mark.parametrize("eo", [True, False])
def test_noalloc_matches_apply_MdagM_on_two_calls(eo):
    # first call: 16^3 x 32 (the largest standard lattice that fits the static scratch), two rhs
    ctx1, ref1, out1 = _apply_both((32, 16, 16, 16), [0.156, 0.1575], eo, 9000)
    assert bool((out1 == ref1).all()), float((out1 - ref1).abs().max())
    # second call: a smaller lattice in a new context on the same GPU, one rhs
    ctx2, ref2, out2 = _apply_both((4, 4, 6, 8), [0.12], eo, 9010)
    assert bool((out2 == ref2).all()), float((out2 - ref2).abs().max())


def test_noalloc_rejects_lattices_beyond_the_scratch():
    dims = (24, 16, 16, 32)   # V * 192 bytes = 37.7 MB > 32 MiB
    ctx = make_ctx(dims, synth.unit_links(dims))
    x = ctx.half_spinor()
    out = ctx.half_spinor()
    with pytest.raises(whmc.WhmcError) as e:
        ctx.apply_MdagM_noalloc(x, [0.12], out)
    assert e.value.status == 1   # EARG
    assert ctx.V * 192 > whmc.NOALLOC_SCRATCH_BYTES
