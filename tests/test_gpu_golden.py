"""The 32^3 x 64 solve of the benchmark (smooth links seed 3000, width 0.3; source seed 3003;
kappa = 0.1575) against the oracle's own solution stored at 4096 sampled sites
(tests/golden/cg_32x64_kappa0.1575.*, written by tests/golden/make_cg_32x64.py, which calls only
the oracle; its CG reached a true residual of 7.5e-15).  The GPU solves run in the launch
configuration of the benchmark (streaming links, per-XCD slice schedule)."""
import json
import os

import numpy as np
import pytest
import torch

from paper_1805_03560_amd import synth, whmc

from gpu_util import dev

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DIMS = (64, 32, 32, 32)


@pytest.fixture(scope="module")
def case():
    z = np.load(os.path.join(HERE, "cg_32x64_kappa0.1575.npz"), allow_pickle=False)
    meta = json.load(open(os.path.join(HERE, "cg_32x64_kappa0.1575.json")))
    U = synth.smooth_links(DIMS, 3000, width=0.3, threads=16)
    ctx = whmc.Context(DIMS)
    ctx.load_gauge(torch.from_numpy(U).to(dev()), unitarity_tol=1e-11)
    del U
    b = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(ctx.Vh, 3003)).to(dev()), 0)
    yield ctx, b, z["sites"], z["x"], meta
    ctx.close()


def _sampled(ctx, x, sites):
    return ctx.unpack_spinor(x, 0).index_select(0, torch.from_numpy(sites).to(dev())).cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_fp64_solve_matches_the_oracle_solution(case):
    ctx, b, sites, ref, meta = case
    x, st = ctx.cg_solve(b, [0.1575], whmc.cg_params(tol=1e-14, maxiter=2000))
    assert st[0]["converged"]
    got = _sampled(ctx, x, sites)
    assert _rel(got, ref) < 1e-11
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-11
    # the norm of the whole solution against the oracle's
    assert float(torch.linalg.vector_norm(x)) == pytest.approx(meta["norm_x"], rel=1e-11)


@pytest.mark.parametrize("prm", [dict(), dict(links=whmc.L12), dict(links=whmc.L8),
                                 dict(prec=whmc.F32, links=whmc.L12, delta=1e-4),
                                 dict(prec=whmc.F16, links=whmc.L12, delta=1e-2),
                                 dict(prec=whmc.F16, links=whmc.L8, delta=1e-2)])
def test_workload_solves_to_1e10_against_the_oracle(case, prm):
    """every solver format of the benchmark reaches the true residual 1e-10; its error against the
    oracle solution is then bounded by cond(A) x 1e-10 (cond ~ 10 on this field: 2e-10 measured)"""
    ctx, b, sites, ref, _ = case
    x, st = ctx.cg_solve(b, [0.1575], whmc.cg_params(tol=1e-10, **prm))
    assert st[0]["converged"] and st[0]["true_residual"] <= 1e-10
    assert _rel(_sampled(ctx, x, sites), ref) < 5e-9
