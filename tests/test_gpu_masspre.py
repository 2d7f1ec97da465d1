"""GPU parity of mass preconditioning combined with the filter (Sec. 1, 5) against the oracle.

The oracle computes each ratio action from its definition (two solves); the library uses the
equivalent two-term series, so the action parity also checks that identity on the GPU.
Tolerances as for the filter: solves to 1e-14 on both sides, forces 1e-10 relative."""
import numpy as np
import pytest

from oracle import masspre
from oracle.lattice import Lattice
from paper_1805_03560_amd import synth, whmc

from gpu_util import algebra_to_numpy, make_ctx, pack_half, rel_err, to_dev, unpack_half

pytestmark = pytest.mark.gpu

SOLVER = whmc.cg_params(tol=1e-14, check_every=4)


def _sources(lat, n, seed):
    return np.stack([synth.gaussian_spinor(lat.Vh, seed + f) for f in range(n)])


# (heavier kappas, kappa, k, n_t, n_max)
CASES = [((0.13,), 0.156, 2, 7, 29), ((0.10, 0.14), 0.156, 1, 5, 19), ((), 0.156, 2, 7, 29)]


@pytest.mark.parametrize("kappas,kappa,k,n_t,n_max", CASES)
@pytest.mark.parametrize("dims,gen,scale", [((4, 4, 4, 4), "haar", 1.0), ((4, 2, 2, 8), "smooth", 0.8)])
def test_masspre_heatbath_action_force_parity(kappas, kappa, k, n_t, n_max, dims, gen, scale):
    lat = Lattice(dims)
    U = synth.haar_links(dims, 5000) if gen == "haar" else synth.smooth_links(dims, 5000, width=0.3)
    kappas = tuple(scale * v for v in kappas)
    kappa = scale * kappa
    p = masspre.MassPreParams(kappa=kappa, kappas=kappas, k=k, n_t=n_t, n_max=n_max, tol=1e-14)
    nf = len(kappas) + 1
    etas = _sources(lat, nf, 5010)
    ctx = make_ctx(dims, U)
    mp = whmc.masspre(kappas, k=k, n_t=n_t, n_max=n_max)

    phis_ref = masspre.mp_heatbath(lat, U, list(etas), p)
    got = unpack_half(ctx, ctx.masspre_heatbath(pack_half(ctx, etas), mp, kappa, solver=SOLVER), nf)
    got = got.reshape(nf, lat.Vh, 4, 3)     # one field unpacks without the field axis
    for f in range(nf):
        assert rel_err(got[f], phis_ref[f]) < 1e-10, f

    phi_b = pack_half(ctx, np.stack(phis_ref))
    S = ctx.masspre_action(phi_b, mp, kappa, solver=SOLVER)
    H_ref = masspre.mp_hamiltonian(lat, U, np.zeros((*dims, 4, 8)), phis_ref, p)
    from oracle import gauge, hpe
    chain = list(kappas) + [kappa]
    S_G = gauge.gauge_action(lat, U, p.beta + hpe.delta_beta(kappa, k))    # the gauge term of the target kappa
    assert sum(S) == pytest.approx(H_ref - S_G, rel=1e-11)
    for i in range(len(kappas)):
        ref = masspre.ratio_action_series(lat, U, phis_ref[i + 1], chain[i], chain[i + 1], k, n_max)
        assert S[i + 1] == pytest.approx(ref, rel=1e-11)
        # the definition M~(kappa_{i+1})^{-1} M~(kappa_i) phi, up to the truncation at n_max
        assert S[i + 1] == pytest.approx(masspre.ratio_action(lat, U, phis_ref[i + 1], chain[i], chain[i + 1], k,
                                                              n_max), rel=1e-9)
        # heat bath sets each ratio action to the norm of its source
        assert S[i + 1] == pytest.approx(float(np.vdot(etas[i + 1], etas[i + 1]).real), rel=1e-9)

    refs = masspre.mp_forces(lat, phis_ref, p)
    total = 0.0
    for t in range(1, nf + 1):
        F = algebra_to_numpy(ctx, ctx.masspre_force(phi_b, mp, kappa, term=t, solver=SOLVER))
        ref = refs[t](U)
        assert rel_err(F, ref) < 1e-10, t
        total = total + ref
    F = algebra_to_numpy(ctx, ctx.masspre_force(phi_b, mp, kappa, term=0, solver=SOLVER))
    assert rel_err(F, total) < 1e-10


def _wp(p, integrator):
    return whmc.masspre_hmc_params(beta=p.beta, kappa=p.kappa, mp=whmc.masspre(p.kappas, k=p.k, n_t=p.n_t,
                                                                                n_max=p.n_max),
                                   integrator=integrator, lam=p.lam, m=p.m, msub=p.msub, tau=p.tau,
                                   md_solver=SOLVER, action_solver=SOLVER)


@pytest.mark.parametrize("integrator,kappas,k", [("omelyan", (0.12,), 2), ("leapfrog", (0.10, 0.13), 1)])
def test_masspre_trajectory_parity(integrator, kappas, k):
    dims = (4, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 5030)
    pi = synth.gaussian_momenta(dims, 5031)
    p = masspre.MassPreParams(kappa=0.15, kappas=kappas, k=k, n_t=6, n_max=19, integrator=integrator, m=3,
                              msub=(2, 2, 1)[:len(kappas) + 1], tau=0.5, tol=1e-14)
    etas = _sources(lat, len(kappas) + 1, 5032)
    ref = masspre.mp_trajectory(lat, U, pi, list(etas), 0.5, p)
    ctx = make_ctx(dims, U)
    wp = _wp(p, whmc.OMELYAN if integrator == "omelyan" else whmc.LEAPFROG)
    res = ctx.masspre_trajectory(wp, ctx.pack_algebra(to_dev(pi)), pack_half(ctx, etas), 0.5)
    assert res["H0"] == pytest.approx(ref["H0"], rel=1e-12)
    assert res["dH"] == pytest.approx(ref["dH"], abs=1e-8)
    assert bool(res["accepted"]) == ref["accepted"]
    assert rel_err(ctx.export_gauge().cpu().numpy(), ref["U"]) < 1e-10


def test_masspre_md_reversibility_and_dtau_scaling():
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 5040)
    pi0 = synth.gaussian_momenta(dims, 5041)
    etas = _sources(lat, 3, 5042)
    ctx = make_ctx(dims, U)
    dHs = []
    for m in (4, 8, 16):    # at m = 2 the ratio is still 5.7, not yet asymptotic
        p = masspre.MassPreParams(kappa=0.15, kappas=(0.11, 0.13), k=2, n_t=8, n_max=8, integrator="omelyan", m=m,
                                  msub=(1, 1, 2), tau=0.5)
        wp = _wp(p, whmc.OMELYAN)
        ctx.load_gauge(to_dev(U))
        phi = ctx.masspre_heatbath(pack_half(ctx, etas), wp.mp, p.kappa, solver=SOLVER)
        pi = ctx.pack_algebra(to_dev(pi0))
        H0 = ctx.masspre_hamiltonian(wp, pi, phi)
        ctx.masspre_md_integrate(wp, pi, phi)
        dHs.append(ctx.masspre_hamiltonian(wp, pi, phi) - H0)
        if m == 8:
            ctx.masspre_md_integrate(wp, -pi, phi)   # flip momenta and integrate back
            assert float(np.sum(np.abs(ctx.export_gauge().cpu().numpy() - U) ** 2)) < 1e-20
    assert 3.0 < dHs[0] / dHs[1] < 5.5 and 3.3 < dHs[1] / dHs[2] < 4.8, dHs


def test_masspre_without_ratios_is_the_filter_trajectory():
    dims = (4, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 5050)
    pi = synth.gaussian_momenta(dims, 5051)
    eta = synth.gaussian_spinor(lat.Vh, 5052)
    ctx = make_ctx(dims, U)
    fp = whmc.hmc_params(beta=5.6, kappa=0.15, k=2, n_t=6, n_max=29, integrator=whmc.OMELYAN, m=3, m0=2, tau=0.5,
                         md_solver=SOLVER, action_solver=SOLVER)
    ref = ctx.hmc_trajectory(fp, ctx.pack_algebra(to_dev(pi)), pack_half(ctx, eta), 0.5)
    U_ref = ctx.export_gauge().cpu().numpy()
    ctx.load_gauge(to_dev(U))
    wp = whmc.masspre_hmc_params(beta=5.6, kappa=0.15, mp=whmc.masspre((), k=2, n_t=6, n_max=29),
                                 integrator=whmc.OMELYAN, m=3, msub=(2,), tau=0.5, md_solver=SOLVER,
                                 action_solver=SOLVER)
    res = ctx.masspre_trajectory(wp, ctx.pack_algebra(to_dev(pi)), pack_half(ctx, eta), 0.5)
    assert res["H0"] == pytest.approx(ref["H0"], rel=1e-13)
    assert res["dH"] == pytest.approx(ref["dH"], abs=1e-10)
    assert rel_err(ctx.export_gauge().cpu().numpy(), U_ref) < 1e-12


def test_masspre_rejects_bad_arguments():
    dims = (4, 2, 2, 4)
    lat = Lattice(dims)
    ctx = make_ctx(dims, synth.smooth_links(dims, 5060))
    phi = pack_half(ctx, _sources(lat, 2, 5061))
    with pytest.raises(whmc.WhmcError):
        ctx.masspre_action(phi, whmc.masspre((0.16,)), 0.15)           # heavier kappa above kappa
    with pytest.raises(whmc.WhmcError):
        ctx.masspre_action(phi, whmc.masspre((0.13, 0.12)), 0.15)      # not increasing
    with pytest.raises(whmc.WhmcError):
        ctx.masspre_force(phi, whmc.masspre((0.12,)), 0.15, term=3)


def test_masspre_four_heavier_kappas():
    """n = WHMC_MAX_MASSPRE: four ratios, each with its own series, against the oracle."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 5070)
    kappas, kappa = (0.09, 0.11, 0.13, 0.145), 0.156
    p = masspre.MassPreParams(kappa=kappa, kappas=kappas, k=2, n_t=7, n_max=29, tol=1e-14)
    etas = _sources(lat, 5, 5071)
    ctx = make_ctx(dims, U)
    mp = whmc.masspre(kappas, k=2, n_t=7, n_max=29)
    phis_ref = masspre.mp_heatbath(lat, U, list(etas), p)
    got = unpack_half(ctx, ctx.masspre_heatbath(pack_half(ctx, etas), mp, kappa, solver=SOLVER), 5)
    for f in range(5):
        assert rel_err(got[f], phis_ref[f]) < 1e-10, f
    phi_b = pack_half(ctx, np.stack(phis_ref))
    refs = masspre.mp_forces(lat, phis_ref, p)
    for t in range(1, 6):
        F = algebra_to_numpy(ctx, ctx.masspre_force(phi_b, mp, kappa, term=t, solver=SOLVER))
        assert rel_err(F, refs[t](U)) < 1e-10, t
