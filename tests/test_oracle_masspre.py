"""Pins for the oracle of mass preconditioning combined with the filter (oracle/masspre.py).

- The ratio M_oo(k_hi)^{-1} M_oo(k_lo) equals rho + (1 - rho) M_oo(k_hi)^{-1} (both are polynomials
  in the one matrix D = H_oe H_eo); checked on vectors and on the action computed both ways.
- Heat bath then action gives |eta|^2; the force is the derivative of the action defined by the
  solves (finite differences, not the series form the force uses).
- The determinant split: with dense matrices on 2^3 x 4, log det M(kappa)^dag M(kappa) equals the
  heavy factor plus the ratios.
- The HMC: second order in dtau, reversible, and n = 0 is the filter HMC."""
import numpy as np
import pytest

from oracle import dirac, hmc, masspre, rooted
from oracle.lattice import Lattice
from oracle.su3 import expm_ah, from_coords
from paper_1805_03560_amd import synth

DIMS = (2, 2, 2, 4)


def _setup(seed, gen="haar"):
    lat = Lattice(DIMS)
    U = synth.haar_links(DIMS, seed) if gen == "haar" else synth.smooth_links(DIMS, seed, width=0.3)
    return lat, U


def test_ratio_is_the_two_term_series():
    lat, U = _setup(500)
    k_lo, k_hi = 0.12, 0.15
    phi = synth.gaussian_spinor(lat.Vh, 501)
    rho = (k_lo / k_hi) ** 2
    lhs = masspre.moo_inverse(lat, U, dirac.apply_Moo(lat, U, phi, k_lo), k_hi, 1e-14)
    rhs = rho * phi + (1 - rho) * masspre.moo_inverse(lat, U, phi, k_hi, 1e-14)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()
    S_def = masspre.ratio_action(lat, U, phi, k_lo, k_hi)
    assert S_def == pytest.approx(rooted.remainder_action(lat, U, phi, [rho], 1 - rho, k_hi), rel=1e-12)


def test_ratio_heatbath_gives_the_source_norm():
    lat, U = _setup(510)
    eta = synth.gaussian_spinor(lat.Vh, 511)
    phi = masspre.ratio_heatbath(lat, U, eta, 0.11, 0.155)
    assert masspre.ratio_action(lat, U, phi, 0.11, 0.155) == pytest.approx(float(np.vdot(eta, eta).real), rel=1e-11)


def test_ratio_force_is_the_derivative_of_the_action():
    lat, U = _setup(520)
    k_lo, k_hi = 0.12, 0.15
    phi = synth.gaussian_spinor(lat.Vh, 521)
    F = masspre.ratio_force(lat, U, phi, k_lo, k_hi)
    om = synth.random_algebra(lat.dims, 522)
    S = lambda V: masspre.ratio_action(lat, V, phi, k_lo, k_hi)
    shift = lambda e: np.einsum("...ab,...bc->...ac", expm_ah(e * from_coords(om)), U)
    h = 1e-3
    fd = (8 * (S(shift(h)) - S(shift(-h))) - (S(shift(2 * h)) - S(shift(-2 * h)))) / (12 * h)
    assert float(np.sum(om * F)) == pytest.approx(fd, rel=1e-6)


def test_determinant_splits_into_heavy_factor_and_ratios():
    """dense: log det M_oo(kappa)^dag M_oo(kappa) = log det of the heaviest factor plus the logs of
    the ratio matrices whose Gaussian integrals the ratio fields represent."""
    lat, U = _setup(530)
    Hm = dirac.dense_H(lat, U)
    blk = dirac.dense_blocks(lat, Hm)
    D = blk["oe"] @ blk["eo"]
    I = np.eye(D.shape[0])
    M = lambda k: I - k * k * D
    ks = [0.10, 0.13, 0.155]
    logdet = lambda A: np.linalg.slogdet(A)[1]
    total = logdet(M(ks[-1]).conj().T @ M(ks[-1]))
    parts = logdet(M(ks[0]).conj().T @ M(ks[0]))
    for lo, hi in zip(ks[:-1], ks[1:]):
        R = np.linalg.solve(M(hi), M(lo))           # the ratio operator of the action
        parts -= logdet(R.conj().T @ R)             # its Gaussian integral is 1 / det(R^dag R)
    assert total == pytest.approx(parts, rel=1e-12)


def _hmc_setup(seed, p):
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, seed, width=0.3)
    pi = synth.gaussian_momenta(DIMS, seed + 1)
    etas = [synth.gaussian_spinor(lat.Vh, seed + 2 + f) for f in range(len(p.kappas) + 1)]
    return lat, U, pi, etas


def test_mp_md_is_second_order_and_reversible():
    base = masspre.MassPreParams(kappa=0.15, kappas=(0.11, 0.13), k=2, n_t=8, n_max=8, integrator="omelyan", m=2,
                                 msub=(1, 1, 2), tau=0.5)
    lat, U, pi, etas = _hmc_setup(540, base)
    phis = masspre.mp_heatbath(lat, U, etas, base)
    dHs = []
    for m in (2, 4, 8):
        p = masspre.MassPreParams(**{**base.__dict__, "m": m})
        U1, pi1 = masspre.mp_integrate(lat, U, pi, phis, p)
        dHs.append(masspre.mp_hamiltonian(lat, U1, pi1, phis, p) - masspre.mp_hamiltonian(lat, U, pi, phis, p))
        if m == 2:
            U2, _ = masspre.mp_integrate(lat, U1, -pi1, phis, p)
            assert float(np.sum(np.abs(U - U2) ** 2)) < 1e-22
    r1, r2 = dHs[0] / dHs[1], dHs[1] / dHs[2]
    assert 3.0 < r1 < 5.5 and 3.5 < r2 < 4.6, dHs


def test_mp_without_ratios_is_the_filter_hmc():
    p = masspre.MassPreParams(kappa=0.15, kappas=(), k=1, n_t=5, n_max=19, integrator="leapfrog", m=3, msub=(2,),
                              tau=0.4)
    lat, U, pi, etas = _hmc_setup(550, p)
    ref = hmc.trajectory(lat, U, pi, etas[0], 0.5, hmc.HMCParams(beta=p.beta, kappa=0.15, k=1, n_t=5, n_max=19,
                                                                   integrator="leapfrog", m=3, m0=2, tau=0.4,
                                                                   tol=1e-14))
    res = masspre.mp_trajectory(lat, U, pi, etas, 0.5, p)
    assert res["H0"] == pytest.approx(ref["H0"], rel=1e-13)
    assert res["dH"] == pytest.approx(ref["dH"], abs=1e-10)
    assert np.abs(res["U_end"] - ref["U_end"]).max() < 1e-13
