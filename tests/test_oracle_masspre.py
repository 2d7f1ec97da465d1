"""Pins for the oracle of mass preconditioning combined with the filter (oracle/masspre.py).

- The ratio M~(k_hi)^{-1} M~(k_lo) equals g(x)/(1 - x) = sum_n b_n x^n + alpha M_oo(k_hi)^{-1}:
  against dense matrix functions (scipy expm) on 2^3 x 4, and on vectors against the definition
  (series of M~ and M~^{-1}); without the filter it is rho + (1 - rho) M_oo(k_hi)^{-1}.
- Heat bath then action gives |eta|^2; the force is the derivative of the action defined by the
  solves (finite differences, not the series form the force uses).
- The determinant split with dense matrices: log|det M(kappa)|^2 equals the heavy filtered factor,
  the ratios and the gauge term -2 Re Tr sum_j K(kappa)^j / j.
- The HMC: second order in dtau, reversible, and n = 0 is the filter HMC."""
import numpy as np
import pytest
import scipy.linalg

from oracle import dirac, hmc, masspre, rooted
from oracle.lattice import Lattice
from oracle.su3 import expm_ah, from_coords
from paper_1805_03560_amd import synth

DIMS = (2, 2, 2, 4)


def _setup(seed, gen="haar"):
    lat = Lattice(DIMS)
    U = synth.haar_links(DIMS, seed) if gen == "haar" else synth.smooth_links(DIMS, seed, width=0.3)
    return lat, U


def _dense(lat, U):
    blk = dirac.dense_blocks(lat, dirac.dense_H(lat, U))
    D = blk["oe"] @ blk["eo"]
    I = np.eye(D.shape[0])
    M = lambda kap: I - kap * kap * D
    Mt = lambda kap, k: M(kap) @ scipy.linalg.expm(sum(np.linalg.matrix_power(kap * kap * D, j) / j
                                                       for j in range(1, k + 1))) if k else M(kap)
    return D, I, M, Mt


@pytest.mark.parametrize("k", [0, 1, 2])
def test_ratio_coefficients_against_dense_matrix_functions(k):
    lat, U = _setup(500)
    D, I, M, Mt = _dense(lat, U)
    k_lo, k_hi = 0.12, 0.15
    R = np.linalg.solve(Mt(k_hi, k), Mt(k_lo, k))
    b, al = masspre.ratio_coefficients((k_lo / k_hi) ** 2, k, 60)
    x = k_hi * k_hi * D
    series = al * np.linalg.inv(M(k_hi))
    xn = I.copy()
    for bn in b:
        series = series + bn * xn
        xn = xn @ x
    assert np.abs(series - R).max() < 1e-12 * np.abs(R).max()
    if k == 0:
        rho = (k_lo / k_hi) ** 2
        assert b[0] == pytest.approx(rho, rel=1e-15) and max(abs(v) for v in b[1:]) < 1e-16
        assert al == pytest.approx(1 - rho, rel=1e-15)


def test_ratio_definition_equals_the_series_form():
    lat, U = _setup(505)
    k_lo, k_hi, k = 0.12, 0.15, 2
    phi = synth.gaussian_spinor(lat.Vh, 506)
    b, al = masspre.ratio_coefficients((k_lo / k_hi) ** 2, k, 40)
    S_def = masspre.ratio_action(lat, U, phi, k_lo, k_hi, k, 40)
    assert S_def == pytest.approx(rooted.remainder_action(lat, U, phi, b, al, k_hi), rel=1e-11)


def test_ratio_heatbath_gives_the_source_norm():
    lat, U = _setup(510)
    eta = synth.gaussian_spinor(lat.Vh, 511)
    phi = masspre.ratio_heatbath(lat, U, eta, 0.11, 0.155, 2, 40)
    assert masspre.ratio_action(lat, U, phi, 0.11, 0.155, 2, 40) == pytest.approx(float(np.vdot(eta, eta).real),
                                                                                    rel=1e-10)


@pytest.mark.parametrize("k", [0, 2])
def test_ratio_force_is_the_derivative_of_the_action(k):
    lat, U = _setup(520)
    k_lo, k_hi = 0.12, 0.15
    phi = synth.gaussian_spinor(lat.Vh, 521)
    F = masspre.ratio_force(lat, U, phi, k_lo, k_hi, k, 40)
    om = synth.random_algebra(lat.dims, 522)
    S = lambda V: masspre.ratio_action(lat, V, phi, k_lo, k_hi, k, 40)
    shift = lambda e: np.einsum("...ab,...bc->...ac", expm_ah(e * from_coords(om)), U)
    h = 1e-3
    fd = (8 * (S(shift(h)) - S(shift(-h))) - (S(shift(2 * h)) - S(shift(-2 * h)))) / (12 * h)
    assert float(np.sum(om * F)) == pytest.approx(fd, rel=1e-6)


def test_filtered_ratio_force_is_small():
    """the filter on the ratio cancels its low orders in K: its force is far below the force of the
    unfiltered ratio on the same field and source (the point of filtering every factor)."""
    lat, U = _setup(525)     # rough field: 2 % (on a near-free smooth field the infrared keeps ~20 %)
    phi = synth.gaussian_spinor(lat.Vh, 526)
    f0 = masspre.ratio_force(lat, U, phi, 0.13, 0.15, 0, 30)
    f2 = masspre.ratio_force(lat, U, phi, 0.13, 0.15, 2, 30)
    assert np.sum(f2 * f2) < 0.1 * np.sum(f0 * f0)


def test_determinant_splits_into_heavy_factor_ratios_and_gauge_term():
    lat, U = _setup(530)
    D, I, M, Mt = _dense(lat, U)
    k = 2
    ks = [0.10, 0.13, 0.155]
    logdet = lambda A: np.linalg.slogdet(A)[1]
    total = 2 * logdet(M(ks[-1]))
    parts = 2 * logdet(Mt(ks[0], k))
    for lo, hi in zip(ks[:-1], ks[1:]):
        R = np.linalg.solve(Mt(hi, k), Mt(lo, k))   # the ratio operator of the action
        parts -= logdet(R.conj().T @ R)             # its Gaussian integral is 1 / det(R^dag R)
    K = ks[-1] ** 2 * D
    parts -= 2 * np.trace(K + K @ K / 2).real       # the gauge term of the filter at kappa
    assert total == pytest.approx(parts, rel=1e-12)


def _hmc_setup(seed, p):
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, seed, width=0.3)
    pi = synth.gaussian_momenta(DIMS, seed + 1)
    etas = [synth.gaussian_spinor(lat.Vh, seed + 2 + f) for f in range(len(p.kappas) + 1)]
    return lat, U, pi, etas


def test_mp_md_is_second_order_and_reversible():
    """n_t = n_max: the force is the exact derivative of the series-form action in H."""
    base = masspre.MassPreParams(kappa=0.15, kappas=(0.12,), k=2, n_t=8, n_max=8, integrator="omelyan", m=2,
                                 msub=(1, 1), tau=0.3)
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
    assert 3.5 < r1 < 4.8 and 3.6 < r2 < 4.5, dHs


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
