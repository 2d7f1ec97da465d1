"""Pins for the oracle's HMC: both integrators are second order (Delta H ~ dtau^2), the
trajectory is reversible to rounding (eq. reverse), the heat bath makes S~_PF = |eta|^2, and
Metropolis follows min[1, exp(-Delta H)]."""
import numpy as np
import pytest

from oracle import hmc, hpe
from oracle.lattice import Lattice
from paper_1805_03560_amd import synth

DIMS = (2, 2, 2, 4)


def _setup(seed=200):
    lat = Lattice(DIMS)
    U = synth.smooth_links(DIMS, seed, width=0.3)
    pi = synth.gaussian_momenta(DIMS, seed + 1)
    eta = synth.gaussian_spinor(lat.Vh, seed + 2)
    return lat, U, pi, eta


@pytest.mark.parametrize("integrator,k,n_t", [("leapfrog", 0, 0), ("omelyan", 2, 7)])
def test_delta_H_scales_as_dtau_squared(integrator, k, n_t):
    """with n_t = n_max the force is the exact derivative of the action in H, so Delta H -> 0 as
    dtau^2; with n_t < n_max a dtau-independent truncation part remains (Sec. 2)."""
    lat, U, pi, eta = _setup()
    dHs = []
    for m in (2, 4, 8):
        p = hmc.HMCParams(beta=5.6, kappa=0.15, k=k, n_t=n_t, n_max=n_t, integrator=integrator,
                          m=m, m0=2, tau=0.5, tol=1e-14)
        phi = hpe.heatbath_phi(lat, U, eta, p.kappa, p.k, p.n_max)
        U1, pi1 = hmc.integrate(lat, U, pi, phi, p)
        dHs.append(hmc.hamiltonian(lat, U1, pi1, phi, p) - hmc.hamiltonian(lat, U, pi, phi, p))
    r1, r2 = dHs[0] / dHs[1], dHs[1] / dHs[2]
    assert 3.0 < r1 < 5.5 and 3.5 < r2 < 4.6, dHs


def test_reversibility_to_rounding():
    lat, U, pi, eta = _setup(210)
    p = hmc.HMCParams(beta=5.6, kappa=0.15, k=1, n_t=5, n_max=19, integrator="omelyan", m=3, m0=2, tau=0.5,
                      tol=1e-14)
    phi = hpe.heatbath_phi(lat, U, eta, p.kappa, p.k, p.n_max)
    delta = hmc.reversibility(lat, U, pi, phi, p)
    assert delta < 1e-22


def test_heat_bath_gives_eta_norm_and_metropolis():
    lat, U, pi, eta = _setup(220)
    p = hmc.HMCParams(beta=5.6, kappa=0.15, k=2, n_t=5, n_max=29, integrator="leapfrog", m=2, m0=2, tau=0.3,
                      tol=1e-14)
    phi = hpe.heatbath_phi(lat, U, eta, p.kappa, p.k, p.n_max)
    S = hpe.filtered_action(lat, U, phi, p.kappa, p.k, p.n_max, tol=1e-14)
    assert S == pytest.approx(float(np.sum(np.abs(eta) ** 2)), rel=1e-10)
    res = hmc.trajectory(lat, U, pi, eta, 0.5, p)
    assert res["accepted"] == (0.5 < np.exp(-res["dH"]))
    assert abs(res["dH"]) < 1.0
    res_rej = hmc.trajectory(lat, U, pi, eta, 1.0 - 1e-16 if res["dH"] > 0 else 2.0, p)
    assert not res_rej["accepted"] and np.array_equal(res_rej["U"], U)
