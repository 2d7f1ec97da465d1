"""Mass preconditioning combined with kappa^(2k) filtering (oracle, test only).

Sec. 1 splits the fermion matrix into factors, each with its own pseudo-fermion field and its own
time scale.  The conclusion (Sec. 5) proposes combining the filter with mass preconditioning.
Reading: with heavier hopping parameters kappa_1 < ... < kappa_n < kappa_{n+1} = kappa,
    det M_oo(kappa) = det M_oo(kappa_1) prod_{i=1..n} det M_oo(kappa_{i+1}) / det M_oo(kappa_i).
The heaviest factor is the one that is filtered: det M_oo(kappa_1) = det M~(kappa_1) times the
gauge term of the filter at kappa_1 (beta -> beta + 96 kappa_1^4 for k = 2), so its field has the
action |M~(kappa_1)^{-1} phi_1|^2 of Sec. 2.  Each ratio has the action
    S_i = |M_oo(kappa_{i+1})^{-1} M_oo(kappa_i) phi|^2      (Gaussian integral = the ratio of det M^dag M)
with the heat bath phi = M_oo(kappa_i)^{-1} M_oo(kappa_{i+1}) eta.

Force of a ratio.  M_oo(kappa) = 1 - kappa^2 D with D = H_oe H_eo for every kappa, so the two
factors commute and, with rho = kappa_i^2 / kappa_{i+1}^2,
    M_oo(kappa_{i+1})^{-1} M_oo(kappa_i) = rho + (1 - rho) M_oo(kappa_{i+1})^{-1},
a series action with b_0 = rho and alpha = 1 - rho at kappa_{i+1}; its force is the Horner
construction of Sec. 2 with those two coefficients.  The action itself is computed from the
definition above, so the tests compare the two forms.

HMC levels (reading): gauge action on level 0, the filtered heavy field on level 1, the ratios on
levels 2 .. n + 1 from the heaviest to the lightest (the lightest has the smallest force and the
most expensive solve, so it takes the coarsest step).
"""
from dataclasses import dataclass

import numpy as np

from . import dirac, gauge, hmc, hpe
from .force import solve_MMdag_oo
from .rooted import series_force


def moo_inverse(lat, U, v, kappa, tol):
    """M_oo(kappa)^{-1} v = M_oo^dag (M_oo M_oo^dag)^{-1} v."""
    return dirac.apply_Moo_dag(lat, U, solve_MMdag_oo(lat, U, v, kappa, tol), kappa)


def ratio_action(lat, U, phi, k_lo, k_hi, tol=1e-14):
    """|M_oo(k_hi)^{-1} M_oo(k_lo) phi|^2, from the definition."""
    z = moo_inverse(lat, U, dirac.apply_Moo(lat, U, phi, k_lo), k_hi, tol)
    return float(np.vdot(z, z).real)


def ratio_heatbath(lat, U, eta, k_lo, k_hi, tol=1e-14):
    """phi = M_oo(k_lo)^{-1} M_oo(k_hi) eta."""
    return moo_inverse(lat, U, dirac.apply_Moo(lat, U, eta, k_hi), k_lo, tol)


def ratio_force(lat, U, phi, k_lo, k_hi, tol=1e-14):
    """force of the ratio action as the series rho + (1 - rho) M_oo(k_hi)^{-1}."""
    rho = (k_lo / k_hi) ** 2
    return series_force(lat, U, phi, [rho], 1.0 - rho, k_hi, tol)


@dataclass
class MassPreParams:
    beta: float = 5.6
    kappa: float = 0.156
    kappas: tuple = (0.14,)     # kappa_1 < ... < kappa_n < kappa
    k: int = 2                  # filter of the heaviest factor
    n_t: int = 15
    n_max: int = 29
    integrator: str = "omelyan"
    lam: float = 1.0 / 6.0
    m: int = 4                  # steps of the lightest ratio per trajectory
    msub: tuple = (2, 2)        # m_0 .. m_n: steps of level l-1 per step of level l
    tau: float = 1.0
    tol: float = 1e-14


def _chain(p):
    return list(p.kappas) + [p.kappa]


def mp_hamiltonian(lat, U, pi, phis, p):
    ks = _chain(p)
    H = 0.5 * float(np.sum(pi * pi)) + gauge.gauge_action(lat, U, p.beta + hpe.delta_beta(ks[0], p.k))
    H += hpe.filtered_action(lat, U, phis[0], ks[0], p.k, p.n_max, p.tol)
    for i in range(len(p.kappas)):
        H += ratio_action(lat, U, phis[i + 1], ks[i], ks[i + 1], p.tol)
    return H


def mp_forces(lat, phis, p):
    ks = _chain(p)
    beta_eff = p.beta + hpe.delta_beta(ks[0], p.k)
    out = [lambda U: gauge.gauge_force(lat, U, beta_eff),
           lambda U: hpe.filtered_force(lat, U, phis[0], ks[0], p.k, p.n_t, p.tol)]
    for i in range(len(p.kappas)):
        out.append(lambda U, i=i: ratio_force(lat, U, phis[i + 1], ks[i], ks[i + 1], p.tol))
    return out


def mp_heatbath(lat, U, etas, p):
    ks = _chain(p)
    return [hpe.heatbath_phi(lat, U, etas[0], ks[0], p.k, p.n_max)] + \
        [ratio_heatbath(lat, U, etas[i + 1], ks[i], ks[i + 1], p.tol) for i in range(len(p.kappas))]


def mp_integrate(lat, U, pi, phis, p):
    return hmc.integrate_levels(lat, U, pi, mp_forces(lat, phis, p), list(p.msub[:len(p.kappas) + 1]), p.m,
                                p.integrator, p.lam, p.tau)


def mp_trajectory(lat, U0, pi0, etas, u, p):
    phis = mp_heatbath(lat, U0, etas, p)
    H0 = mp_hamiltonian(lat, U0, pi0, phis, p)
    U1, pi1 = mp_integrate(lat, U0, pi0, phis, p)
    H1 = mp_hamiltonian(lat, U1, pi1, phis, p)
    dH = H1 - H0
    acc = bool(u < np.exp(-dH))
    return {"U": U1 if acc else U0, "U_end": U1, "pi_end": pi1, "dH": dH, "accepted": acc, "H0": H0, "H1": H1,
            "phis": phis}
