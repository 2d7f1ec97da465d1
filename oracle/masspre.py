"""Mass preconditioning combined with kappa^(2k) filtering (oracle, test only).

Sec. 1 splits the fermion matrix into factors, each with its own pseudo-fermion field and its own
time scale; the conclusion (Sec. 5) proposes combining the filter with mass preconditioning and
remarks that the term of the heaviest mass might then be dropped.  Reading: every factor carries
the filter of Sec. 2, M~(kappa) = M_oo(kappa) exp(sum_{j<=k} K(kappa)^j / j), and one gauge term
remains, that of the target kappa:
    det M_oo(kappa) = det M~(kappa_1) prod_{i=1..n} det M~(kappa_{i+1}) / det M~(kappa_i)
                      * exp(-sum_{j<=k} Tr K(kappa)^j / j),        kappa_1 < ... < kappa_{n+1} = kappa,
so the gauge action is taken at beta + 96 kappa^4 (k = 2), the heaviest field has the action
|M~(kappa_1)^{-1} phi_1|^2, and each ratio
    S_i = |M~(kappa_{i+1})^{-1} M~(kappa_i) phi|^2,   heat bath phi = M~(kappa_i)^{-1} M~(kappa_{i+1}) eta.
Only with the filter on the ratios as well do their low orders in K cancel (up to x^(k+1)), so that
their forces are small; det M~(kappa_1) then tends to 1 for a heavy kappa_1, the paper's remark.

Series form of a ratio.  M_oo(kappa) = 1 - kappa^2 D with D = H_oe H_eo for every kappa, so with
x = K(kappa_{i+1}) and rho = kappa_i^2 / kappa_{i+1}^2 (K(kappa_i) = rho x) all factors commute and
    M~(kappa_{i+1})^{-1} M~(kappa_i) = g(x) / (1 - x),  g(x) = (1 - rho x) exp(sum_{j<=k} (rho^j - 1) x^j / j),
              = sum_n b_n x^n + alpha M_oo(kappa_{i+1})^{-1},  alpha = g(1),  b_n = sum_{m<=n} g_m - alpha,
the construction of eq. (restM).  Action (at n_max) and force (at n_t) use this series, so that
the force is the exact derivative of the action for n_t = n_max; `ratio_action` computes the
action from the definition instead, and the tests compare both forms.

HMC levels (reading): gauge action on level 0, the filtered heavy field on level 1, the ratios on
levels 2 .. n + 1 from the heaviest to the lightest.
"""
from dataclasses import dataclass

import mpmath
import numpy as np

from . import dirac, gauge, hmc, hpe
from .force import solve_MMdag_oo
from .rooted import remainder_action, series_force


def moo_inverse(lat, U, v, kappa, tol):
    """M_oo(kappa)^{-1} v = M_oo^dag (M_oo M_oo^dag)^{-1} v."""
    return dirac.apply_Moo_dag(lat, U, solve_MMdag_oo(lat, U, v, kappa, tol), kappa)


def ratio_coefficients(rho, k, n):
    """(b_0 .. b_n, alpha) of g(x) / (1 - x), g = (1 - rho x) exp(sum_{j<=k} (rho^j - 1) x^j / j)."""
    r = mpmath.mpf(rho)
    a = [mpmath.mpf(0)] * (n + 1)
    for j in range(1, min(k, n) + 1):
        a[j] = (r ** j - 1) / j
    E = [mpmath.mpf(1)] + [mpmath.mpf(0)] * n          # exp(a): E' = a' E
    for m in range(1, n + 1):
        E[m] = mpmath.fsum(i * a[i] * E[m - i] for i in range(1, m + 1)) / m
    g = [E[m] - (r * E[m - 1] if m >= 1 else 0) for m in range(n + 1)]
    alpha = (1 - r) * mpmath.exp(mpmath.fsum((r ** j - 1) / j for j in range(1, k + 1)))
    b, s = [], mpmath.mpf(0)
    for m in range(n + 1):
        s += g[m]
        b.append(float(s - alpha))
    return b, float(alpha)


def ratio_action(lat, U, phi, k_lo, k_hi, k, n_max, tol=1e-14):
    """|M~(k_hi)^{-1} M~(k_lo) phi|^2 from the definition (series of M~ and M~^{-1} at n_max)."""
    v = hpe.heatbath_phi(lat, U, phi, k_lo, k, n_max)            # M~(k_lo) phi
    z = hpe.filtered_inverse(lat, U, v, k_hi, k, n_max, tol)     # M~(k_hi)^{-1} v
    return float(np.vdot(z, z).real)


def ratio_action_series(lat, U, phi, k_lo, k_hi, k, n, tol=1e-14):
    """the ratio action through its series form truncated at n (the action of the Hamiltonian, so
    that the force at n_t = n_max is its exact derivative)."""
    b, al = ratio_coefficients((k_lo / k_hi) ** 2, k, n)
    return remainder_action(lat, U, phi, b, al, k_hi, tol)


def ratio_heatbath(lat, U, eta, k_lo, k_hi, k, n_max, tol=1e-14):
    """phi = M~(k_lo)^{-1} M~(k_hi) eta."""
    return hpe.filtered_inverse(lat, U, hpe.heatbath_phi(lat, U, eta, k_hi, k, n_max), k_lo, k, n_max, tol)


def ratio_force(lat, U, phi, k_lo, k_hi, k, n_t, tol=1e-14):
    """force of the ratio action through its series form truncated at n_t."""
    b, al = ratio_coefficients((k_lo / k_hi) ** 2, k, n_t)
    return series_force(lat, U, phi, b, al, k_hi, tol)


@dataclass
class MassPreParams:
    beta: float = 5.6
    kappa: float = 0.156
    kappas: tuple = (0.14,)     # kappa_1 < ... < kappa_n < kappa
    k: int = 2                  # filter order of every factor
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
    H = 0.5 * float(np.sum(pi * pi)) + gauge.gauge_action(lat, U, p.beta + hpe.delta_beta(p.kappa, p.k))
    H += hpe.filtered_action(lat, U, phis[0], ks[0], p.k, p.n_max, p.tol)
    for i in range(len(p.kappas)):
        H += ratio_action_series(lat, U, phis[i + 1], ks[i], ks[i + 1], p.k, p.n_max, p.tol)
    return H


def mp_forces(lat, phis, p):
    ks = _chain(p)
    beta_eff = p.beta + hpe.delta_beta(p.kappa, p.k)
    out = [lambda U: gauge.gauge_force(lat, U, beta_eff),
           lambda U: hpe.filtered_force(lat, U, phis[0], ks[0], p.k, p.n_t, p.tol)]
    for i in range(len(p.kappas)):
        out.append(lambda U, i=i: ratio_force(lat, U, phis[i + 1], ks[i], ks[i + 1], p.k, p.n_t, p.tol))
    return out


def mp_heatbath(lat, U, etas, p):
    ks = _chain(p)
    return [hpe.heatbath_phi(lat, U, etas[0], ks[0], p.k, p.n_max)] + \
        [ratio_heatbath(lat, U, etas[i + 1], ks[i], ks[i + 1], p.k, p.n_max, p.tol) for i in range(len(p.kappas))]


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
