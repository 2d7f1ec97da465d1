"""HMC trajectory with Sexton-Weingarten levels (oracle, test only).

Sec. 1: H = (1/2)(Pi,Pi) + S(U, phi); the trajectory is heat bath, molecular dynamics, then
Metropolis with P_acc = min[1, exp(-Delta H)].  Equations of motion dPi/dtau = -F,
dU/dtau = Pi U.  The printed update steps carry an extra i and a + sign that contradict these
equations for antihermitian Pi; we read them as
    P(eps): Pi -> Pi - eps F ,      T(eps): U -> exp(eps Pi) U .
Omelyan (eq. Omel): P(l e) T(e/2) P((1-2l) e) T(e/2) P(l e), leapfrog is l = 1/2 collapsed to
P(e/2) T(e) P(e/2).  Levels (Sec. 1): level i step e_i = 2 m_{i-1} e_{i-1} (Omelyan) or
m_{i-1} e_{i-1} (leapfrog), and
    T_i = P_i(l e_i) [T_{i-1}]^{m_{i-1}} P_i((1-2l) e_i) [T_{i-1}]^{m_{i-1}} P_i(l e_i).
Sec. 4.1 puts the gauge action on the fine level 0 and the pseudo-fermion action on level 1.
No steps are merged: every P of the scheme is executed as written.

The random numbers (momenta pi, pseudo-fermion source eta, Metropolis u) are inputs.
"""
from dataclasses import dataclass

import numpy as np

from . import gauge, hpe
from .su3 import expm_ah, from_coords


@dataclass
class HMCParams:
    beta: float = 5.6
    kappa: float = 0.156
    k: int = 0                 # filter order: 0 none, 1 kappa^2, 2 kappa^4
    n_t: int = 0               # truncation in the force
    n_max: int = 0             # truncation in the action / heat bath
    integrator: str = "omelyan"  # or "leapfrog"
    lam: float = 1.0 / 6.0
    m: int = 10                # coarse (pseudo-fermion) steps per trajectory
    m0: int = 4                # gauge steps per coarse half-step (Omelyan) / step (leapfrog)
    tau: float = 1.0
    tol: float = 1e-13


def hamiltonian(lat, U, pi, phi_o, p):
    beta_eff = p.beta + hpe.delta_beta(p.kappa, p.k)
    return (0.5 * float(np.sum(pi * pi)) + gauge.gauge_action(lat, U, beta_eff)
            + hpe.filtered_action(lat, U, phi_o, p.kappa, p.k, p.n_max, p.tol))


def _level_forces(lat, phi_o, p):
    beta_eff = p.beta + hpe.delta_beta(p.kappa, p.k)
    return [
        lambda U: gauge.gauge_force(lat, U, beta_eff),
        lambda U: hpe.filtered_force(lat, U, phi_o, p.kappa, p.k, p.n_t, p.tol),
    ]


def integrate_levels(lat, U, pi, forces, nsub, m, integrator, lam, tau):
    """molecular dynamics over tau with levels 0..L: forces[l](U) is the force of level l, one
    (half, for Omelyan) step of level l >= 1 holds nsub[l-1] steps of level l-1, and level L
    takes m steps.  Returns (U', pi')."""
    state = {"U": U.copy(), "pi": pi.copy()}

    def P(level, eps):
        state["pi"] = state["pi"] - eps * forces[level](state["U"])

    def T(eps):
        state["U"] = np.einsum("...ab,...bc->...ac", expm_ah(eps * from_coords(state["pi"])), state["U"])

    omel = integrator == "omelyan"
    lam = lam if omel else 0.5

    def run(level, eps):
        if omel:
            P(level, lam * eps)
            sub(level, eps / 2)
            P(level, (1 - 2 * lam) * eps)
            sub(level, eps / 2)
            P(level, lam * eps)
        else:
            P(level, eps / 2)
            sub(level, eps)
            P(level, eps / 2)

    def sub(level, span):
        """the inner part between two P_level steps, covering MD time `span`."""
        if level == 0:
            T(span)
        else:
            n = nsub[level - 1]
            for _ in range(n):
                run(level - 1, span / n)

    top = len(forces) - 1
    for _ in range(m):
        run(top, tau / m)
    return state["U"], state["pi"]


def integrate(lat, U, pi, phi_o, p):
    """molecular dynamics over tau (gauge on level 0, m0 steps per level-1 block; pseudo-fermion
    on level 1, m steps); returns (U', pi')."""
    return integrate_levels(lat, U, pi, _level_forces(lat, phi_o, p), [p.m0], p.m, p.integrator, p.lam, p.tau)


def trajectory(lat, U0, pi0, eta_o, u, p):
    """one HMC trajectory; returns dict with U (new field), dH, accepted, H0, H1, phi."""
    phi_o = hpe.heatbath_phi(lat, U0, eta_o, p.kappa, p.k, p.n_max)
    H0 = hamiltonian(lat, U0, pi0, phi_o, p)
    U1, pi1 = integrate(lat, U0, pi0, phi_o, p)
    H1 = hamiltonian(lat, U1, pi1, phi_o, p)
    dH = H1 - H0
    acc = bool(u < np.exp(-dH))
    return {"U": U1 if acc else U0, "U_end": U1, "pi_end": pi1, "dH": dH, "accepted": acc,
            "H0": H0, "H1": H1, "phi": phi_o}


def reversibility(lat, U0, pi0, phi_o, p):
    """Delta of eq. (reverse): integrate, flip the momenta, integrate back."""
    U1, pi1 = integrate(lat, U0, pi0, phi_o, p)
    U2, _ = integrate(lat, U1, -pi1, phi_o, p)
    return float(np.sum(np.abs(U0 - U2) ** 2))
