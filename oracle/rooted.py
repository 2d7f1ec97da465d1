"""Rooted polynomials as UV filters, Sec. 2.1 (oracle, test only).

Powers count K = kappa^2 H_oe H_eo on odd sites (Sec. 2.2), x stands for K, M_oo = 1 - x.
Reading of the recursion: the runs of Sec. 4.2 name n_1, n_2 and N_1 = N_2 = N for j_max = 2,
so the polynomials are W_1, W_2 and the chain starts at M_1 = M~ of eq. (tildeM) (M_oo for no
hopping-parameter expansion, k = 0).  This reading reproduces the alpha column of Table RunPoly1
and the alpha of Sec. 4.2.2.
    p_j(x) = W_j^{-1} = the Taylor polynomial of degree n_j of M_j(x)^{-1/N},
    M_{j+1} = W_j^{-N} M_j = p_j^N M_j                  (j = 1 .. j_max),
    M_{j_max+1}^{-1} = g(x) / (1 - x),   g(x) = exp(-sum_{i<=k} x^i/i) prod_j p_j(x)^{-N},
                     = sum_n b_n x^n + alpha M_oo^{-1}      (eq. restM)
    alpha = g(1) = exp(-sum_{i<=k} 1/i) prod_j p_j(1)^{-N},   b_n = sum_{m<=n} g_m - alpha.
All Taylor coefficients are rational (roots and exponentials of series with rational
coefficients), so p_j and g_m are computed exactly with Fractions; alpha with mpmath.

Since det M~ = prod_j (det W_j)^N det M_{j_max+1}, two flavours are represented by
    S = sum_j sum_{i=1}^{N} |p_j(K) phi_{j,i}|^2 + |M_{j_max+1}^{-1} phi_r|^2
(plus the gauge term of M~, Sec. 2), with the heat baths (eq. initPseudo)
    phi_{j,i} = W_j eta = p_j(K)^{-1} eta   (a solve with the polynomial operator),
    phi_r = M_{j_max+1} eta = prod_j p_j(K)^N M~ eta.
The force of |(sum_n c_n K^n + a M_oo^{-1}) phi|^2 is the Horner construction of Sec. 2 for any
coefficients c_n and a; with a = 0 (the polynomial fields) it has no inverse and no (X~, Y~) pair.

HMC (Sec. 4.2): the runs use several time scales with step counts m_0, m_1, m_2 and m.  Reading:
the gauge action sits on level 0, the term of p_j on level j and the remainder on level
j_max + 1 (forces ordered from the largest, cheapest to the smallest, most expensive); one step
of level l holds m_{l-1} steps of level l - 1, and the remainder takes m steps per trajectory.
"""
from dataclasses import dataclass
from fractions import Fraction

import mpmath
import numpy as np

from . import dirac, gauge, hmc, hpe
from .force import expand_pair_eo, force_from_pairs
from .solve import cg

mpmath.mp.dps = 50


# ---------------------------------------------------------------- power series (exact)

def _exp(a, n):
    """Taylor coefficients 0..n of exp(a(x)) for a series a with a[0] = 0: E' = a' E."""
    E = [Fraction(0)] * (n + 1)
    E[0] = Fraction(1)
    for m in range(1, n + 1):
        E[m] = sum(i * a[i] * E[m - i] for i in range(1, m + 1)) / m
    return E


def _log(p, n):
    """Taylor coefficients 0..n of log p(x) for a polynomial p with p[0] = 1: L' = p' / p."""
    inv = [Fraction(0)] * (n + 1)
    inv[0] = Fraction(1)
    for m in range(1, n + 1):
        inv[m] = -sum(p[i] * inv[m - i] for i in range(1, min(m, len(p) - 1) + 1))
    L = [Fraction(0)] * (n + 1)
    for m in range(1, n + 1):
        L[m] = sum(i * p[i] * inv[m - i] for i in range(1, min(m, len(p) - 1) + 1)) / m
    return L


def polynomials(N, ns, k):
    """[p_1, p_2, ...] as exact coefficient lists of degrees ns."""
    n = max(ns, default=0)
    logM = [Fraction(0)] + [Fraction(-1, i) for i in range(1, n + 1)]   # log(1 - x)
    for i in range(1, min(k, n) + 1):
        logM[i] += Fraction(1, i)                                          # + sum_{i<=k} x^i / i
    out = []
    for nj in ns:
        pj = _exp([-c / N for c in logM[: nj + 1]], nj)                    # M_j^{-1/N} to degree n_j
        out.append(pj)
        Lp = _log(pj, n)
        logM = [logM[i] + N * Lp[i] for i in range(n + 1)]                 # M_{j+1} = p_j^N M_j
    return out


def alpha(N, ns, k):
    """alpha of eq. (restM) = exp(-sum_{i<=k} 1/i) prod_j p_j(1)^{-N}."""
    a = mpmath.exp(-mpmath.fsum(mpmath.mpf(1) / i for i in range(1, k + 1)))
    for pj in polynomials(N, ns, k):
        s = sum(pj)
        a /= (mpmath.mpf(s.numerator) / s.denominator) ** N
    return a


def remainder_b(N, ns, k, n_max):
    """b_0 .. b_{n_max} of eq. (restM): b_n = sum_{m<=n} g_m - alpha."""
    ps = polynomials(N, ns, k)
    lg = [Fraction(0)] * (n_max + 1)
    for i in range(1, min(k, n_max) + 1):
        lg[i] -= Fraction(1, i)
    for pj in ps:
        Lp = _log(pj, n_max)
        lg = [lg[i] - N * Lp[i] for i in range(n_max + 1)]
    g = _exp(lg, n_max)
    a = alpha(N, ns, k)
    out, s = [], Fraction(0)
    for m in range(n_max + 1):
        s += g[m]
        out.append(mpmath.mpf(s.numerator) / s.denominator - a)
    return out


def coefficients_f64(N, ns, k, n_max):
    """(list of p_j as float arrays, b as float array, alpha float)."""
    ps = [np.array([float(c) for c in p]) for p in polynomials(N, ns, k)]
    return ps, np.array([float(v) for v in remainder_b(N, ns, k, n_max)]), float(alpha(N, ns, k))


# ---------------------------------------------------------------- actions, heat baths, forces

def poly_apply(lat, U, coef, v, kappa, dagger=False):
    """sum_n coef[n] K^n v (K^dag for dagger), Horner."""
    out = coef[-1] * v
    for c in coef[-2::-1]:
        out = c * v + (dirac.apply_Kdag(lat, U, out, kappa) if dagger else dirac.apply_K(lat, U, out, kappa))
    return out


def poly_action(lat, U, phi, coef, kappa):
    """|p(K) phi|^2."""
    z = poly_apply(lat, U, coef, phi, kappa)
    return float(np.vdot(z, z).real)


def poly_heatbath(lat, U, eta, coef, kappa, tol=1e-14):
    """phi = p(K)^{-1} eta by CG on p^dag p phi = p^dag eta."""
    A = lambda v: poly_apply(lat, U, coef, poly_apply(lat, U, coef, v, kappa), kappa, dagger=True)
    phi, _, _ = cg(A, poly_apply(lat, U, coef, eta, kappa, dagger=True), tol=tol)
    return phi


def remainder_inverse(lat, U, phi, b, al, kappa, tol=1e-14):
    """(sum_n b_n K^n + alpha M_oo^{-1}) phi."""
    return poly_apply(lat, U, b, phi, kappa) + al * hpe._minv(lat, U, phi, kappa, tol)


def remainder_action(lat, U, phi, b, al, kappa, tol=1e-14):
    z = remainder_inverse(lat, U, phi, b, al, kappa, tol)
    return float(np.vdot(z, z).real)


def remainder_heatbath(lat, U, eta, ps, N, kappa, k, n_max):
    """phi_r = prod_j p_j(K)^N M~ eta (M~ eta truncated at n_max as in hpe.heatbath_phi)."""
    v = hpe.heatbath_phi(lat, U, eta, kappa, k, n_max)
    for p in ps:
        for _ in range(N):
            v = poly_apply(lat, U, p, v, kappa)
    return v


def series_force(lat, U, phi, c, a, kappa, tol=1e-14):
    """force of |(sum_{n<=len(c)-1} c_n K^n + a M_oo^{-1}) phi|^2 by the Horner scheme of Sec. 2:
    Y_n = c_n phi, Y_{i-1} = c_{i-1} phi + K Y_i; Y~ = a M_oo^{-1} phi; X_1 = Y_0 + Y~,
    X_i = K^dag X_{i-1}; X~ = M_oo^{-dag} X_1; pairs (X~, Y~) (only for a != 0), (X_i, Y_i)."""
    n = len(c) - 1
    Ys = [None] * (n + 1)
    Ys[n] = c[n] * phi
    for i in range(n, 0, -1):
        Ys[i - 1] = c[i - 1] * phi + dirac.apply_K(lat, U, Ys[i], kappa)
    X1 = Ys[0].copy()
    pairs = []
    if a != 0.0:
        Yt = a * hpe._minv(lat, U, phi, kappa, tol)
        X1 = X1 + Yt
        pairs.append(expand_pair_eo(lat, U, hpe._minv_dag(lat, U, X1, kappa, tol), Yt))
    X = X1
    for i in range(1, n + 1):
        if i > 1:
            X = hpe._next_X(lat, U, X, kappa)
        pairs.append(expand_pair_eo(lat, U, X, Ys[i]))
    return force_from_pairs(lat, U, pairs, kappa ** 2)


# ---------------------------------------------------------------- HMC with the rooted action

@dataclass
class RootedHMCParams:
    beta: float = 5.6
    kappa: float = 0.1575
    N: int = 2
    ns: tuple = (4, 8)          # degrees n_1 .. n_jmax
    k: int = 0                  # filter of M_1 = M~
    n_t: int = 20               # remainder truncation in the force
    n_max: int = 40             # remainder truncation in action and heat bath
    integrator: str = "leapfrog"
    lam: float = 1.0 / 6.0
    m: int = 4                  # remainder steps per trajectory
    msub: tuple = (2, 2, 2)     # m_0, m_1, ..., m_jmax
    tau: float = 1.0
    tol: float = 1e-13


def rooted_hamiltonian(lat, U, pi, phis, p):
    """(1/2)(Pi,Pi) + S_G + sum_j sum_i |p_j(K) phi_{j,i}|^2 + |remainder phi_r|^2 (at n_max)."""
    ps, b, al = coefficients_f64(p.N, p.ns, p.k, p.n_max)
    H = 0.5 * float(np.sum(pi * pi)) + gauge.gauge_action(lat, U, p.beta + hpe.delta_beta(p.kappa, p.k))
    for j, pj in enumerate(ps):
        for i in range(p.N):
            H += poly_action(lat, U, phis[j * p.N + i], pj, p.kappa)
    return H + remainder_action(lat, U, phis[-1], b, al, p.kappa, p.tol)


def rooted_forces(lat, phis, p):
    """forces of the levels: gauge, the polynomial terms, the remainder (at n_t)."""
    ps, b, al = coefficients_f64(p.N, p.ns, p.k, p.n_t)
    beta_eff = p.beta + hpe.delta_beta(p.kappa, p.k)
    out = [lambda U: gauge.gauge_force(lat, U, beta_eff)]
    for j, pj in enumerate(ps):
        out.append(lambda U, j=j, pj=pj: sum(series_force(lat, U, phis[j * p.N + i], pj, 0.0, p.kappa, p.tol)
                                             for i in range(p.N)))
    out.append(lambda U: series_force(lat, U, phis[-1], b, al, p.kappa, p.tol))
    return out


def rooted_integrate(lat, U, pi, phis, p):
    return hmc.integrate_levels(lat, U, pi, rooted_forces(lat, phis, p), list(p.msub[:len(p.ns) + 1]), p.m,
                                p.integrator, p.lam, p.tau)


def rooted_heatbath(lat, U, etas, p):
    ps, _, _ = coefficients_f64(p.N, p.ns, p.k, 0)
    phis = [poly_heatbath(lat, U, etas[j * p.N + i], ps[j], p.kappa, p.tol)
            for j in range(len(ps)) for i in range(p.N)]
    return phis + [remainder_heatbath(lat, U, etas[-1], ps, p.N, p.kappa, p.k, p.n_max)]


def rooted_trajectory(lat, U0, pi0, etas, u, p):
    """heat bath of all jmax*N + 1 fields, H0, multi-level MD, H1, Metropolis."""
    phis = rooted_heatbath(lat, U0, etas, p)
    H0 = rooted_hamiltonian(lat, U0, pi0, phis, p)
    U1, pi1 = rooted_integrate(lat, U0, pi0, phis, p)
    H1 = rooted_hamiltonian(lat, U1, pi1, phis, p)
    dH = H1 - H0
    acc = bool(u < np.exp(-dH))
    return {"U": U1 if acc else U0, "U_end": U1, "pi_end": pi1, "dH": dH, "accepted": acc, "H0": H0, "H1": H1,
            "phis": phis}
