"""Hopping-parameter-expansion ("kappa^k") filtering, Sec. 2 and 2.2 (oracle, test only).

With K = kappa^2 H_oe H_eo on odd sites (Sec. 2.2: kappa H -> K, and indices count powers of
K), M_oo = 1 - K and the filtered matrix of eq. (tildeM) is
    M~ = M_oo exp( sum_{j<=k} K^j / j ),
so kappa^2-filtering is k = 1 and kappa^4-filtering is k = 2; k = 0 is the plain action.

Coefficients (Sec. 2):
    M~^{-1} = exp(-sum_{j<=k} x^j/j) / (1 - x) = sum_n a_n x^n ,  alpha = exp(-sum_{j<=k} 1/j),
    b_n = a_n - alpha,  so  M~^{-1} = sum_n b_n K^n + alpha M_oo^{-1}.
The action uses the sum up to n_max, the force up to n_t (Sec. 2: truncation).
The heat bath phi = M~ eta (eq. initPseudo applied to M~) needs c_n, the Taylor coefficients
of exp(+sum_{j<=k} x^j/j); the paper's printed truncation values equal these c_n.

Force (Sec. 2, Horner scheme):
    Y_{n_t} = b_{n_t} phi,  Y_{i-1} = b_{i-1} phi + K Y_i,      (the phi is implied in the text)
    Y~ = alpha M_oo^{-1} phi,   X_1 = Y_0 + Y~,   X_i = K^dag X_{i-1},   X~ = M_oo^{-dag} X_1,
    delta S~ = 2 Re[ X~^dag dK Y~ + sum_{i=1}^{n_t} X_i^dag dK Y_i ].
(The adjoints K^dag and M_oo^{-dag} are what the variation of |M~^{-1} phi|^2 produces; the
recursion and X~ are printed without them.)  Each X^dag dK Y term expands into one full-lattice
dH contraction with kappa^2 (see oracle.force).

Gauge part, eq. (ModGauge): S~_G = S_G + 2 sum_{n<=k} (1/n) Tr K^n.  Tr K = (kappa^2/2) Tr H^2
vanishes and Tr K^2 = (kappa^4/2) Tr H^4 = -32 kappa^4 sum_p Re Tr U_p as long as no lattice
extent is 1, 2 or 4 (no winding loops of length 2 or 4), i.e. beta -> beta + 96 kappa^4 for
k = 2 (Sec. 2).
"""
from fractions import Fraction

import mpmath
import numpy as np

from . import dirac
from .force import expand_pair_eo, force_from_pairs, solve_MMdag_oo

mpmath.mp.dps = 50


def exp_series(sign, k, n):
    """Taylor coefficients 0..n of exp(sign * sum_{j<=k} x^j / j), exact rationals.

    g = exp(h) satisfies g' = h' g, i.e. m g_m = sum_{j=1}^{min(m,k)} j h_j g_{m-j}, and here
    j h_j = sign for every j <= k.
    """
    g = [Fraction(1)] + [Fraction(0)] * n
    for m in range(1, n + 1):
        g[m] = Fraction(sign) * sum(g[m - j] for j in range(1, min(m, k) + 1)) / m
    return g


def alpha(k):
    """alpha = exp(-sum_{j<=k} 1/j)  (Sec. 2)."""
    return mpmath.exp(-mpmath.fsum(mpmath.mpf(1) / j for j in range(1, k + 1)))


def coefficients(k, n):
    """(a_n, b_n, c_n) as 50-digit mpmath numbers for orders 0..n, and alpha."""
    e = exp_series(-1, k, n)
    a, acc = [], Fraction(0)
    for m in range(n + 1):
        acc += e[m]
        a.append(acc)
    al = alpha(k)
    to_mp = lambda q: mpmath.mpf(q.numerator) / q.denominator
    b = [to_mp(x) - al for x in a]
    c = [to_mp(x) for x in exp_series(+1, k, n)]
    return [to_mp(x) for x in a], b, c, al


def coefficients_f64(k, n):
    _, b, c, al = coefficients(k, n)
    return np.array([float(x) for x in b]), np.array([float(x) for x in c]), float(al)


def delta_beta(kappa, k):
    """beta shift from eq. (ModGauge): 0 for k <= 1, 96 kappa^4 for k = 2 (Sec. 2)."""
    if k <= 1:
        return 0.0
    if k == 2:
        return 96.0 * kappa ** 4
    raise ValueError("only k <= 2 is tractable in closed form (Sec. 2)")


# ---------------------------------------------------------------- action, heat bath, force

def _minv(lat, U, phi_o, kappa, tol):
    """M_oo^{-1} phi = M_oo^dag (M_oo M_oo^dag)^{-1} phi."""
    return dirac.apply_Moo_dag(lat, U, solve_MMdag_oo(lat, U, phi_o, kappa, tol), kappa)


def _minv_dag(lat, U, v, kappa, tol):
    """M_oo^{-dag} v = M_oo (M_oo^dag M_oo)^{-1} v."""
    from .solve import cg
    A = lambda w: dirac.apply_MooDagMoo(lat, U, w, kappa)
    s, _, _ = cg(A, v, tol=tol)
    return dirac.apply_Moo(lat, U, s, kappa)


def _next_X(lat, U, x, kappa):
    """X_i = K^dag X_{i-1}."""
    return dirac.apply_Kdag(lat, U, x, kappa)


def poly_K(lat, U, coef, v, kappa):
    """sum_n coef[n] K^n v by Horner's scheme."""
    acc = coef[-1] * v
    for cn in coef[-2::-1]:
        acc = cn * v + dirac.apply_K(lat, U, acc, kappa)
    return acc


def filtered_inverse(lat, U, phi_o, kappa, k, n_max, tol=1e-13):
    """M~^{-1} phi = sum_{n<=n_max} b_n K^n phi + alpha M_oo^{-1} phi."""
    b, _, al = coefficients_f64(k, n_max)
    return poly_K(lat, U, b, phi_o, kappa) + al * _minv(lat, U, phi_o, kappa, tol)


def filtered_action(lat, U, phi_o, kappa, k, n_max, tol=1e-13):
    """S~_PF = |M~^{-1} phi|^2, eq. (ModPF)."""
    z = filtered_inverse(lat, U, phi_o, kappa, k, n_max, tol)
    return float(np.vdot(z.reshape(-1), z.reshape(-1)).real)


def heatbath_phi(lat, U, eta_o, kappa, k, n_max):
    """phi = M~ eta = M_oo sum_{n<=n_max} c_n K^n eta, eq. (initPseudo) for M~."""
    _, c, _ = coefficients_f64(k, n_max)
    return dirac.apply_Moo(lat, U, poly_K(lat, U, c, eta_o, kappa), kappa)


def filtered_force(lat, U, phi_o, kappa, k, n_t, tol=1e-13):
    """F~ in algebra coordinates, following the Horner recursion of Sec. 2 step by step."""
    b, _, al = coefficients_f64(k, n_t)
    Ys = [None] * (n_t + 1)
    Ys[n_t] = b[n_t] * phi_o
    for i in range(n_t, 0, -1):
        Ys[i - 1] = b[i - 1] * phi_o + dirac.apply_K(lat, U, Ys[i], kappa)
    Y_tilde = al * _minv(lat, U, phi_o, kappa, tol)
    Xs = [None] * (n_t + 1)
    if n_t >= 1:
        Xs[1] = Ys[0] + Y_tilde
        for i in range(2, n_t + 1):
            Xs[i] = _next_X(lat, U, Xs[i - 1], kappa)
    X1 = Ys[0] + Y_tilde
    X_tilde = _minv_dag(lat, U, X1, kappa, tol)
    pairs = [expand_pair_eo(lat, U, X_tilde, Y_tilde)]
    pairs += [expand_pair_eo(lat, U, Xs[i], Ys[i]) for i in range(1, n_t + 1)]
    return force_from_pairs(lat, U, pairs, kappa ** 2)


# ---------------------------------------------------------------- traces of powers of H

def polyakov_re_tr(lat, U, mu, sign):
    """sum_x sign * Re Tr of the straight loop of L_mu links along mu starting at x."""
    P = U[..., mu, :, :].copy()
    for step in range(1, lat.dims[mu]):
        P = np.einsum("...ab,...bc->...ac", P, np.roll(U[..., mu, :, :], -step, axis=mu))
    return sign * float(np.trace(P, axis1=-2, axis2=-1).real.sum())
