"""Pseudo-fermion action and force (oracle, test only).

Sec. 1, eq. (WePe_action): S_PF = |M^{-1} phi|^2.
Sec. 2: delta S_PF = -X^dag delta M Y + h.c. with X = (M M^dag)^{-1} phi, Y = M^{-1} phi.

With M = 1 - kappa H and delta U_{x,mu} = omega_{x,mu} U_{x,mu}, writing the variation of the
two H entries that contain U_{x,mu} and reading off (omega, F) = delta_omega S gives, link by
link,
    F_{x,mu} = -kappa P_TA( U_{x,mu} Q_{x,mu} - R_{x,mu} U^dag_{x,mu} )
    Q_{ca} = sum_s [(1 - gamma_mu) Y(x+mu)]_{s c} conj(X(x)_{s a})
    R_{ca} = sum_s [(1 + gamma_mu) Y(x)]_{s c} conj(X(x+mu)_{s a})
where the shifted fields carry the anti-periodic time sign.  For the even/odd matrix of
Sec. 2.2, delta M_oo = -kappa^2 (delta H_oe H_eo + H_oe delta H_eo), so the same contraction
applies with kappa -> kappa^2 to the full-lattice pair X = (H_oe^dag X_o, X_o),
Y = (H_eo Y_o, Y_o).
"""
import numpy as np

from . import dirac
from .gamma import P_MINUS, P_PLUS
from .solve import cg
from .su3 import proj_ta, to_coords


def link_derivative(lat, U, X, Y):
    """G_{x,mu} = U Q - R U^dag for full-lattice spinors X, Y; shape (dims, 4, 3, 3)."""
    G = np.zeros(U.shape, dtype=np.complex128)
    Xc = X.conj()
    for mu in range(4):
        Umu = U[..., mu, :, :]
        Q = np.einsum("...sc,...sa->...ca", dirac.spin_mul(P_MINUS[mu], lat.fwd(Y, mu)), Xc)
        R = np.einsum("...sc,...sa->...ca", dirac.spin_mul(P_PLUS[mu], Y), lat.fwd(X, mu).conj())
        G[..., mu, :, :] = np.einsum("...ab,...bc->...ac", Umu, Q) - np.einsum(
            "...ab,...cb->...ac", R, Umu.conj())
    return G


def force_from_pairs(lat, U, pairs, kappa_eff):
    """F = -kappa_eff sum_pairs P_TA(G(X, Y)) in algebra coordinates, shape (dims, 4, 8)."""
    G = np.zeros(U.shape, dtype=np.complex128)
    for X, Y in pairs:
        G += link_derivative(lat, U, X, Y)
    return to_coords(-kappa_eff * proj_ta(G))


def expand_pair_eo(lat, U, X_o, Y_o):
    """odd-site pair -> full-lattice pair (H_oe^dag X_o, X_o), (H_eo Y_o, Y_o)."""
    X_e = dirac.apply_Hblock(lat, U, X_o, 0, dagger=True)
    Y_e = dirac.apply_Hblock(lat, U, Y_o, 0)
    return lat.to_full(X_e, 0) + lat.to_full(X_o, 1), lat.to_full(Y_e, 0) + lat.to_full(Y_o, 1)


# ---------------------------------------------------------------- full lattice

def pf_action_full(lat, U, phi, kappa, tol=1e-13):
    MMd = lambda v: dirac.apply_M(lat, U, dirac.apply_Mdag(lat, U, v, kappa), kappa)
    X, _, _ = cg(MMd, phi, tol=tol)
    Y = dirac.apply_Mdag(lat, U, X, kappa)
    return float(np.vdot(Y.reshape(-1), Y.reshape(-1)).real)


def pf_force_full(lat, U, phi, kappa, tol=1e-13):
    MMd = lambda v: dirac.apply_M(lat, U, dirac.apply_Mdag(lat, U, v, kappa), kappa)
    X, _, _ = cg(MMd, phi, tol=tol)
    Y = dirac.apply_Mdag(lat, U, X, kappa)
    return force_from_pairs(lat, U, [(X, Y)], kappa)


# ---------------------------------------------------------------- even / odd

def solve_MMdag_oo(lat, U, phi_o, kappa, tol=1e-13):
    """X_o = (M_oo M_oo^dag)^{-1} phi_o."""
    A = lambda v: dirac.apply_Moo(lat, U, dirac.apply_Moo_dag(lat, U, v, kappa), kappa)
    X, _, _ = cg(A, phi_o, tol=tol)
    return X


def pf_action_eo(lat, U, phi_o, kappa, tol=1e-13):
    Y = dirac.apply_Moo_dag(lat, U, solve_MMdag_oo(lat, U, phi_o, kappa, tol), kappa)
    return float(np.vdot(Y.reshape(-1), Y.reshape(-1)).real)


def pf_force_eo(lat, U, phi_o, kappa, tol=1e-13):
    X_o = solve_MMdag_oo(lat, U, phi_o, kappa, tol)
    Y_o = dirac.apply_Moo_dag(lat, U, X_o, kappa)
    return force_from_pairs(lat, U, [expand_pair_eo(lat, U, X_o, Y_o)], kappa ** 2)
