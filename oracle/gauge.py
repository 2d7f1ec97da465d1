"""Wilson plaquette action, plaquette observable and gauge force (oracle, test only).

Sec. 1: S_G = -(beta/3) sum_x sum_{mu>nu} Re Tr(U_{x,mu} U_{x+mu,nu} U^dag_{x+nu,mu} U^dag_{x,nu}).
Sec. 4.1: plaquette P = (1 / 3 N_p) sum_p Re Tr U_p.
The force follows from (omega, F) = delta_omega S with delta U = omega U (Sec. 1):
F_{x,mu} = (beta/6) P_TA(U_{x,mu} Sigma_{x,mu}), Sigma = sum over the six staples.
The gauge field is periodic in every direction.
"""
import numpy as np

from .su3 import proj_ta, to_coords


def _mm(a, b):
    return np.einsum("...ij,...jk->...ik", a, b)


def _dag(a):
    return np.swapaxes(a.conj(), -1, -2)


def _shift(lat, field, mu, step):
    """field(x + step*mu) with periodic gauge boundaries."""
    return np.roll(field, -step, axis=mu)


def plaquette_field(lat, U, mu, nu):
    Umu, Unu = U[..., mu, :, :], U[..., nu, :, :]
    return _mm(_mm(Umu, _shift(lat, Unu, mu, 1)), _mm(_dag(_shift(lat, Umu, nu, 1)), _dag(Unu)))


def plaquette_sum(lat, U):
    """sum over all plaquettes of Re Tr U_p."""
    s = 0.0
    for mu in range(4):
        for nu in range(mu):
            s += np.trace(plaquette_field(lat, U, mu, nu), axis1=-2, axis2=-1).real.sum()
    return float(s)


def plaquette(lat, U):
    """<P> = sum_p Re Tr U_p / (3 N_p), N_p = 6 V."""
    return plaquette_sum(lat, U) / (3.0 * 6 * lat.V)


def gauge_action(lat, U, beta):
    return -beta / 3.0 * plaquette_sum(lat, U)


def staple_sum(lat, U, mu):
    """sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)]."""
    S = np.zeros(U.shape[:4] + (3, 3), dtype=np.complex128)
    Umu = U[..., mu, :, :]
    for nu in range(4):
        if nu == mu:
            continue
        Unu = U[..., nu, :, :]
        up = _mm(_mm(_shift(lat, Unu, mu, 1), _dag(_shift(lat, Umu, nu, 1))), _dag(Unu))
        Unu_m = _shift(lat, Unu, nu, -1)                       # U_nu(x - nu)
        down = _mm(_mm(_dag(_shift(lat, Unu_m, mu, 1)), _dag(_shift(lat, Umu, nu, -1))), Unu_m)
        S += up + down
    return S


def gauge_force(lat, U, beta):
    """F_G in algebra coordinates, shape (L_t, L_z, L_y, L_x, 4, 8)."""
    F = np.zeros(U.shape[:4] + (4, 8))
    for mu in range(4):
        F[..., mu, :] = to_coords(beta / 6.0 * proj_ta(_mm(U[..., mu, :, :], staple_sum(lat, U, mu))))
    return F
