"""SU(3) algebra helpers for the oracle (test infrastructure only).

Momenta are antihermitian traceless (Sec. 1); with T_a = i lambda_a / 2 (Gell-Mann lambda_a)
Pi = sum_a pi_a T_a and the scalar product of eq. (Sproduct), (Pi,Pi) = -2 sum Tr Pi^2,
becomes sum_a pi_a^2.  Forces use the same coordinates: (omega, F) = sum_a omega_a f_a.
"""
import numpy as np

LAMBDA = np.zeros((8, 3, 3), dtype=np.complex128)
LAMBDA[0][0, 1] = LAMBDA[0][1, 0] = 1
LAMBDA[1][0, 1] = -1j
LAMBDA[1][1, 0] = 1j
LAMBDA[2][0, 0], LAMBDA[2][1, 1] = 1, -1
LAMBDA[3][0, 2] = LAMBDA[3][2, 0] = 1
LAMBDA[4][0, 2] = -1j
LAMBDA[4][2, 0] = 1j
LAMBDA[5][1, 2] = LAMBDA[5][2, 1] = 1
LAMBDA[6][1, 2] = -1j
LAMBDA[6][2, 1] = 1j
LAMBDA[7][0, 0] = LAMBDA[7][1, 1] = 1 / np.sqrt(3)
LAMBDA[7][2, 2] = -2 / np.sqrt(3)

T = 0.5j * LAMBDA          # antihermitian generators, Tr(T_a T_b) = -delta_ab / 2


def from_coords(c):
    """algebra coordinates (..., 8) -> antihermitian traceless matrices (..., 3, 3)."""
    return np.einsum("...a,aij->...ij", c, T)


def to_coords(A):
    """antihermitian traceless (..., 3, 3) -> coordinates a_a = -2 Tr(T_a A)."""
    return (-2.0 * np.einsum("aij,...ji->...a", T, A)).real


def proj_ta(A):
    """antihermitian traceless part: (A - A^dag)/2 - Tr(A - A^dag)/6."""
    B = 0.5 * (A - np.swapaxes(A.conj(), -1, -2))
    tr = np.trace(B, axis1=-2, axis2=-1)
    return B - tr[..., None, None] / 3.0 * np.eye(3)


def expm_ah(A):
    """exp(A) for antihermitian A via the eigen-decomposition of the hermitian iA."""
    w, Q = np.linalg.eigh(1j * A)
    return np.einsum("...ik,...k,...jk->...ij", Q, np.exp(-1j * w), Q.conj())
