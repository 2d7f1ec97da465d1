"""Dirac matrices for the oracle (test infrastructure only).

The paper writes H with (1 -/+ gamma_mu) but never fixes a basis (Sec. 1, definition of H).
We take the Euclidean chiral basis, hermitian, {gamma_mu, gamma_nu} = 2 delta_mu_nu:

    gamma_0 = [[0, 1], [1, 0]],   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   (k = 1, 2, 3)

in 2x2 spin blocks, gamma_mu acting along array axis mu (mu = 0 is time), and
gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3.
"""
import numpy as np

_I2 = np.eye(2, dtype=np.complex128)
_SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def _block(a, b, c, d):
    return np.block([[a, b], [c, d]])


_Z2 = np.zeros((2, 2), dtype=np.complex128)

GAMMA = np.stack(
    [_block(_Z2, _I2, _I2, _Z2)]
    + [_block(_Z2, -1j * s, 1j * s, _Z2) for s in _SIGMA]
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE = np.eye(4, dtype=np.complex128)

# spin projectors that appear in the hopping matrix
P_MINUS = np.stack([ONE - GAMMA[mu] for mu in range(4)])   # forward hop: (1 - gamma_mu)
P_PLUS = np.stack([ONE + GAMMA[mu] for mu in range(4)])    # backward hop: (1 + gamma_mu)
