"""Seeded synthetic inputs: gauge fields, pseudo-fermion sources and momenta.

This module holds no arithmetic of the method itself (no hopping matrix, solver, force or
integrator step); it only draws random numbers and turns them into valid inputs.  Tests feed
the same arrays to the oracle and to the HIP library, and ``bench.py`` uses it for its
workloads.  All outputs are numpy arrays in the canonical layouts of the C header:

* gauge field   complex128 (L_t, L_z, L_y, L_x, 4, 3, 3)
* spinor        complex128 (n_sites, 4, 3)
* momenta       float64    (L_t, L_z, L_y, L_x, 4, 8)   (coordinates on T_a = i lambda_a / 2)

The paper simulates thermalised beta = 5.6 ensembles; none ship with it, so two generators
stand in for them: Haar-random links (rough, plaquette ~ 0) and "smooth" links
exp(i sum_a theta_a lambda_a / 2) with theta_a ~ N(0, width^2) (plaquette ~ 0.79 at width 0.3).
"""
import numpy as np

_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
for _a, (_i, _j) in enumerate([(0, 1), (0, 2), (1, 2)]):
    _GELL_MANN[2 * _a][_i, _j] = _GELL_MANN[2 * _a][_j, _i] = 1.0
    _GELL_MANN[2 * _a + 1][_i, _j], _GELL_MANN[2 * _a + 1][_j, _i] = -1j, 1j
_GELL_MANN[6] = np.diag([1.0, -1.0, 0.0])
_GELL_MANN[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
# reorder into the standard lambda_1 .. lambda_8 numbering
_GELL_MANN = _GELL_MANN[[0, 1, 6, 2, 3, 4, 5, 7]]


def rng(seed):
    return np.random.default_rng(seed)


def haar_su3(n, seed):
    """n Haar-distributed SU(3) matrices: QR of a complex Gaussian, phases of diag(R) moved
    into Q, then the determinant phase divided out by its principal cube root."""
    g = rng(seed)
    z = (g.standard_normal((n, 3, 3)) + 1j * g.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def haar_links(dims, seed):
    dims = tuple(dims)
    n = int(np.prod(dims)) * 4
    return haar_su3(n, seed).reshape(dims + (4, 3, 3))


def unit_links(dims):
    dims = tuple(dims)
    U = np.zeros(dims + (4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def smooth_links(dims, seed, width=0.3, threads=None):
    """exp(i sum_a theta_a lambda_a / 2), theta_a ~ N(0, width^2), exponentiated with torch."""
    import torch
    dims = tuple(dims)
    n = int(np.prod(dims)) * 4
    theta = rng(seed).standard_normal((n, 8)) * width
    out = np.empty((n, 3, 3), dtype=np.complex128)
    chunk = 1 << 20
    old = torch.get_num_threads()
    if threads:
        torch.set_num_threads(threads)
    try:
        for s in range(0, n, chunk):
            A = np.einsum("na,aij->nij", 0.5j * theta[s:s + chunk], _GELL_MANN)
            out[s:s + chunk] = torch.linalg.matrix_exp(torch.from_numpy(A)).numpy()
    finally:
        torch.set_num_threads(old)
    return out.reshape(dims + (4, 3, 3))


def gaussian_spinor(n_sites, seed):
    """complex Gaussian with density exp(-|eta|^2): Re and Im parts ~ N(0, 1/2)."""
    g = rng(seed)
    return (g.standard_normal((n_sites, 4, 3)) + 1j * g.standard_normal((n_sites, 4, 3))) / np.sqrt(2.0)


def gaussian_momenta(dims, seed):
    """pi_a ~ N(0, 1) on every link, i.e. density exp(-(Pi,Pi)/2)."""
    return rng(seed).standard_normal(tuple(dims) + (4, 8))


def random_algebra(dims, seed, scale=1.0):
    return rng(seed).standard_normal(tuple(dims) + (4, 8)) * scale


def gauge_transform(dims, seed):
    """one Haar SU(3) matrix per site, shape (dims, 3, 3)."""
    dims = tuple(dims)
    return haar_su3(int(np.prod(dims)), seed).reshape(dims + (3, 3))


def uniform(seed):
    return float(rng(seed).random())
