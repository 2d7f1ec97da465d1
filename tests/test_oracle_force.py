"""Pins for the oracle's solver, actions and forces: dense linear algebra, closed forms at U = 1,
central finite differences of the actions along random algebra directions, covariance."""
import numpy as np
import pytest

from oracle import dirac, force, gauge
from oracle.lattice import Lattice
from oracle.solve import cg
from oracle.su3 import expm_ah, from_coords, proj_ta, to_coords
from paper_1805_03560_amd import synth


def _perturb(U, omega, eps):
    """U_{x,mu} -> exp(eps omega_{x,mu}) U_{x,mu}  (delta U = omega U, Sec. 1)."""
    return np.einsum("...ab,...bc->...ac", expm_ah(eps * from_coords(omega)), U)


def _fd(S, U, omega, eps=1e-4):
    """fourth-order central difference of S along omega."""
    f = lambda e: S(_perturb(U, omega, e))
    return (8 * (f(eps) - f(-eps)) - (f(2 * eps) - f(-2 * eps))) / (12 * eps)


def test_su3_coordinates_round_trip_and_scalar_product():
    c = np.random.default_rng(0).standard_normal((5, 8))
    A = from_coords(c)
    np.testing.assert_allclose(A, -np.swapaxes(A.conj(), -1, -2), atol=1e-15)
    np.testing.assert_allclose(np.trace(A, axis1=-2, axis2=-1), 0, atol=1e-15)
    np.testing.assert_allclose(to_coords(A), c, atol=1e-14)
    # (Pi, Pi) = -2 Tr Pi^2 = sum pi_a^2  (eq. Sproduct)
    np.testing.assert_allclose(-2 * np.trace(A @ A, axis1=-2, axis2=-1).real, (c * c).sum(-1), rtol=1e-14)
    E = expm_ah(A)
    np.testing.assert_allclose(E @ np.swapaxes(E.conj(), -1, -2), np.broadcast_to(np.eye(3), E.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(E), 1, atol=1e-14)
    # exp against a long Taylor series
    T = np.broadcast_to(np.eye(3, dtype=complex), A.shape).copy()
    term = T.copy()
    for n in range(1, 40):
        term = term @ A / n
        T = T + term
    np.testing.assert_allclose(E, T, atol=1e-13)


def test_cg_matches_dense_solve():
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 71)
    kappa = 0.156
    blk = dirac.dense_blocks(lat, dirac.dense_H(lat, U))
    Moo = np.eye(blk["oo"].shape[0]) - kappa ** 2 * blk["oe"] @ blk["eo"]
    b = synth.gaussian_spinor(lat.Vh, 72)
    x, it, res = cg(lambda v: dirac.apply_MooDagMoo(lat, U, v, kappa), b, tol=1e-14)
    assert res <= 1e-14 and it > 0
    ref = np.linalg.solve(Moo.conj().T @ Moo, b.reshape(-1))
    np.testing.assert_allclose(x.reshape(-1), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_cg_free_field_fourier_solution():
    """at U = 1 M^dag M is diagonal in momentum space: a single plane wave b gives
    x = b / [(1 - 2k sum cos p)^2 + 4k^2 sum sin^2 p] exactly."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = synth.unit_links(dims)
    kappa = 0.12
    p = [np.pi / 4, 2 * np.pi / 4, 0.0, 6 * np.pi / 4]
    phase = np.exp(1j * sum(p[mu] * lat.coords[mu] for mu in range(4)))
    u = np.random.default_rng(1).standard_normal((4, 3)) + 0j
    b = phase[..., None, None] * u
    lam = (1 - 2 * kappa * sum(np.cos(q) for q in p)) ** 2 + 4 * kappa ** 2 * sum(np.sin(q) ** 2 for q in p)
    A = lambda v: dirac.apply_Mdag(lat, U, dirac.apply_M(lat, U, v, kappa), kappa)
    x, _, res = cg(A, b, tol=1e-14)
    np.testing.assert_allclose(x, b / lam, atol=1e-13)


def test_gauge_action_unit_field_and_plaquette():
    dims = (2, 4, 2, 4)
    lat = Lattice(dims)
    U = synth.unit_links(dims)
    assert gauge.plaquette(lat, U) == pytest.approx(1.0, abs=1e-15)
    assert gauge.gauge_action(lat, U, 5.6) == pytest.approx(-5.6 / 3 * 3 * 6 * lat.V, rel=1e-15)
    np.testing.assert_allclose(gauge.gauge_force(lat, U, 5.6), 0, atol=1e-14)
    # the smooth generator gives a plaquette near 0.79, Haar near 0
    assert 0.75 < gauge.plaquette(lat, synth.smooth_links(dims, 3)) < 0.83
    assert abs(gauge.plaquette(Lattice((4, 4, 4, 4)), synth.haar_links((4, 4, 4, 4), 4))) < 0.05


def test_gauge_force_finite_difference():
    dims = (2, 2, 4, 2)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 81)
    beta = 5.6
    F = gauge.gauge_force(lat, U, beta)
    for seed in (82, 83):
        omega = synth.random_algebra(dims, seed)
        fd = _fd(lambda V: gauge.gauge_action(lat, V, beta), U, omega)
        assert np.sum(omega * F) == pytest.approx(fd, rel=1e-8)


def test_pf_force_full_lattice_finite_difference():
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 91)
    kappa = 0.156
    phi = synth.gaussian_spinor(lat.V, 92).reshape(dims + (4, 3))
    F = force.pf_force_full(lat, U, phi, kappa, tol=1e-14)
    for seed in (93, 94):
        omega = synth.random_algebra(dims, seed)
        fd = _fd(lambda V: force.pf_action_full(lat, V, phi, kappa, tol=1e-14), U, omega)
        assert np.sum(omega * F) == pytest.approx(fd, rel=1e-7)


@pytest.mark.parametrize("dims,seed", [((2, 2, 2, 2), 101), ((4, 2, 2, 4), 102)])
def test_pf_force_eo_finite_difference(dims, seed):
    lat = Lattice(dims)
    U = synth.haar_links(dims, seed)
    kappa = 0.156
    phi = synth.gaussian_spinor(lat.Vh, seed + 1)
    F = force.pf_force_eo(lat, U, phi, kappa, tol=1e-14)
    for s in (seed + 2, seed + 3):
        omega = synth.random_algebra(dims, s)
        fd = _fd(lambda V: force.pf_action_eo(lat, V, phi, kappa, tol=1e-14), U, omega)
        assert np.sum(omega * F) == pytest.approx(fd, rel=1e-7)


def test_pf_force_gauge_covariance():
    """F_{x,mu} -> g_x F_{x,mu} g_x^dag when U -> U^g and phi -> g phi."""
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 111)
    g = synth.gauge_transform(dims, 112)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ab,...bc,...dc->...ad", g, U[..., mu, :, :],
                                      np.roll(g, -1, axis=mu).conj())
    kappa = 0.15
    phi = synth.gaussian_spinor(lat.Vh, 113)
    phig = lat.to_half(np.einsum("...ab,...sb->...sa", g, lat.to_full(phi, 1)), 1)
    F = from_coords(force.pf_force_eo(lat, U, phi, kappa, tol=1e-14))
    Fg = from_coords(force.pf_force_eo(lat, Ug, phig, kappa, tol=1e-14))
    rot = np.einsum("...ab,...mbc,...dc->...mad", g, F, g.conj())
    np.testing.assert_allclose(Fg, rot, atol=1e-10)


def test_proj_ta_properties():
    A = np.random.default_rng(2).standard_normal((4, 3, 3)) + 1j * np.random.default_rng(3).standard_normal((4, 3, 3))
    P = proj_ta(A)
    np.testing.assert_allclose(P, -np.swapaxes(P.conj(), -1, -2), atol=1e-15)
    np.testing.assert_allclose(np.trace(P, axis1=-2, axis2=-1), 0, atol=1e-15)
    # Re Tr(omega A) = Re Tr(omega P_TA(A)) for every antihermitian traceless omega
    w = from_coords(np.random.default_rng(4).standard_normal((4, 8)))
    np.testing.assert_allclose(np.trace(w @ A, axis1=-2, axis2=-1).real,
                               np.trace(w @ P, axis1=-2, axis2=-1).real, atol=1e-14)
