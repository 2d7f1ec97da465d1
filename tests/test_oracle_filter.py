"""Pins for the hopping-parameter-expansion filter: the paper's printed numbers (tests/golden),
its closed formulas for k = 1, the defining identity of M~^{-1} against a dense matrix
exponential, traces of powers of H against the plaquette closed form, and finite differences of
the filtered action."""
import json
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg

from oracle import dirac, gauge, hpe
from oracle.lattice import Lattice
from oracle.su3 import expm_ah, from_coords
from paper_1805_03560_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _agrees_to_printed_digits(value, printed, digits):
    """|value - printed| below one unit of the last printed digit (the paper prints '1.98...',
    sometimes truncated, sometimes rounded)."""
    unit = 10.0 ** (math.floor(math.log10(abs(printed))) - digits + 1)
    return abs(value - printed) < unit


@pytest.mark.parametrize("key,k", [("truncation_terms_k1", 1), ("truncation_terms_k2", 2)])
def test_printed_truncation_values_are_heat_bath_coefficients(key, k):
    """Sec. 4.1 prints the size of the last kept terms at n_t and n_max; they agree with the
    Taylor coefficients c_n of exp(sum_{j<=k} x^j/j) (the series of M~ / M_oo)."""
    g = GOLDEN[key]
    _, _, c, _ = hpe.coefficients(k, max(g["n"]))
    for n, printed in zip(g["n"], g["printed"]):
        assert _agrees_to_printed_digits(float(c[n]), printed, g["printed_digits"])


def test_k1_coefficients_match_the_closed_formulas():
    """Sec. 2 (k = 1): a_n = sum_{i<=n} (-1)^i/i!, alpha = e^{-1}, b_n = -sum_{i>n} (-1)^i/i!."""
    a, b, c, al = hpe.coefficients(1, 25)
    assert float(al) == pytest.approx(GOLDEN["alpha_k1"]["value"], rel=1e-16)
    for n in range(26):
        an = mpmath.fsum((-1) ** i / mpmath.factorial(i) for i in range(n + 1))
        bn = -mpmath.fsum((-1) ** i / mpmath.factorial(i) for i in range(n + 1, n + 80))
        assert abs(a[n] - an) < mpmath.mpf(10) ** -45
        assert abs(b[n] - bn) < mpmath.mpf(10) ** -45
        assert abs(c[n] - 1 / mpmath.factorial(n)) < mpmath.mpf(10) ** -45


def test_alpha_generator_against_printed_limits():
    """Sec. 4.2: the N -> infinity values of alpha equal exp(-sum_{j<=k} 1/j) at k = 32, 42."""
    g = GOLDEN["alpha_limits"]
    for k, printed, d in zip(g["k"], g["printed"], g["printed_digits"]):
        assert _agrees_to_printed_digits(float(hpe.alpha(k)), printed, d)
    assert float(hpe.alpha(2)) == pytest.approx(math.exp(-1.5), rel=1e-15)


def test_b_n_is_the_tail_sum_and_decays():
    """b_n = a_n - alpha = -sum_{i>n} e_i (the form Sec. 2 prints for k = 1), so b_n -> 0;
    k = 0 is the unfiltered action (alpha = 1, all b_n = 0)."""
    for k in range(0, 5):
        _, b, _, al = hpe.coefficients(k, 40)
        e = hpe.exp_series(-1, k, 300)
        for n in (0, 3, 17, 40):
            tail = -mpmath.fsum(mpmath.mpf(q.numerator) / q.denominator for q in e[n + 1:])
            assert abs(b[n] - tail) < mpmath.mpf(10) ** -40
        assert abs(b[40]) < 1e-12
        if k == 0:
            assert al == 1 and all(x == 0 for x in b)


@pytest.mark.parametrize("k,nmax", [(1, 19), (2, 29)])
def test_filtered_inverse_matches_dense_definition(k, nmax):
    """Sec. 2: sum_{n<=nmax} b_n K^n + alpha M_oo^{-1} = [M_oo exp(sum_{j<=k} K^j/j)]^{-1}."""
    dims = (2, 2, 2, 4)
    kappa = 0.156
    lat = Lattice(dims)
    U = synth.haar_links(dims, 121)
    blk = dirac.dense_blocks(lat, dirac.dense_H(lat, U))
    K = kappa ** 2 * blk["oe"] @ blk["eo"]
    Moo = np.eye(K.shape[0]) - K
    Mt = Moo @ scipy.linalg.expm(sum(np.linalg.matrix_power(K, j) / j for j in range(1, k + 1)))
    phi = synth.gaussian_spinor(lat.Vh, 122)
    ref = np.linalg.solve(Mt, phi.reshape(-1))
    got = hpe.filtered_inverse(lat, U, phi, kappa, k, nmax, tol=1e-14).reshape(-1)
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())
    # heat bath: M~ eta with the truncated c-series reproduces the dense M~ eta
    eta = synth.gaussian_spinor(lat.Vh, 123)
    np.testing.assert_allclose(hpe.heatbath_phi(lat, U, eta, kappa, k, nmax).reshape(-1), Mt @ eta.reshape(-1),
                               atol=1e-12 * np.abs(eta).max())


@pytest.mark.parametrize("k,n_t", [(0, 0), (1, 5), (2, 7)])
def test_filtered_force_finite_difference(k, n_t):
    """the Horner force of Sec. 2 is the derivative of S~_PF truncated at the same order."""
    dims = (2, 2, 2, 4)
    kappa = 0.156
    lat = Lattice(dims)
    U = synth.haar_links(dims, 131 + k)
    phi = synth.gaussian_spinor(lat.Vh, 140 + k)
    F = hpe.filtered_force(lat, U, phi, kappa, k, n_t, tol=1e-14)
    S = lambda V: hpe.filtered_action(lat, V, phi, kappa, k, n_t, tol=1e-14)
    for s in (150, 151):
        omega = synth.random_algebra(dims, s)
        eps = 1e-4
        f = lambda e: S(np.einsum("...ab,...bc->...ac", expm_ah(e * from_coords(omega)), U))
        fd = (8 * (f(eps) - f(-eps)) - (f(2 * eps) - f(-2 * eps))) / (12 * eps)
        assert np.sum(omega * F) == pytest.approx(fd, rel=1e-7)


# ---------------------------------------------------------------- traces of powers of H

def _dense_traces(lat, U, nmax):
    Hm = dirac.dense_H(lat, U)
    out, P = [], np.eye(Hm.shape[0], dtype=complex)
    for n in range(1, nmax + 1):
        P = P @ Hm
        out.append(np.trace(P))
    return Hm, out


def test_odd_traces_vanish_and_TrH2_on_2x4():
    """Sec. 2: odd powers do not contribute, n = 2 vanishes unless a length-2 loop winds.
    On 2^4 the length-2 winding gives Tr H^2 = 16 sum_{x,mu} s_mu Re Tr(U_{x,mu} U_{x+mu,mu})."""
    dims = (2, 2, 2, 2)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 161)
    Hm, tr = _dense_traces(lat, U, 3)
    assert abs(tr[0]) < 1e-10 and abs(tr[2]) < 1e-9
    wind = sum(hpe.polyakov_re_tr(lat, U, mu, -1.0 if mu == 0 else 1.0) for mu in range(4))
    assert tr[1].real == pytest.approx(16 * wind, rel=1e-12)
    assert abs(tr[1].imag) < 1e-10


def test_TrH4_is_the_plaquette_term_on_3x4():
    """Sec. 2: Tr H^4 = -64 sum_p Re Tr U_p when no length-4 loop winds (beta shift 96 kappa^4),
    and Tr H^2 = 0 when no length-2 loop winds."""
    dims = (3, 3, 3, 3)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 171)
    Hm, tr = _dense_traces(lat, U, 4)
    assert abs(tr[1]) < 1e-9
    assert tr[3].real == pytest.approx(-64 * gauge.plaquette_sum(lat, U), rel=1e-11)
    # eq. (ModGauge) at order 4: S_G + 2 (1/4) kappa^4 Tr H^4 is S_G at beta + 96 kappa^4
    kappa, beta = 0.156, 5.6
    lhs = gauge.gauge_action(lat, U, beta) + 2 * (kappa ** 4 / 4) * tr[3].real
    rhs = gauge.gauge_action(lat, U, beta + GOLDEN["delta_beta"]["coefficient"] * kappa ** 4)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_TrH4_on_4x4_has_polyakov_winding_terms():
    """on 4^4 the length-4 straight loops wind: Tr H^4 = -64 sum_p Re Tr U_p
    + 64 sum_{x,mu} s_mu Re Tr P_mu(x) with s_0 = -1 from the anti-periodic time direction."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims)
    U = synth.haar_links(dims, 181)
    Hm = dirac.dense_H(lat, U)
    H2 = Hm @ Hm
    tr4 = np.sum(H2 * H2.T)
    wind = sum(hpe.polyakov_re_tr(lat, U, mu, -1.0 if mu == 0 else 1.0) for mu in range(4))
    assert tr4.real == pytest.approx(-64 * gauge.plaquette_sum(lat, U) + 64 * wind, rel=1e-11)


def test_traces_of_K_relate_to_traces_of_H():
    """Tr K = (kappa^2/2) Tr H^2 and Tr K^2 = (kappa^4/2) Tr H^4 on an even/odd lattice."""
    dims = (2, 2, 2, 2)
    lat = Lattice(dims)
    kappa = 0.156
    U = synth.haar_links(dims, 191)
    Hm, tr = _dense_traces(lat, U, 4)
    blk = dirac.dense_blocks(lat, Hm)
    K = kappa ** 2 * blk["oe"] @ blk["eo"]
    assert np.trace(K) == pytest.approx(kappa ** 2 / 2 * tr[1], rel=1e-12)
    assert np.trace(K @ K) == pytest.approx(kappa ** 4 / 2 * tr[3], rel=1e-12)
    # the oracle's apply_K agrees with the dense K
    x = synth.gaussian_spinor(lat.Vh, 192)
    np.testing.assert_allclose(dirac.apply_K(lat, U, x, kappa).reshape(-1), K @ x.reshape(-1), atol=1e-13)
    np.testing.assert_allclose(dirac.apply_Kdag(lat, U, x, kappa).reshape(-1), K.conj().T @ x.reshape(-1),
                               atol=1e-13)


def test_delta_beta():
    assert hpe.delta_beta(0.156, 1) == 0.0
    assert hpe.delta_beta(0.156, 2) == pytest.approx(96 * 0.156 ** 4)
