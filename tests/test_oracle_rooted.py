"""Pins of the rooted-polynomial oracle (Sec. 2.1) to the paper and to the mathematics."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import dirac, gauge, rooted
from oracle.lattice import Lattice
from oracle.su3 import expm_ah, from_coords
from paper_1805_03560_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("case", GOLDEN["alpha_rooted"]["cases"])
def test_alpha_matches_the_printed_values(case):
    a = rooted.alpha(case["N"], tuple(case["n"]), case["k"])
    printed = case["printed"]
    digits = len(printed.split(".")[1])
    # the paper truncates: the printed digits are the leading digits of alpha
    assert mpmath.floor(a * 10 ** digits) == int(printed.replace(".", "").lstrip("0") or "0"), (a, printed)


def test_alpha_tends_to_the_large_N_limit():
    # the paper states alpha -> exp(-sum_{j<=n_2} 1/j) for N -> infinity; the gap shrinks like 1/N
    lim = math.exp(-sum(1.0 / j for j in range(1, 33)))
    gaps = [float(rooted.alpha(N, (8, 32), 0)) - lim for N in (64, 256, 1024)]
    assert all(g > 0 for g in gaps) and gaps[0] > gaps[1] > gaps[2]
    assert gaps[0] / gaps[1] == pytest.approx(4.0, rel=0.1) and gaps[2] < 1.2e-5


@pytest.mark.parametrize("N,ns,k", [(2, (8, 32), 0), (4, (6, 20), 2)])
def test_polynomials_and_remainder_against_direct_evaluation(N, ns, k):
    ps = rooted.polynomials(N, ns, k)
    mp = mpmath.mpf
    hk = lambda x: mpmath.fsum(x ** i / i for i in range(1, k + 1))
    Mt = lambda x: (1 - x) * mpmath.exp(hk(x))          # M~(x)
    pv = lambda p, x: mpmath.fsum(mp(c.numerator) / c.denominator * x ** i for i, c in enumerate(p))
    # p_1 is the Taylor polynomial of M~^{-1/N}: the error at small x is O(x^{n_1 + 1})
    x = mp("0.01")
    err = abs(pv(ps[0], x) - Mt(x) ** (mp(-1) / N))
    assert err < 10 * x ** (ns[0] + 1)
    # p_2 approximates (p_1^N M~)^{-1/N}
    err = abs(pv(ps[1], x) - (pv(ps[0], x) ** N * Mt(x)) ** (mp(-1) / N))
    assert err < 10 * x ** (ns[1] + 1)
    # eq. (restM) at x = 0.4: sum_n b_n x^n + alpha / (1 - x) = 1 / (p_1^N p_2^N M~)
    b = rooted.remainder_b(N, ns, k, 150)
    a = rooted.alpha(N, ns, k)
    x = mp("0.4")
    lhs = mpmath.fsum(bn * x ** n for n, bn in enumerate(b)) + a / (1 - x)
    rhs = 1 / (pv(ps[0], x) ** N * pv(ps[1], x) ** N * Mt(x))
    assert abs(lhs - rhs) < mp("1e-20")


def _lattice(seed):
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    return lat, synth.haar_links(dims, seed)


def test_heat_baths_invert_the_actions():
    lat, U = _lattice(40)
    kappa = 0.12
    ps, b, a = rooted.coefficients_f64(3, (4, 10), 0, 60)
    eta = synth.gaussian_spinor(lat.Vh, 41)
    for p in ps:
        phi = rooted.poly_heatbath(lat, U, eta, p, kappa)
        assert rooted.poly_action(lat, U, phi, p, kappa) == pytest.approx(np.vdot(eta, eta).real, rel=1e-11)
    phr = rooted.remainder_heatbath(lat, U, eta, ps, 3, kappa, 0, 60)
    assert rooted.remainder_action(lat, U, phr, b, a, kappa) == pytest.approx(np.vdot(eta, eta).real, rel=1e-10)


@pytest.mark.parametrize("which", ["poly", "remainder"])
def test_force_is_the_derivative_of_the_action(which):
    lat, U = _lattice(50)
    kappa = 0.13
    ps, b, a = rooted.coefficients_f64(2, (4, 9), 0, 14)
    phi = synth.gaussian_spinor(lat.Vh, 51)
    if which == "poly":
        c, al = ps[1], 0.0
        S = lambda V: rooted.poly_action(lat, V, phi, c, kappa)
    else:
        c, al = b, a
        S = lambda V: rooted.remainder_action(lat, V, phi, c, al, kappa)
    F = rooted.series_force(lat, U, phi, c, al, kappa)
    om = synth.random_algebra(lat.dims, 52)
    shift = lambda e: np.einsum("...ab,...bc->...ac", expm_ah(e * from_coords(om)), U)
    # the remainder action contains a solve to 1e-14, whose noise limits the difference quotient
    h = 1e-4 if which == "poly" else 1e-3
    fd = (8 * (S(shift(h)) - S(shift(-h))) - (S(shift(2 * h)) - S(shift(-2 * h)))) / (12 * h)
    assert float(np.sum(om * F)) == pytest.approx(fd, rel=1e-7 if which == "poly" else 1e-5)


# ---------------------------------------------------------------- HMC with the rooted action

def _hmc_setup(seed, p):
    from oracle import hmc   # noqa: F401  (integrate_levels is shared with the filter HMC)
    dims = (2, 2, 2, 4)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, seed, width=0.3)
    pi = synth.gaussian_momenta(dims, seed + 1)
    etas = [synth.gaussian_spinor(lat.Vh, seed + 2 + f) for f in range(len(p.ns) * p.N + 1)]
    return lat, U, pi, etas


def test_rooted_md_is_second_order_in_the_step_size():
    """n_t = n_max: the force is the derivative of the action in H, so Delta H falls as dtau^2 when
    every level's step is halved (leapfrog, Sec. 4.2)."""
    base = rooted.RootedHMCParams(kappa=0.15, N=2, ns=(3, 6), n_t=12, n_max=12, m=2, msub=(1, 1, 2), tau=0.5,
                                  tol=1e-14)
    lat, U, pi, etas = _hmc_setup(300, base)
    phis = rooted.rooted_heatbath(lat, U, etas, base)
    dHs = []
    for m in (2, 4, 8):
        p = rooted.RootedHMCParams(**{**base.__dict__, "m": m})
        U1, pi1 = rooted.rooted_integrate(lat, U, pi, phis, p)
        dHs.append(rooted.rooted_hamiltonian(lat, U1, pi1, phis, p) - rooted.rooted_hamiltonian(lat, U, pi, phis, p))
    r1, r2 = dHs[0] / dHs[1], dHs[1] / dHs[2]
    assert 3.0 < r1 < 5.5 and 3.5 < r2 < 4.6, dHs


def test_rooted_md_is_reversible():
    p = rooted.RootedHMCParams(kappa=0.15, N=2, ns=(3, 6), k=1, n_t=8, n_max=20, m=2, msub=(2, 1, 2), tau=0.4,
                               tol=1e-14)
    lat, U, pi, etas = _hmc_setup(310, p)
    phis = rooted.rooted_heatbath(lat, U, etas, p)
    U1, pi1 = rooted.rooted_integrate(lat, U, pi, phis, p)
    U2, _ = rooted.rooted_integrate(lat, U1, -pi1, phis, p)
    assert float(np.sum(np.abs(U - U2) ** 2)) < 1e-22


def test_rooted_without_polynomials_is_the_filter_hmc():
    """jmax = 0: one remainder field with the filter's coefficients on level 1 -- the trajectory of
    the kappa^4 filter (a separate code path: hpe's tail-sum coefficients and filtered action)."""
    from oracle import hmc
    p = rooted.RootedHMCParams(kappa=0.15, N=3, ns=(), k=2, n_t=6, n_max=29, integrator="omelyan", m=2,
                               msub=(2,), tau=0.3, tol=1e-14)
    lat, U, pi, etas = _hmc_setup(320, p)
    ref = hmc.trajectory(lat, U, pi, etas[0], 0.5, hmc.HMCParams(beta=p.beta, kappa=p.kappa, k=2, n_t=6, n_max=29,
                                                                   integrator="omelyan", m=2, m0=2, tau=0.3,
                                                                   tol=1e-14))
    res = rooted.rooted_trajectory(lat, U, pi, etas, 0.5, p)
    assert res["H0"] == pytest.approx(ref["H0"], rel=1e-12)
    assert res["dH"] == pytest.approx(ref["dH"], rel=1e-8, abs=1e-10)
    assert np.abs(res["U_end"] - ref["U_end"]).max() < 1e-12


def test_rooted_heat_bath_sets_the_action_to_the_source_norm():
    """after the heat bath, every term of the action equals |eta|^2 of its sources: exact for the
    polynomial terms, up to the truncation at n_max for the remainder."""
    p = rooted.RootedHMCParams(kappa=0.15, N=2, ns=(3, 7), k=2, n_max=60, tol=1e-14)
    lat, U, pi, etas = _hmc_setup(330, p)
    phis = rooted.rooted_heatbath(lat, U, etas, p)
    H = rooted.rooted_hamiltonian(lat, U, pi, phis, p)
    S_G = gauge.gauge_action(lat, U, p.beta + 96 * p.kappa ** 4)
    eta2 = sum(float(np.vdot(e, e).real) for e in etas)
    assert H - 0.5 * float(np.sum(pi * pi)) - S_G == pytest.approx(eta2, rel=1e-10)
