"""Pins of the run analysis: integrated autocorrelation time on processes with a known answer,
and the acceptance relations of Sec. 3 on Gaussian Delta H (where they hold exactly)."""
import math

import numpy as np
import pytest

from paper_1805_03560_amd import analysis


def ar1(n, rho, seed):
    g = np.random.default_rng(seed)
    e = g.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / math.sqrt(1 - rho * rho)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + e[i]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.8, 0.95])
def test_tau_int_of_ar1_process(rho):
    # AR(1): Gamma(t) / Gamma(0) = rho^t, tau_int = 1/2 + sum_t rho^t = (1 + rho) / (2 (1 - rho))
    exact = (1 + rho) / (2 * (1 - rho))
    x = ar1(400_000, rho, 7)
    t, dt, W = analysis.tau_int(x)
    assert abs(t - exact) < max(4 * dt, 0.02 * exact), (t, dt, exact, W)


def test_mean_error_matches_the_spread_of_independent_runs():
    rho, n = 0.9, 20_000
    means, errs = [], []
    for s in range(40):
        m, e, _ = analysis.mean_err(ar1(n, rho, 100 + s))
        means.append(m)
        errs.append(e)
    # the quoted error estimates the standard deviation of the mean over independent runs
    assert np.std(means) == pytest.approx(np.mean(errs), rel=0.3)


def test_acceptance_relations_for_gaussian_dH():
    # dH ~ N(v/2, v) satisfies <exp(-dH)> = 1 exactly, and then
    # <min(1, exp(-dH))> = erfc(sqrt(v / 8))
    g = np.random.default_rng(3)
    for v in (0.02, 0.0886, 0.3):
        dh = g.normal(v / 2, math.sqrt(v), 2_000_000)
        assert np.mean(np.exp(-dh)) == pytest.approx(1.0, abs=5e-3)
        assert np.mean(np.minimum(1.0, np.exp(-dh))) == pytest.approx(analysis.creutz_pacc(v), abs=2e-3)
    assert analysis.creutz_pacc(0.0) == 1.0


def test_summarize_synthetic_run():
    g = np.random.default_rng(5)
    v = 0.09
    recs = []
    for i in range(3000):
        dh = float(g.normal(v / 2, math.sqrt(v)))
        recs.append({"traj": i, "plaquette": 0.57 + 1e-3 * g.standard_normal(), "dH": dh,
                     "accepted": int(g.random() < min(1.0, math.exp(-dh))), "cg_iters": 100, "seconds": 0.1,
                     "F_PF2": 1000 + g.standard_normal()})
    s = analysis.summarize(recs, therm=1000)
    assert s["n"] == 2000 and s["first"] == 1000
    assert s["plaquette"]["mean"] == pytest.approx(0.57, abs=5 * s["plaquette"]["err"])
    assert s["var_dH"]["value"] == pytest.approx(v, rel=0.1)
    assert s["P_acc"]["mean"] == pytest.approx(s["P_acc_from_var_dH"], abs=0.02)
    assert s["exp_minus_dH"]["mean"] == pytest.approx(1.0, abs=0.05)
    assert s["var_F_PF2"]["value"] == pytest.approx(1.0, rel=0.15)


def test_probe_columns_are_summarised():
    recs = [{"traj": i, "plaquette": 0.5, "dH": 0.1 * (-1) ** i, "accepted": 1, "cg_iters": 1, "seconds": 0.1,
             "dH_nt5": 0.2 * (-1) ** i, "dH_nt15": 0.1 * (-1) ** i} for i in range(40)]
    s = analysis.summarize(recs)
    assert s["probe_n_t=5"]["var_dH"] == pytest.approx(0.04)
    assert s["probe_n_t=15"]["P_acc"] == pytest.approx(0.5 * (1 + np.exp(-0.1)))
    assert list(k for k in s if k.startswith("probe")) == ["probe_n_t=5", "probe_n_t=15"]


def test_chains_are_pooled_and_compared():
    rng = np.random.default_rng(3)
    chains = [[{"traj": i, "plaquette": 0.57 + 0.001 * c + 1e-4 * rng.standard_normal(), "dH": 0.1 * rng.standard_normal(),
                "accepted": 1, "cg_iters": 1, "seconds": 0.1} for i in range(60)] for c in range(3)]
    s = analysis.summarize_chains(chains, therm=10)
    assert [c["n"] for c in s["chains"]] == [50, 50, 50] and s["pooled"]["n"] == 150
    b = s["plaquette_between_chains"]
    assert b["mean"] == pytest.approx(0.571, abs=1e-4) and b["err"] == pytest.approx(0.001 / 3 ** 0.5, rel=0.1)


def test_ensemble_command_line_is_checked_before_the_gpu():
    from paper_1805_03560_amd import ensemble
    base = ["--out", "unused"]
    ok = [["--rooted", "4", "8", "32", "--msub", "6", "5", "4"], ["--masspre", "0.14", "--msub", "6", "2"],
          ["--probe-nt", "4", "5"], ["--rooted", "4", "8", "32"]]
    for extra in ok:
        ensemble.check_args(ensemble.parse(base + extra))
    bad = [["--rooted", "4", "8", "--masspre", "0.14"], ["--rooted", "4", "8", "32", "--msub", "6", "5"],
           ["--masspre", "0.12", "0.14", "--msub", "6", "2"], ["--rooted", "4", "8", "--probe-nt", "5"]]
    for extra in bad:
        with pytest.raises(SystemExit):
            ensemble.check_args(ensemble.parse(base + extra))
