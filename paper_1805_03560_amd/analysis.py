"""Analysis of HMC runs: averages with autocorrelation-corrected errors and the acceptance checks
of Sec. 3.

- integrated autocorrelation time tau_int with the automatic window of U. Wolff, Comput. Phys.
  Commun. 156 (2004) 143 (Gamma(t) summed up to the first W where the estimated systematic
  error exp(-W/tau) falls below the statistical one sqrt(tau/(W N)); S = 1.5);
- the error of a mean, sqrt(2 tau_int Var / N);
- P_acc = <min(1, exp(-dH))>, <exp(-dH)> (= 1 by detailed balance, Sec. 3), Var(dH) and the
  high-acceptance estimate P_acc = erfc(sqrt(Var(dH) / 8)) of Sec. 3;
- Var((F, F)) of the force norms recorded at trajectory starts.

    python -m paper_1805_03560_amd.analysis RUN/traj.jsonl --therm 200
"""
import argparse
import json
import math
import sys

import numpy as np


def tau_int(x, S=1.5):
    """(tau_int, its error, window W) of the series x, automatic windowing (Wolff 2004)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 4:
        return 0.5, 0.0, 0
    d = x - x.mean()
    g0 = float(np.dot(d, d)) / n
    if g0 == 0.0:
        return 0.5, 0.0, 0
    # Gamma(t) for t < n/2 via FFT, normalised by the number of pairs
    f = np.fft.rfft(d, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[: n // 2] / (n - np.arange(n // 2))
    rho = acf / g0
    tau = 0.5
    W = 0
    for w in range(1, n // 2):
        tau = 0.5 + float(np.sum(rho[1:w + 1]))
        tw = S / math.log((2 * tau + 1) / (2 * tau - 1)) if tau > 0.5 else 1e-12
        if math.exp(-w / tw) - tw / math.sqrt(w * n) < 0:
            W = w
            break
    else:
        W = n // 2 - 1
    tau = tau * (1.0 + (2 * W + 1) / n)   # leading bias of the estimated mean in Gamma
    dtau = tau * math.sqrt((4 * W + 2) / n)
    return tau, dtau, W


def mean_err(x, S=1.5):
    """(mean, error, tau_int) with the error sqrt(2 tau_int Var / N)."""
    x = np.asarray(x, dtype=np.float64)
    t, _, _ = tau_int(x, S)
    var = float(np.var(x))
    return float(x.mean()), math.sqrt(2.0 * max(t, 0.5) * var / len(x)), t


def creutz_pacc(var_dh):
    """P_acc predicted from Var(dH) for high acceptance (Sec. 3)."""
    return math.erfc(math.sqrt(var_dh / 8.0))


def summarize(records, therm=0):
    recs = [r for r in records if r["traj"] >= therm]
    if not recs:
        return {}
    out = {"n": len(recs), "first": recs[0]["traj"], "last": recs[-1]["traj"]}
    P = [r["plaquette"] for r in recs]
    m, e, t = mean_err(P)
    out["plaquette"] = {"mean": m, "err": e, "tau_int": t}
    dh = np.array([r["dH"] for r in recs])
    pacc = np.minimum(1.0, np.exp(-np.clip(dh, -700, 700)))
    m, e, _ = mean_err(pacc)
    out["P_acc"] = {"mean": m, "err": e}
    out["accept_rate"] = float(np.mean([r["accepted"] for r in recs]))
    m, e, _ = mean_err(np.exp(-np.clip(dh, -700, 700)))
    out["exp_minus_dH"] = {"mean": m, "err": e}
    var = float(np.var(dh))
    m2, e2, _ = mean_err((dh - dh.mean()) ** 2)
    out["var_dH"] = {"value": var, "err": e2}
    out["P_acc_from_var_dH"] = creutz_pacc(var)
    out["max_abs_dH"] = float(np.max(np.abs(dh)))
    out["cg_iters_per_traj"] = float(np.mean([r["cg_iters"] for r in recs]))
    out["seconds_per_traj"] = float(np.mean([r["seconds"] for r in recs]))
    for key in sorted({k for r in recs for k in r if k.startswith("F_") and k.endswith("2")}):
        v = [r[key] for r in recs if key in r]
        if len(v) > 2:
            v = np.asarray(v)
            m4, e4, _ = mean_err((v - v.mean()) ** 2)
            out[f"var_{key}"] = {"value": float(np.var(v)), "err": e4, "mean": float(v.mean())}
    # Delta H probes at other force truncations from the same starting points (ensemble --probe-nt)
    for key in sorted({k for r in recs for k in r if k.startswith("dH_nt")}, key=lambda k: int(k[5:])):
        v = np.array([r[key] for r in recs if key in r])
        if len(v) > 2:
            m, e, _ = mean_err(np.minimum(1.0, np.exp(-np.clip(v, -700, 700))))
            m2, e2, _ = mean_err((v - v.mean()) ** 2)
            out[f"probe_n_t={key[5:]}"] = {"P_acc": m, "P_acc_err": e, "var_dH": float(np.var(v)), "var_dH_err": e2,
                                           "n": int(len(v))}
    return out


def load(path):
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def summarize_chains(chains, therm=0):
    """independent chains of one action: each chain's summary, the summary of the pooled records
    (the first `therm` trajectories of every chain dropped), and <P> with the error from the
    spread of the chain means (which does not trust the windowed error of short chains)."""
    out = {"chains": [summarize(c, therm) for c in chains]}
    pooled = [r for c in chains for r in c if r["traj"] >= therm]
    out["pooled"] = summarize(pooled)
    means = np.array([c["plaquette"]["mean"] for c in out["chains"] if c])
    if len(means) > 1:
        out["plaquette_between_chains"] = {"mean": float(means.mean()),
                                           "err": float(means.std(ddof=1) / math.sqrt(len(means))),
                                           "n_chains": int(len(means))}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="summarise HMC runs written by paper_1805_03560_amd.ensemble; several "
                                             "files are taken as independent chains of one action")
    ap.add_argument("jsonl", nargs="+")
    ap.add_argument("--therm", type=int, default=0, help="drop trajectories with index below this (per chain)")
    a = ap.parse_args(argv)
    if len(a.jsonl) == 1:
        print(json.dumps(summarize(load(a.jsonl[0]), a.therm), indent=1))
    else:
        print(json.dumps(summarize_chains([load(f) for f in a.jsonl], a.therm), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
