"""The ensemble driver on a small lattice: records are complete and a run resumed from its
checkpoint reproduces the uninterrupted run exactly (per-trajectory random streams, deterministic
reductions)."""
import json
import os

import pytest

from paper_1805_03560_amd import ensemble

pytestmark = pytest.mark.gpu

ARGS = ["--dims", "4", "4", "4", "4", "--kappa", "0.15", "--filter", "1", "6", "12", "--m", "3", "--m0", "2",
        "--tau", "0.5", "--seed", "11", "--forces"]


def read(d):
    with open(os.path.join(d, "traj.jsonl")) as f:
        return [json.loads(line) for line in f]


def test_ensemble_run_and_resume(tmp_path):
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    ensemble.main(ARGS + ["--ntraj", "3", "--out", a])
    ensemble.main(ARGS + ["--ntraj", "2", "--out", b])
    ensemble.main(ARGS + ["--ntraj", "1", "--out", b, "--resume", os.path.join(b, "U_last.npy"), "--first", "2"])
    ra, rb = read(a), read(b)
    assert [r["traj"] for r in ra] == [0, 1, 2] and [r["traj"] for r in rb] == [0, 1, 2]
    for x, y in zip(ra, rb):
        for key in ("plaquette", "dH", "accepted", "u", "F_PF2", "F_G2", "cg_iters"):
            assert x[key] == y[key], key
    for r in ra:
        assert 0.0 < r["plaquette"] < 1.0 and r["F_PF2"] > 0 and r["F_G2"] > 0 and r["cg_iters"] > 0
        assert r["accepted"] == int(r["u"] < min(1.0, r["exp_mdH"]))


ROOTED = ["--dims", "4", "4", "4", "4", "--kappa", "0.13", "--filter", "0", "12", "30", "--rooted", "2", "3", "6",
          "--msub", "2", "1", "2", "--m", "2", "--integrator", "leapfrog", "--tau", "0.5", "--seed", "12", "--forces",
          "--md-prec", "f32"]


def test_rooted_ensemble_run_and_resume(tmp_path):
    """the rooted-polynomial mode: one force record per term, and an exact resume."""
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    ensemble.main(ROOTED + ["--ntraj", "2", "--out", a])
    ensemble.main(ROOTED + ["--ntraj", "1", "--out", b])
    ensemble.main(ROOTED + ["--ntraj", "1", "--out", b, "--resume", os.path.join(b, "U_last.npy"), "--first", "1"])
    ra, rb = read(a), read(b)
    for x, y in zip(ra, rb):
        for key in ("plaquette", "dH", "accepted", "F_PF12", "F_PF22", "F_PF32", "F_G2", "cg_iters", "poly_iters"):
            assert x[key] == y[key], key
    for r in ra:
        assert r["F_PF12"] > 0 and r["F_PF22"] > 0 and r["F_PF32"] > 0 and r["poly_iters"] > 0


MASSPRE = ["--dims", "4", "4", "4", "4", "--kappa", "0.15", "--filter", "2", "7", "29", "--masspre", "0.12",
           "--msub", "2", "2", "--m", "2", "--integrator", "omelyan", "--tau", "0.5", "--seed", "13", "--forces"]


def test_masspre_ensemble_run_and_resume(tmp_path):
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    ensemble.main(MASSPRE + ["--ntraj", "2", "--out", a])
    ensemble.main(MASSPRE + ["--ntraj", "1", "--out", b])
    ensemble.main(MASSPRE + ["--ntraj", "1", "--out", b, "--resume", os.path.join(b, "U_last.npy"), "--first", "1"])
    ra, rb = read(a), read(b)
    for x, y in zip(ra, rb):
        for key in ("plaquette", "dH", "accepted", "F_PF12", "F_PF22", "F_G2", "cg_iters"):
            assert x[key] == y[key], key
    for r in ra:
        assert r["F_PF12"] > 0 and r["F_PF22"] > 0 and r["cg_iters"] > 0


def test_probe_nt_reproduces_the_trajectory_at_its_own_n_t(tmp_path):
    """a probe at the production n_t integrates the same (U, pi, phi): its Delta H is the
    trajectory's; other n_t give other Delta H, and the field is left as the trajectory found it."""
    a = str(tmp_path / "a")
    ensemble.main(ARGS + ["--ntraj", "2", "--out", a, "--probe-nt", "6", "3"])
    b = str(tmp_path / "b")
    ensemble.main(ARGS + ["--ntraj", "2", "--out", b])
    for x, y in zip(read(a), read(b)):
        assert x["dH_nt6"] == pytest.approx(x["dH"], rel=1e-12, abs=1e-12)
        assert x["dH_nt3"] != x["dH"]
        assert x["dH"] == y["dH"] and x["plaquette"] == y["plaquette"]
