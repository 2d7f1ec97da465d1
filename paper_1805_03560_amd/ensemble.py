"""Ensemble generation: two-flavour Wilson HMC with kappa^k filtering on one GPU.

Runs the trajectory of Sec. 1 (heat bath of Pi and eta, phi = M~ eta; molecular dynamics with the
Omelyan or leapfrog integrator on two time scales; Metropolis step) through
`Context.hmc_trajectory` and records per trajectory the plaquette P = Re Tr U_p / 3 averaged over
all plaquettes (Sec. 4.1), Delta H, the acceptance, exp(-Delta H) (Sec. 3), the solver iterations
and optionally the squared norms (F, F) of the pseudo-fermion and gauge forces at the start of
the trajectory, whose variances over the ensemble enter the acceptance estimate of Sec. 3.

All random numbers are drawn per trajectory from a generator seeded with (seed, trajectory
index): pi_a ~ N(0, 1) on every link, Re and Im of eta ~ N(0, 1/2) (density exp(-|eta|^2)),
u ~ U[0, 1) for the accept test.  Components are independent, so they are drawn directly in the
library's device layouts.  A run can therefore stop at any trajectory and be resumed from its
gauge-field checkpoint with the same stream of random numbers; the solver blocking is fixed, so
a resumed run reproduces the uninterrupted one bit for bit.

    python -m paper_1805_03560_amd.ensemble --dims 24 12 12 12 --beta 5.6 --kappa 0.156 \\
        --filter 2 15 29 --integrator omelyan --m 6 --m0 4 --tau 1.41421356 --ntraj 500 \\
        --out run_k4 [--resume run_k4/U_last.npy --first 500] [--max-seconds 1000]

With --rooted N n_1 .. n_jmax the pseudo-fermion action is the rooted-polynomial one of Sec. 2.1
(built on the filter of --filter, whose n_t and n_max then truncate the remainder) on the
multi-level scheme of Sec. 4.2: --msub m_0 .. m_jmax, --m remainder steps, e.g. the 16^3 x 32 runs

    python -m paper_1805_03560_amd.ensemble --dims 32 16 16 16 --beta 5.6 --kappa 0.1575 \\
        --filter 0 160 400 --rooted 4 8 32 --msub 6 5 4 --m 5 --integrator leapfrog --out run_N4

With --masspre kappa_1 .. kappa_n the determinant is split by mass preconditioning (Sec. 1, 5):
the heaviest factor carries the filter of --filter at kappa_1, each ratio
det M_oo(kappa_{i+1}) / det M_oo(kappa_i) has its own field and level (--msub m_0 .. m_n).

Writes <out>/traj.jsonl (one JSON record per trajectory) and <out>/U_last.npy (the gauge field
after the last trajectory, complex128 (L_t, L_z, L_y, L_x, 4, 3, 3)).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--dims", type=int, nargs=4, default=[24, 12, 12, 12], metavar=("LT", "LZ", "LY", "LX"))
    ap.add_argument("--beta", type=float, default=5.6)
    ap.add_argument("--kappa", type=float, default=0.156)
    ap.add_argument("--filter", type=int, nargs=3, default=[2, 15, 29], metavar=("K", "N_T", "N_MAX"),
                    help="kappa^(2K) filtering with the series truncated at n_t (force) and n_max (action)")
    ap.add_argument("--integrator", choices=["omelyan", "leapfrog"], default="omelyan")
    ap.add_argument("--lam", type=float, default=1.0 / 6.0)
    ap.add_argument("--m", type=int, default=6, help="coarse (pseudo-fermion) steps per trajectory")
    ap.add_argument("--m0", type=int, default=4, help="fine (gauge) steps per coarse step")
    ap.add_argument("--tau", type=float, default=math.sqrt(2.0), help="trajectory length, (Pi,Pi) = -2 sum Tr Pi^2")
    ap.add_argument("--ntraj", type=int, default=100)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--start", choices=["hot", "cold"], default="hot")
    ap.add_argument("--resume", default=None, help="gauge field .npy to start from")
    ap.add_argument("--first", type=int, default=0, help="index of the first trajectory (random stream)")
    ap.add_argument("--md-tol", type=float, default=1e-10)
    ap.add_argument("--md-prec", choices=["f64", "f32", "f16"], default="f64",
                    help="Krylov precision of the force solves (mixed precision with FP64 reliable updates, "
                         "12-real links; the true FP64 residual still reaches --md-tol)")
    ap.add_argument("--action-tol", type=float, default=1e-12)
    ap.add_argument("--rhs-lanes", type=int, default=2,
                    help="multi-RHS blocking of the two-rhs force solves (fixed, not autotuned, so that runs are "
                         "bitwise reproducible: the blocking sets the summation order of the reductions)")
    ap.add_argument("--rooted", type=int, nargs="+", default=None, metavar="N_OR_DEGREE",
                    help="rooted polynomials: root order N, then the degrees n_1 .. n_jmax (Sec. 2.1)")
    ap.add_argument("--masspre", type=float, nargs="+", default=None, metavar="KAPPA_I",
                    help="mass preconditioning: heavier hopping parameters kappa_1 < ... < kappa_n (Sec. 1, 5)")
    ap.add_argument("--msub", type=int, nargs="+", default=None,
                    help="rooted / mass-preconditioned action: steps of level l-1 per step of level l, l = 1 ..")
    ap.add_argument("--heatbath-tol", type=float, default=1e-12, help="rooted action: CG on p_j^dag p_j")
    ap.add_argument("--forces", action="store_true", help="record (F,F) of every force at each start")
    ap.add_argument("--probe-nt", type=int, nargs="+", default=None, metavar="N_T",
                    help="filter action only: at each trajectory start also integrate the same (U, pi, phi) with "
                         "these force truncations and record their Delta H (field not updated); the equilibrium "
                         "does not depend on n_t, so averages over the run give P_acc(n_t) (Sec. 4.1)")
    ap.add_argument("--max-seconds", type=float, default=None, help="stop after this much wall time")
    ap.add_argument("--compare-solvers", action="store_true",
                    help="at the end, time BiCGstab on M_oo against CG on the normal equations on the final field")
    ap.add_argument("--out", required=True)
    ap.add_argument("--checkpoint", default=None,
                    help="where the gauge field is saved (default <out>/U_last.npy); 16^3 x 32 is 75 MB")
    return ap.parse_args(argv)


def compare_solvers(ctx, whmc, torch, b, kappa):
    """BiCGstab on M_oo vs CG on the normal equations for M_oo x = b, both to |b - M x| / |b| <= 1e-10"""
    res = {}
    stream = ctx.stream
    bn = float(torch.linalg.vector_norm(b))

    def timed(fn):
        fn()   # warm-up of this path
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    (x, st), ms = timed(lambda: ctx.bicgstab_solve(b, kappa, params=whmc.cg_params(tol=1e-10)))
    r = float(torch.linalg.vector_norm(b - ctx.apply_Moo(x, kappa))) / bn
    res["bicgstab"] = {"ms": round(ms, 2), "iters": st["iters"], "hops": 4 * st["iters"], "residual_Moo": r}
    # CG on the normal equations: tolerance on |M^dag b - A x| / |M^dag b| tightened until the
    # M_oo residual is below 1e-10 as well
    bd = ctx.apply_Moo(b, kappa, dagger=True)
    for tol in (1e-10, 3e-11, 1e-11):
        (xs, sts), ms = timed(lambda: ctx.cg_solve(bd, [kappa], whmc.cg_params(tol=tol)))
        r = float(torch.linalg.vector_norm(b - ctx.apply_Moo(xs, kappa))) / bn
        if r <= 1e-10:
            break
    res["cg_normal_equations"] = {"ms": round(ms, 2), "iters": sts[0]["iters"], "hops": 4 * sts[0]["iters"],
                                  "residual_Moo": r, "cg_tol": tol}
    res["speedup_bicgstab_vs_cgne"] = round(res["cg_normal_equations"]["ms"] / res["bicgstab"]["ms"], 3)
    return res


def probe_nt(ctx, whmc, a, p, pi, eta, rec):
    """Delta H of the molecular dynamics from the current field with each n_t in a.probe_nt
    (same pi and phi as the trajectory that follows); the field is restored afterwards."""
    k, _, n_max = a.filter
    U0 = ctx.export_gauge()
    phi = ctx.heatbath_phi(eta, k, p.filter.n_t, n_max, a.kappa)
    H0 = ctx.hamiltonian(p, pi, phi)
    for nt in a.probe_nt:
        q = whmc.hmc_params(beta=a.beta, kappa=a.kappa, k=k, n_t=nt, n_max=n_max, integrator=p.integrator,
                            lam=p.lam, m=p.m, m0=p.m0, tau=p.tau, md_solver=p.md_solver,
                            action_solver=p.action_solver)
        pic = pi.clone()
        ctx.md_integrate(q, pic, phi)
        rec[f"dH_nt{nt}"] = ctx.hamiltonian(q, pic, phi) - H0
        ctx.load_gauge(U0, unitarity_tol=0.0)


def draws(torch, dev, seed, traj, n_pi, n_eta):
    """(pi, eta, u) of trajectory `traj`: a generator seeded with (seed, traj)."""
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed) * 1_000_003 + int(traj))
    pi = torch.randn(n_pi, generator=g, device=dev, dtype=torch.float64)
    eta = torch.randn(n_eta, generator=g, device=dev, dtype=torch.float64) * math.sqrt(0.5)
    u = float(torch.rand(1, generator=g, device=dev, dtype=torch.float64).item())
    return pi, eta, u


def check_args(a):
    """consistency of the command line, before anything touches the GPU (SystemExit on error)."""
    if a.rooted and a.masspre:
        raise SystemExit("--rooted and --masspre are separate actions")
    if a.rooted and len(a.rooted) < 1:
        raise SystemExit("--rooted needs the root order N")
    n_levels = (len(a.rooted) - 1 if a.rooted else len(a.masspre) if a.masspre else None)
    if n_levels is not None and a.msub is not None and len(a.msub) != n_levels + 1:
        raise SystemExit("--msub needs m_0 .. m_n: one more value than there are polynomials (--rooted) or "
                         "heavier kappas (--masspre)")
    if a.probe_nt and (a.rooted or a.masspre):
        raise SystemExit("--probe-nt applies to the filter action only")


def main(argv=None):
    a = parse(argv)
    check_args(a)
    import torch
    from paper_1805_03560_amd import synth, whmc

    os.makedirs(a.out, exist_ok=True)
    ckpt = a.checkpoint or os.path.join(a.out, "U_last.npy")
    if os.path.dirname(ckpt):
        os.makedirs(os.path.dirname(ckpt), exist_ok=True)
    dims = tuple(a.dims)
    V = int(np.prod(dims))
    Vh = V // 2
    ctx = whmc.Context(dims, device=0)
    dev = ctx.device
    if a.resume:
        U = np.load(a.resume)
    elif a.start == "hot":
        U = synth.haar_links(dims, a.seed)
    else:
        U = synth.unit_links(dims)
    ctx.load_gauge(torch.from_numpy(U).to(dev), unitarity_tol=1e-10)
    k, n_t, n_max = a.filter
    integ = whmc.OMELYAN if a.integrator == "omelyan" else whmc.LEAPFROG
    if a.md_prec == "f64":
        md = whmc.cg_params(tol=a.md_tol, rhs_block=1, rhs_lanes=a.rhs_lanes)
    else:
        prec, delta = (whmc.F32, 1e-4) if a.md_prec == "f32" else (whmc.F16, 1e-2)
        md = whmc.cg_params(tol=a.md_tol, prec=prec, links=whmc.L12, delta=delta, rhs_block=1,
                            rhs_lanes=a.rhs_lanes)
    act = whmc.cg_params(tol=a.action_tol)
    if a.masspre:
        mp = whmc.masspre(a.masspre, k=k, n_t=n_t, n_max=n_max)
        msub = a.msub or [a.m0] + [1] * mp.n
        p = whmc.masspre_hmc_params(beta=a.beta, kappa=a.kappa, mp=mp, integrator=integ, lam=a.lam, m=a.m,
                                    msub=msub, tau=a.tau, md_solver=md, action_solver=act)
        n_fields = mp.n + 1
    elif a.rooted:
        r = whmc.rooted(a.rooted[0], a.rooted[1:], k=k, n_t=n_t, n_max=n_max)
        msub = a.msub or [a.m0] + [1] * r.jmax
        p = whmc.rooted_hmc_params(beta=a.beta, kappa=a.kappa, rooted_action=r, integrator=integ, lam=a.lam, m=a.m,
                                   msub=msub, tau=a.tau, md_solver=md, action_solver=act,
                                   heatbath_solver=whmc.cg_params(tol=a.heatbath_tol))
        n_fields = r.jmax * r.N + 1
    else:
        p = whmc.hmc_params(beta=a.beta, kappa=a.kappa, k=k, n_t=n_t, n_max=n_max, integrator=integ, lam=a.lam,
                            m=a.m, m0=a.m0, tau=a.tau, md_solver=md, action_solver=act)
        n_fields = 1
    n_pi = 64 * Vh                # 2 parities x 4 directions x 8 generators x Vh
    n_eta = 24 * Vh * n_fields    # 12 complex components x Vh per pseudo-fermion field
    log = open(os.path.join(a.out, "traj.jsonl"), "a")
    t_start = time.time()
    done = 0
    for traj in range(a.first, a.first + a.ntraj):
        pi, eta, u = draws(torch, dev, a.seed, traj, n_pi, n_eta)
        rec = {"traj": traj}
        if a.forces:
            # gauge action with the filter's shift at kappa (truncations play no part in it)
            fg = ctx.force(ctx.half_spinor(), k, 0, 0, a.kappa, a.beta, flags=whmc.FORCE_GAUGE)
            rec["F_G2"] = float(torch.dot(fg, fg))
            if a.masspre:
                phi = ctx.masspre_heatbath(eta, p.mp, a.kappa, solver=act)
                for term in range(1, p.mp.n + 2):
                    f = ctx.masspre_force(phi, p.mp, a.kappa, term=term, solver=md)
                    rec[f"F_PF{term}2"] = float(torch.dot(f, f))
            elif a.rooted:
                phi, _ = ctx.rooted_heatbath(eta, p.rooted, a.kappa, solver=p.heatbath_solver)
                for term in range(1, p.rooted.jmax + 2):
                    f = ctx.rooted_force(phi, p.rooted, a.kappa, term=term, solver=md)
                    rec[f"F_PF{term}2"] = float(torch.dot(f, f))
            else:
                phi = ctx.heatbath_phi(eta, k, n_t, n_max, a.kappa)
                fpf = ctx.force(phi, k, n_t, n_max, a.kappa, a.beta, flags=whmc.FORCE_PF, solver=md)
                rec["F_PF2"] = float(torch.dot(fpf, fpf))
        if a.probe_nt:
            probe_nt(ctx, whmc, a, p, pi, eta, rec)
        if a.masspre:
            r = ctx.masspre_trajectory(p, pi, eta, u)
        elif a.rooted:
            r = ctx.rooted_trajectory(p, pi, eta, u)
        else:
            r = ctx.hmc_trajectory(p, pi, eta, u)
        rec.update({"plaquette": r["plaquette"], "dH": r["dH"], "accepted": int(r["accepted"]), "u": u,
                    "exp_mdH": math.exp(-r["dH"]) if r["dH"] > -700 else float("inf"),
                    "cg_iters": int(r["cg_iters"]), "n_solves": int(r["n_solves"]), "seconds": r["seconds"]})
        if a.rooted:
            rec["poly_iters"] = int(r["poly_iters"])
        log.write(json.dumps(rec) + "\n")
        log.flush()
        done += 1
        if done % 10 == 0 or done == a.ntraj:
            print(f"[ensemble] traj {traj}: P {rec['plaquette']:.5f} dH {rec['dH']:+.4f} acc {rec['accepted']} "
                  f"iters {rec['cg_iters']} {rec['seconds']:.2f}s", flush=True)
            np.save(ckpt, ctx.export_gauge().cpu().numpy())
        if a.max_seconds is not None and time.time() - t_start > a.max_seconds:
            break
    np.save(ckpt, ctx.export_gauge().cpu().numpy())
    state = {"next_first": a.first + done, "checkpoint": ckpt, "args": vars(a)}
    if a.compare_solvers:
        _, eta, _ = draws(torch, dev, a.seed, -1, 0, 24 * Vh)
        state["solvers"] = compare_solvers(ctx, whmc, torch, eta, a.kappa)
        print(f"[ensemble] M_oo x = b on the final field: {state['solvers']}", flush=True)
    json.dump(state, open(os.path.join(a.out, "state.json"), "w"))
    print(f"[ensemble] {done} trajectories in {time.time() - t_start:.1f}s; next --first {a.first + done}",
          flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
