"""Benchmark of the Wilson-fermion hot path on one MI355X.

Headline (`value`): FP64 apply_H throughput in algorithmic GB/s on the 32^3 x 64 lattice with
smooth synthetic SU(3) links (width 0.3, seed 3000).  One step = the two even/odd hops in the
order the even/odd operator applies them, t_e = H_eo psi_o then psi_o' = H_oe t_e (18-real FP64
links), chained from step to step so that every hop reads the previous hop's output, inputs
resident in HBM.  Algorithmic bytes per hop output site: 2 spinors + 8 links
= 192 + 192 + 8 * 144 = 1536 B.  Beside it: H on a full spinor (one launch; minimal algorithmic
bytes 960 B per site, each link once) and single hops of every storage format repeated on one
input.

After the timed region the second half of the metric is measured on the same GPU (events on
the library's stream): CG to a true FP64 residual of 1e-10 in plain FP64 and in mixed precision
(FP32 and FP16 Krylov bulk, 12-real links, FP64 reliable updates), with the error against the
FP64 solution, hop throughput of the other storage formats, and the filtered force.  The oracle
is timed on the host for `cpu_baseline`.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "apply_H GB/s (% HBM roofline); CG-to-1e-10 time, FP64 vs mixed/multi-RHS"
HBM_PEAK_GBS = 8000.0
DIMS = (64, 32, 32, 32)          # (L_t, L_z, L_y, L_x)
KAPPA = 0.1575
# reliable-update thresholds: the iterated residual may fall by 1e-4 (FP32 bulk, ~1e-7 rounding)
# or 1e-2 (FP16 bulk, ~5e-4 rounding) before r = b - A x is recomputed in FP64
MIXED_F32 = lambda whmc, links=12: whmc.cg_params(tol=1e-10, prec=whmc.F32, links=links, delta=1e-4)
MIXED_F16 = lambda whmc, links=12: whmc.cg_params(tol=1e-10, prec=whmc.F16, links=links, delta=1e-2)
# algorithmic bytes per output site of an even/odd hop: in + out spinor + 8 links
BYTES_PER_SITE = {("f64", 18): 1536, ("f64", 12): 1152, ("f64", 8): 896, ("f32", 18): 768, ("f32", 12): 576,
                  ("f32", 8): 448, ("f16", 12): 296, ("f16", 8): 232}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 30 warm-up steps (~20 ms of load) let the GPU clocks settle: after 3 the first timed hops
    # still run ~2 % slower
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed apply_H region")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a device copy of 2 GiB (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--profile-kernel", choices=["hop_f16_l12", "hop_formats", "mhop_f64_12rhs", "mhop_f16_12rhs",
                                                 "pf_force_24"],
                    help="only run a short workload of one kernel (for rocprofv3 counter passes) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              f"domain decomposition is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_03560_amd import synth, whmc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 copies of 2 GiB")
        return
    if args.profile_kernel:
        profile_kernel(args.profile_kernel, whmc, torch, np)
        return
    T, Z, Y, X = DIMS
    V = T * Z * Y * X
    Vh = V // 2

    t0 = time.time()
    U = synth.smooth_links(DIMS, 3000, width=0.3, threads=min(16, os.cpu_count() or 1))
    log(f"[bench] generated 32^3x64 smooth links in {time.time() - t0:.1f}s")
    ctx = whmc.Context(DIMS, device=0)
    ctx.load_gauge(torch.from_numpy(U).to(dev), unitarity_tol=1e-11)
    del U
    stream = torch.cuda.current_stream(dev)
    psi = [ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3001)).to(dev), 1), ctx.half_spinor()]
    t_e = ctx.half_spinor()
    torch.cuda.synchronize()

    def step(k):
        ctx.apply_H(psi[k & 1], 0, out=t_e)              # t_e = H_eo psi_o
        ctx.apply_H(t_e, 1, out=psi[(k + 1) & 1])        # psi_o' = H_oe t_e

    # setup: the autotuner picks the workgroup schedule of the stencil kernels (time-slice ranges per
    # XCD, or time slabs worked through in chunks of a given size) and the occupancy cap (none, or two
    # workgroups per compute unit) by timing the same hop pair
    tuned = tune_stencil(ctx, whmc)
    log(f"[bench] stencil schedule: {tuned}")

    # ------------------------------------------------------------ timed region: apply_H FP64
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        step(args.warmup + k)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    bytes_per_launch = 1536 * Vh
    value = 2 * bytes_per_launch * args.steps / (ms * 1e-3) / 1e9
    achieved = bytes_per_launch / (ms_per_step / 2 * 1e-3) / 1e9
    log(f"[bench] apply_H FP64 even/odd pair (chained): {ms_per_step:.3f} ms/step, {value:.1f} GB/s "
        f"(wall {wall:.3f}s)")

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "apply_H even/odd hops, FP64, 18-real links, 32^3x64 smooth SU(3) links "
                               "(width 0.3, seed 3000), anti-periodic time; one step = t_e = H_eo psi_o then "
                               "psi_o' = H_oe t_e, chained",
                   "lattice_t_z_y_x": list(DIMS), "sites": V, "kappa": KAPPA},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(bytes_per_launch)},
        "stencil_schedule": tuned,
    }

    if not args.no_extras:
        result.update(extras(ctx, whmc, torch, np, stream, Vh))
    if not args.no_cpu_baseline:
        it16 = result.get("cg_16x32_fp64", {}).get("kappa0.156", {}).get("iters")
        result["cpu_baseline"] = cpu_baseline(it16)
    ctx.close()
    print(json.dumps(result), flush=True)


def profile_kernel(name, whmc, torch, np):
    """a few launches of one kernel on its benchmark workload, for counter passes:
    hop_f16_l12: the chained FP16 even/odd pair (12-real links) on 32^3 x 64;
    hop_formats: the chained pair in every storage format on 32^3 x 64 (3 timed steps each);
    mhop_f64_12rhs / mhop_f16_12rhs: the multi-RHS hop for 12 right-hand sides on 24^3 x 48 with the
    autotuned blocking; pf_force_24: the pair force of 24 (X, Y) pairs (kappa^4 filter, n_t = 23)
    on 32^3 x 64."""
    from paper_1805_03560_amd import synth
    dev = torch.device("cuda", 0)
    if name.startswith("mhop"):
        dims = (48, 24, 24, 24)
        U = synth.smooth_links(dims, 4000, threads=min(16, os.cpu_count() or 1))
    else:
        dims = DIMS
        U = synth.smooth_links(dims, 3000, width=0.3, threads=min(16, os.cpu_count() or 1))
    ctx = whmc.Context(dims, device=0)
    ctx.load_gauge(torch.from_numpy(U).to(dev), unitarity_tol=1e-11)
    tune_stencil(ctx, whmc)
    del U
    Vh = ctx.Vh
    if name == "hop_f16_l12":
        x = ctx.convert_spinor(ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3001)).to(dev), 1),
                               whmc.F64, whmc.F16)
        us = chained_pair_us(ctx, torch, ctx.stream, whmc.F16, whmc.L12, x, steps=5, warmup=2)
        info = {"us_per_hop": us}
    elif name == "hop_formats":
        x64 = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3002)).to(dev), 1)
        info = {}
        for (p, pn), links in [((whmc.F64, "f64"), 18), ((whmc.F64, "f64"), 12), ((whmc.F64, "f64"), 8),
                               ((whmc.F32, "f32"), 12), ((whmc.F32, "f32"), 8), ((whmc.F16, "f16"), 12),
                               ((whmc.F16, "f16"), 8)]:
            xin = x64.clone() if p == whmc.F64 else ctx.convert_spinor(x64, whmc.F64, p)
            info[f"{pn}-{links}_us_per_hop"] = round(chained_pair_us(ctx, torch, ctx.stream, p, links, xin, steps=3,
                                                                     warmup=1), 1)
    elif name.startswith("mhop"):
        n = 12
        prec, links = (whmc.F64, whmc.L18) if "f64" in name else (whmc.F16, whmc.L12)
        b = ctx.pack_spinor(torch.from_numpy(np.stack([synth.gaussian_spinor(Vh, 4100 + r) for r in range(n)]))
                            .to(dev), 0)
        bp = b if prec == whmc.F64 else ctx.convert_spinor(b, whmc.F64, prec, n)
        nb, lanes, order, _ = ctx.autotune(prec, links, n)
        o = ctx.half_spinor(prec, n)
        for _ in range(3):
            ctx.apply_H_multi(bp, 0, n, prec=prec, links=links, rhs_block=nb, rhs_lanes=lanes, rhs_order=order, out=o)
        info = {"blocking": [nb, lanes, order]}
    else:
        phi = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3003)).to(dev), 0)
        ctx.force(phi, 2, 23, 29, KAPPA, 5.6, solver=whmc.cg_params(tol=1e-10))
        info = {"pairs": 24}
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"profile_kernel": name, **info}), flush=True)


def tune_stencil(ctx, whmc):
    """autotune the single-RHS stencil schedule and occupancy cap of a context; returns the choice"""
    sched, chunk, us = ctx.autotune_hop()
    return {"schedule": "slice ranges" if sched == 0 else "time slabs", "chunk_blocks": chunk,
            "wg_per_cu": ctx.get_option(whmc.OPT_HOP_WG_PER_CU) or None, "tuned_us_per_hop": round(us, 1)}


def measured_traffic(bytes_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this kernel, if its
    recorded source digest still matches the stencil sources (else null)."""
    path = os.path.join(ROOT, "profiles", "k_hop_f64_l18_32x64_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    from paper_1805_03560_amd.profsum import source_digest
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def time_events(fn, stream, torch, reps=1):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extras(ctx, whmc, torch, np, stream, Vh):
    from paper_1805_03560_amd import synth
    out = {}
    # H on a full spinor in one launch; minimal algorithmic bytes 960 B per site (each link read
    # once), the kernel reads each link twice (once per parity of the output site)
    full_in = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(2 * Vh, 3004)).to(ctx.device), -1)
    full_out = ctx.full_spinor()
    ctx.apply_H(full_in, -1, out=full_out)
    ms = time_events(lambda: ctx.apply_H(full_in, -1, out=full_out), stream, torch, reps=20)
    out["full_lattice_H_f64_l18"] = {"ms": round(ms, 4),
                                     "GBps_960B_per_site": round(960 * 2 * Vh / (ms * 1e-3) / 1e9, 1),
                                     "GBps_1536B_per_site": round(1536 * 2 * Vh / (ms * 1e-3) / 1e9, 1)}
    log(f"[bench] full-lattice H FP64: {out['full_lattice_H_f64_l18']}")
    out["hop_formats_chained"] = hop_formats(ctx, whmc, torch, stream, Vh)

    # CG to 1e-10: FP64 vs mixed precision (32^3 x 64, kappa = 0.1575)
    b = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3003)).to(ctx.device), 0)
    golden = load_golden(np)
    cgr = {}
    # GPU reference solution: FP64 CG to a true residual of 1e-13
    ref, st = ctx.cg_solve(b, [KAPPA], whmc.cg_params(tol=1e-13))
    ref = ref.clone()
    if golden is not None:
        cgr["fp64_1e-13_vs_oracle"] = err_vs_golden(ctx, ref, golden, np)
    t = {}
    for name, prm in [("fp64", whmc.cg_params(tol=1e-10)),
                      ("fp64_l12", whmc.cg_params(tol=1e-10, links=whmc.L12)),
                      ("fp64_l8", whmc.cg_params(tol=1e-10, links=whmc.L8)),
                      ("mixed_f32_l12", MIXED_F32(whmc)),
                      ("mixed_f32_l8", MIXED_F32(whmc, whmc.L8)),
                      ("mixed_f16_l12", MIXED_F16(whmc)),
                      ("mixed_f16_l8", MIXED_F16(whmc, whmc.L8))]:
        ctx.cg_solve(b, [KAPPA], prm)      # warm-up of this path
        times = []
        for _ in range(3):                  # best of three solves (each one's host checks add jitter)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            x, st = ctx.cg_solve(b, [KAPPA], prm)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = min(times)
        err = float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))
        s = st[0]
        t[name] = ms
        cgr[name] = {"ms": round(ms, 2), "ms_of_3_solves": [round(v, 2) for v in times], "iters": s["iters"],
                     "reliable_updates": s["reliable_updates"], "true_residual": s["true_residual"],
                     "rel_err_vs_fp64_solution": err}
        if golden is not None:
            cgr[name]["rel_err_vs_oracle"] = err_vs_golden(ctx, x, golden, np)["rel_err_sampled"]
        log(f"[bench] CG {name}: {ms:.1f} ms, {s['iters']} iters, res {s['true_residual']:.2e}, err {err:.2e}, "
            f"vs oracle {cgr[name].get('rel_err_vs_oracle')}")
    for name in t:
        if name != "fp64":
            cgr[name]["speedup_vs_fp64"] = round(t["fp64"] / t[name], 3)
    if golden is not None:
        cgr["oracle_solution"] = {"file": "tests/golden/cg_32x64_kappa0.1575.npz", "sites": int(len(golden["sites"])),
                                  "tol": golden["meta"]["cg_tol"], "iterations": golden["meta"]["iterations"]}
    out["cg_32x64_kappa0.1575"] = cgr
    out["cg_16x32_fp64"] = cg_16x32(whmc, torch)

    # M_oo x = b to |b - M_oo x| / |b| <= 1e-10: BiCGstab on M_oo (the paper's solver) against CG on
    # the normal equations M_oo^dag M_oo x = M_oo^dag b (both FP64, 18-real links; 4 hops per
    # iteration).  BiCGstab needs the spectrum of M_oo in the right half-plane: on the smooth
    # synthetic fields of width 0.3 - 0.55 kappa = 0.1575 is past or at their critical kappa, so this
    # comparison runs on a rough field (width 0.8, plaquette ~0.15) at kappa = 0.156; on thermalised
    # beta = 5.6 fields the ensemble driver (--compare-solvers) makes the same comparison
    out["solve_Moo_32x64_width0.8_kappa0.156"] = bicgstab_vs_cgne(whmc, torch)

    out["multi_rhs_24x48"] = multi_rhs(whmc, torch, stream)
    out["hmc_32x64"] = hmc_section(ctx, whmc, torch, stream, Vh)
    out.update(widened_16x32(whmc, torch))

    # kappa^4-filtered pseudo-fermion force (n_t = 15), FP64 solves to 1e-10
    phi = b
    ms = time_events(lambda: ctx.force(phi, 2, 15, 29, KAPPA, 5.6, solver=whmc.cg_params(tol=1e-10)), stream, torch)
    out["force_kappa4_nt15_ms"] = round(ms, 1)
    log(f"[bench] filtered force (kappa^4, n_t=15): {ms:.1f} ms")
    return out


def chained_pair_us(ctx, torch, stream, prec, links, x_odd, steps=20, warmup=5):
    """microseconds per hop of the chained even/odd pair t_e = H_eo x_o, x_o' = H_oe t_e in one storage
    format: every hop reads the previous hop's output from HBM, as in the timed region"""
    xs = [x_odd, torch.empty_like(x_odd)]
    te = torch.empty_like(x_odd)

    def step(k):
        ctx.apply_H(xs[k & 1], 0, prec=prec, links=links, out=te)
        ctx.apply_H(te, 1, prec=prec, links=links, out=xs[(k + 1) & 1])
    for k in range(warmup):
        step(k)
    n = [warmup]

    def run():
        for k in range(steps):
            step(n[0] + k)
    ms = time_events(run, stream, torch)
    return ms * 1e3 / (2 * steps)


def hop_formats(ctx, whmc, torch, stream, Vh):
    """every spinor / link storage format on the chained even/odd pair of the timed region: the
    input of each hop is the previous hop's output, resident in HBM (at 32^3 x 64 the FP64 fields
    are 201 MB, the link arrays 0.2 - 1.2 GB); algorithmic bytes of the format per output site"""
    from paper_1805_03560_amd import synth
    fmt = {}
    x64 = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3002)).to(ctx.device), 1)
    for (p, pn), links in [((whmc.F64, "f64"), 18), ((whmc.F64, "f64"), 12), ((whmc.F64, "f64"), 8),
                           ((whmc.F32, "f32"), 18), ((whmc.F32, "f32"), 12), ((whmc.F32, "f32"), 8),
                           ((whmc.F16, "f16"), 12), ((whmc.F16, "f16"), 8)]:
        xin = x64.clone() if p == whmc.F64 else ctx.convert_spinor(x64, whmc.F64, p)
        us = chained_pair_us(ctx, torch, stream, p, links, xin)
        gbs = BYTES_PER_SITE[(pn, links)] * Vh / (us * 1e-6) / 1e9
        fmt[f"{pn}_l{links}"] = {"us_per_hop": round(us, 1), "bytes_per_site": BYTES_PER_SITE[(pn, links)],
                                 "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 3)}
        log(f"[bench] chained hop {pn}-{links}: {us:.1f} us, {gbs:.0f} GB/s")
    return fmt


def load_golden(np):
    """the oracle's solution of the 32^3 x 64 system at sampled sites, written by
    tests/golden/make_cg_32x64.py (oracle only); None if it is not there"""
    base = os.path.join(ROOT, "tests", "golden", "cg_32x64_kappa0.1575")
    if not (os.path.exists(base + ".npz") and os.path.exists(base + ".json")):
        return None
    z = np.load(base + ".npz", allow_pickle=False)
    return {"sites": z["sites"], "x": z["x"], "meta": json.load(open(base + ".json"))}


def err_vs_golden(ctx, x, golden, np):
    import torch
    sites = torch.from_numpy(golden["sites"]).to(ctx.device)
    got = ctx.unpack_spinor(x, 0).index_select(0, sites).cpu().numpy()
    ref = golden["x"]
    return {"rel_err_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "max_abs_err_over_max_abs": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))}


def cg_16x32(whmc, torch):
    """the plain single-RHS baseline: even/odd FP64 CG to a true residual of 1e-10 on 16^3 x 32
    smooth links (width 0.3, seed 2000), one Gaussian source (seed 2001), kappa = 0.156 and 0.1575
    (both fields fit the 256 MB Infinity Cache)"""
    from paper_1805_03560_amd import synth
    dims = (32, 16, 16, 16)
    U = synth.smooth_links(dims, 2000)
    ctx = whmc.Context(dims, device=0)
    ctx.load_gauge(torch.from_numpy(U).to(ctx.device), unitarity_tol=1e-11)
    b = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(ctx.Vh, 2001)).to(ctx.device), 0)
    res = {"stencil_schedule": tune_stencil(ctx, whmc)}
    for kappa in (0.156, 0.1575):
        prm = whmc.cg_params(tol=1e-10)
        ctx.cg_solve(b, [kappa], prm)
        holder = {}

        def run():
            holder["st"] = ctx.cg_solve(b, [kappa], prm)[1][0]
        ms = time_events(run, ctx.stream, torch)
        s = holder["st"]
        res[f"kappa{kappa}"] = {"ms": round(ms, 2), "iters": s["iters"], "true_residual": s["true_residual"]}
    log(f"[bench] CG 16^3x32 FP64: {res}")
    ctx.close()
    return res


def bicgstab_vs_cgne(whmc, torch):
    from paper_1805_03560_amd import synth
    U = synth.smooth_links(DIMS, 3005, width=0.8, threads=min(16, os.cpu_count() or 1))
    ctx = whmc.Context(DIMS, device=0)
    ctx.load_gauge(torch.from_numpy(U).to(ctx.device), unitarity_tol=1e-11)
    tune_stencil(ctx, whmc)
    del U
    stream = ctx.stream
    Vh = ctx.Vh
    b = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3006)).to(ctx.device), 0)
    from paper_1805_03560_amd.ensemble import compare_solvers
    try:
        res = compare_solvers(ctx, whmc, torch, b, 0.156)
        log(f"[bench] M_oo x = b: BiCGstab {res['bicgstab']}, CGNE {res['cg_normal_equations']}")
    except whmc.WhmcError as e:
        res = {"error": str(e)}
        log(f"[bench] M_oo x = b: {e}")
    ctx.close()
    return res


def multi_rhs(whmc, torch, stream):
    """24^3 x 48, smooth links (seed 4000): batched hop per rhs and masked multi-RHS CG for 4, 8, 12
    Gaussian sources (seeds 4100 + r) with mass-preconditioning shifts kappa' in
    {0.150, 0.153, 0.156, 0.1575}, against the same systems solved one after the other in FP64."""
    from paper_1805_03560_amd import synth
    dims = (48, 24, 24, 24)
    V = dims[0] * dims[1] * dims[2] * dims[3]
    Vh = V // 2
    U = synth.smooth_links(dims, 4000, threads=min(16, os.cpu_count() or 1))
    ctx = whmc.Context(dims, device=0)
    ctx.load_gauge(torch.from_numpy(U).to(ctx.device), unitarity_tol=1e-11)
    del U
    kp = [0.150, 0.153, 0.156, 0.1575]
    res = {"stencil_schedule": tune_stencil(ctx, whmc)}
    for nrhs in (4, 8, 12):
        import numpy as np
        bs = np.stack([synth.gaussian_spinor(Vh, 4100 + r) for r in range(nrhs)])
        b = ctx.pack_spinor(torch.from_numpy(bs).to(ctx.device), 0)
        kappas = [kp[r % 4] for r in range(nrhs)]
        row = {}
        # batched hop per format (autotuned blocking: rhs per thread x lanes per site)
        for pn, p, links, lb, sb in [("f64", whmc.F64, whmc.L18, 1152, 384), ("f32_l12", whmc.F32, whmc.L12, 384, 192),
                                     ("f16_l12", whmc.F16, whmc.L12, 192, 104)]:
            nb, lanes, order, _ = ctx.autotune(p, links, nrhs)
            bp = b if p == whmc.F64 else ctx.convert_spinor(b, whmc.F64, p, nrhs)
            o = ctx.half_spinor(p, nrhs)
            ms = time_events(lambda: ctx.apply_H_multi(bp, 0, nrhs, prec=p, links=links, out=o, rhs_block=nb,
                                                       rhs_lanes=lanes, rhs_order=order), stream, torch, reps=10)
            row[f"hop_{pn}_blocking"] = [nb, lanes, order]
            row[f"hop_{pn}_us_per_rhs"] = round(ms * 1e3 / nrhs, 2)
            row[f"hop_{pn}_GBps"] = round(Vh * (lb + sb * nrhs) / (ms * 1e-3) / 1e9, 1)
        # CG to 1e-10: sequential FP64, masked multi-RHS FP64, masked multi-RHS mixed FP32-12
        def seq():
            for r in range(nrhs):
                ctx.cg_solve(b[r * 24 * Vh:(r + 1) * 24 * Vh], [kappas[r]], whmc.cg_params(tol=1e-10))
        seq()
        t_seq = time_events(seq, stream, torch)
        ref, _ = ctx.cg_solve(b, kappas, whmc.cg_params(tol=1e-12))
        ref = ref.clone()
        for name, prm in [("multi_fp64", whmc.cg_params(tol=1e-10)),
                          ("multi_fp64_l8", whmc.cg_params(tol=1e-10, links=whmc.L8)),
                          ("multi_mixed_f32_l12", MIXED_F32(whmc)),
                          ("multi_mixed_f32_l8", MIXED_F32(whmc, whmc.L8)),
                          ("multi_mixed_f16_l12", MIXED_F16(whmc))]:
            ctx.cg_solve(b, kappas, prm)
            holder = {}

            def run():
                holder["x"], holder["st"] = ctx.cg_solve(b, kappas, prm)
            t = time_events(run, stream, torch)
            st = holder["st"]
            err = max(float(torch.linalg.vector_norm(holder["x"][r * 24 * Vh:(r + 1) * 24 * Vh] -
                                                     ref[r * 24 * Vh:(r + 1) * 24 * Vh]) /
                            torch.linalg.vector_norm(ref[r * 24 * Vh:(r + 1) * 24 * Vh])) for r in range(nrhs))
            row[name] = {"ms": round(t, 2), "speedup_vs_sequential_fp64": round(t_seq / t, 3),
                         "iters": [s["iters"] for s in st], "max_true_residual": max(s["true_residual"] for s in st),
                         "max_rel_err_vs_fp64_1e-12": err}
        row["sequential_fp64_ms"] = round(t_seq, 2)
        res[f"nrhs{nrhs}"] = row
        log(f"[bench] multi-RHS {nrhs}: hop us/rhs f64 {row['hop_f64_us_per_rhs']} {row['hop_f64_blocking']}, f32 "
            f"{row['hop_f32_l12_us_per_rhs']} {row['hop_f32_l12_blocking']}, f16 {row['hop_f16_l12_us_per_rhs']} "
            f"{row['hop_f16_l12_blocking']}; seq {t_seq:.1f} ms, "
            f"multi fp64 {row['multi_fp64']['ms']} ms (8-real {row['multi_fp64_l8']['ms']} ms), mixed f32 "
            f"{row['multi_mixed_f32_l12']['ms']} ms (8-real {row['multi_mixed_f32_l8']['ms']} ms), "
            f"mixed f16 {row['multi_mixed_f16_l12']['ms']} ms")
    ctx.close()
    return res


def hmc_section(ctx, whmc, torch, stream, Vh):
    """32^3 x 64 HMC (beta = 5.6, kappa = 0.1575, kappa^4 filter with n_t = 15, n_max = 29, Omelyan
    lambda = 1/6, gauge on 4 fine steps per coarse step, tau = 1): one trajectory with mixed FP16
    MD solves, one with the kappa^2 filter (n_t = 7, n_max = 19) and the leapfrog integrator at
    m = 20, Delta H at m = 10 and 20, reversibility, and a central finite difference of the
    total action along a random algebra direction against the force."""
    import math
    from paper_1805_03560_amd import synth
    dims = DIMS
    U0 = ctx.export_gauge()
    pi0 = ctx.pack_algebra(torch.from_numpy(synth.gaussian_momenta(dims, 3100)).to(ctx.device))
    eta = ctx.pack_spinor(torch.from_numpy(synth.gaussian_spinor(Vh, 3101)).to(ctx.device), 0)
    md_mixed = whmc.cg_params(tol=1e-10, prec=whmc.F16, links=whmc.L12, delta=1e-2)
    fp64_tight = whmc.cg_params(tol=1e-12)
    mk = lambda m, md: whmc.hmc_params(beta=5.6, kappa=KAPPA, k=2, n_t=15, n_max=29, integrator=whmc.OMELYAN,
                                       lam=1.0 / 6.0, m=m, m0=4, tau=1.0, md_solver=md, action_solver=fp64_tight)
    out = {}
    t0 = time.perf_counter()
    res = ctx.hmc_trajectory(mk(10, md_mixed), pi0, eta, 0.5)
    out["trajectory_m10"] = {"seconds": round(time.perf_counter() - t0, 3), "dH": res["dH"],
                             "accepted": res["accepted"], "plaquette": res["plaquette"],
                             "cg_iters": res["cg_iters"], "n_solves": res["n_solves"]}
    log(f"[bench] HMC 32^3x64 trajectory: {out['trajectory_m10']}")
    # the kappa^2 filter (n_t = 7, n_max = 19) with the leapfrog integrator, m = 20 coarse steps
    ctx.load_gauge(U0, unitarity_tol=0.0)
    p2 = whmc.hmc_params(beta=5.6, kappa=KAPPA, k=1, n_t=7, n_max=19, integrator=whmc.LEAPFROG, lam=0.0, m=20, m0=4,
                         tau=1.0, md_solver=md_mixed, action_solver=fp64_tight)
    t0 = time.perf_counter()
    res = ctx.hmc_trajectory(p2, pi0, eta, 0.5)
    out["trajectory_leapfrog_kappa2_m20"] = {
        "seconds": round(time.perf_counter() - t0, 3), "dH": res["dH"], "accepted": res["accepted"],
        "plaquette": res["plaquette"], "cg_iters": res["cg_iters"], "n_solves": res["n_solves"],
        "note": "timing of one trajectory's kernels; the smooth synthetic field (plaquette 0.79) is far from the "
                "beta = 5.6 equilibrium (about 0.57) and its gauge force is large, which the second-order leapfrog "
                "at m = 20 integrates poorly, so |dH| is large; the paper's 12^3x24 leapfrog runs at equilibrium "
                "are reproduced by the ensemble runs"}
    log(f"[bench] HMC 32^3x64 leapfrog kappa^2 trajectory: {out['trajectory_leapfrog_kappa2_m20']}")
    ctx.load_gauge(U0, unitarity_tol=0.0)
    phi = ctx.heatbath_phi(eta, 2, 15, 29, KAPPA)
    dh = {}
    for m in (10, 20):
        ctx.load_gauge(U0, unitarity_tol=0.0)
        p = mk(m, md_mixed)
        pi = pi0.clone()
        H0 = ctx.hamiltonian(p, pi, phi)
        ctx.md_integrate(p, pi, phi)
        dh[m] = ctx.hamiltonian(p, pi, phi) - H0
        if m == 10:
            ctx.md_integrate(p, -pi, phi)
            U2 = ctx.export_gauge()
            d = (U2 - U0).abs()
            out["reversibility_mixed_1e-10"] = {"max_abs_dU": float(d.max()), "Delta": float((d * d).sum())}
    out["dH"] = {"m10": dh[10], "m20": dh[20], "ratio": dh[10] / dh[20] if dh[20] != 0 else None}
    # reversibility with FP64 solves to 1e-12
    ctx.load_gauge(U0, unitarity_tol=0.0)
    p = mk(10, fp64_tight)
    pi = pi0.clone()
    ctx.md_integrate(p, pi, phi)
    ctx.md_integrate(p, -pi, phi)
    d = (ctx.export_gauge() - U0).abs()
    out["reversibility_fp64_1e-12"] = {"max_abs_dU": float(d.max()), "Delta": float((d * d).sum())}
    log(f"[bench] HMC dH {out['dH']}, reversibility {out['reversibility_mixed_1e-10']} / {out['reversibility_fp64_1e-12']}")
    # finite difference of S_G + S~_PF along a random direction vs (omega, F)
    ctx.load_gauge(U0, unitarity_tol=0.0)
    tight = whmc.cg_params(tol=1e-14, maxiter=20000)
    F = ctx.force(phi, 2, 29, 29, KAPPA, 5.6, flags=whmc.FORCE_PF | whmc.FORCE_GAUGE, solver=tight)
    omega = ctx.pack_algebra(torch.from_numpy(synth.random_algebra(dims, 3102)).to(ctx.device))
    dd = float(torch.dot(omega, F))
    def S(e):
        ctx.load_gauge(U0, unitarity_tol=0.0)
        ctx.update_links(omega, e)
        sg, spf = ctx.action(phi, 2, 29, 29, KAPPA, 5.6, solver=tight)
        return sg + spf
    eps = 1e-3
    fd = (8 * (S(eps) - S(-eps)) - (S(2 * eps) - S(-2 * eps))) / (12 * eps)
    out["force_fd_check"] = {"directional_derivative": dd, "finite_difference": fd,
                             "rel_err": abs(dd - fd) / abs(fd), "eps": eps, "solver_tol": 1e-14}
    log(f"[bench] force FD check: {out['force_fd_check']}")
    ctx.load_gauge(U0, unitarity_tol=0.0)
    return out


def widened_16x32(whmc, torch):
    """The rooted-polynomial action (Sec. 2.1) and mass preconditioning with the filter (Sec. 1, 5)
    on the paper's rooted-polynomial workload, 16^3 x 32 at kappa = 0.1575, here on a synthetic
    smooth field (width 0.55, seed 3200): heat bath, action and per-term force times, and one
    multi-level leapfrog / Omelyan trajectory with tau = sqrt(2) (MD solves FP64 to 1e-10, actions
    to 1e-12).  Rooted: N = 4, n = (8, 32), n_t = 160, n_max = 400, m_0, m_1, m_2 = 6, 5, 4, m = 5
    (Table RunPoly1).  Mass preconditioning: kappa_1 = 0.14, the kappa^4 filter (n_t = 15,
    n_max = 29) on the heavy factor and on the ratio."""
    import numpy as np
    from paper_1805_03560_amd import synth
    dims = (32, 16, 16, 16)
    kappa = 0.1575
    U = synth.smooth_links(dims, 3200, width=0.55)
    ctx = whmc.Context(dims, device=0)
    ctx.load_gauge(torch.from_numpy(U).to(ctx.device), unitarity_tol=1e-11)
    tune_stencil(ctx, whmc)
    U0 = ctx.export_gauge()
    stream = ctx.stream
    Vh = ctx.Vh
    md = whmc.cg_params(tol=1e-10)
    act = whmc.cg_params(tol=1e-12)
    pi0 = ctx.pack_algebra(torch.from_numpy(synth.gaussian_momenta(dims, 3201)).to(ctx.device))
    out = {}

    r = whmc.rooted(4, (8, 32), k=0, n_t=160, n_max=400)
    nf = r.jmax * r.N + 1
    eta = ctx.pack_spinor(torch.from_numpy(np.stack([synth.gaussian_spinor(Vh, 3210 + f) for f in range(nf)]))
                          .to(ctx.device), 0)
    res = {}
    t0 = time.perf_counter()
    phi, it = ctx.rooted_heatbath(eta, r, kappa, solver=act)
    torch.cuda.synchronize()
    res["heatbath"] = {"seconds": round(time.perf_counter() - t0, 3), "poly_cg_iters": it}
    t0 = time.perf_counter()
    res["action"] = {"S": ctx.rooted_action(phi, r, kappa, solver=act), "seconds": round(time.perf_counter() - t0, 3)}
    F = ctx.algebra()
    for term, name in [(1, "force_W1_deg8_x4"), (2, "force_W2_deg32_x4"), (3, "force_remainder_nt160")]:
        ctx.rooted_force(phi, r, kappa, term=term, solver=md, out=F)
        res[name + "_ms"] = round(time_events(lambda: ctx.rooted_force(phi, r, kappa, term=term, solver=md, out=F),
                                              stream, torch), 2)
    p = whmc.rooted_hmc_params(beta=5.6, kappa=kappa, rooted_action=r, integrator=whmc.LEAPFROG, m=5, msub=(6, 5, 4),
                               md_solver=md, action_solver=act, heatbath_solver=act)
    t0 = time.perf_counter()
    tr = ctx.rooted_trajectory(p, pi0, eta, 0.5)
    res["trajectory"] = {"seconds": round(time.perf_counter() - t0, 3), "dH": tr["dH"], "cg_iters": tr["cg_iters"],
                         "n_solves": tr["n_solves"], "poly_iters": tr["poly_iters"],
                         "note": "timing of one trajectory's kernels; the synthetic field is far from equilibrium of "
                                 "the beta = 5.6 rooted action, so |dH| is large (on thermalised fields the same "
                                 "settings give P_acc = 0.77, see the ensemble runs)"}
    out["rooted_16x32_kappa0.1575"] = res
    log(f"[bench] rooted N=4 (8,32) 16^3x32: {res}")

    ctx.load_gauge(U0, unitarity_tol=0.0)
    mp = whmc.masspre((0.14,), k=2, n_t=15, n_max=29)
    eta2 = eta[: 2 * 24 * Vh]
    res = {}
    phi = ctx.masspre_heatbath(eta2, mp, kappa, solver=act)
    for term, name in [(1, "force_heavy_kappa0.14_filtered"), (2, "force_ratio_filtered")]:
        ctx.masspre_force(phi, mp, kappa, term=term, solver=md, out=F)
        res[name + "_ms"] = round(time_events(lambda: ctx.masspre_force(phi, mp, kappa, term=term, solver=md, out=F),
                                              stream, torch), 2)
    p = whmc.masspre_hmc_params(beta=5.6, kappa=kappa, mp=mp, integrator=whmc.OMELYAN, m=5, msub=(4, 2),
                                md_solver=md, action_solver=act)
    t0 = time.perf_counter()
    tr = ctx.masspre_trajectory(p, pi0, eta2, 0.5)
    res["trajectory"] = {"seconds": round(time.perf_counter() - t0, 3), "dH": tr["dH"], "cg_iters": tr["cg_iters"],
                         "n_solves": tr["n_solves"]}
    out["masspre_16x32_kappa0.1575"] = res
    log(f"[bench] mass preconditioning 16^3x32: {res}")
    ctx.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(gpu_iters_16x32=None):
    """The FP64 numpy oracle as it stands, timed on this host on bounded samples (its numpy kernels
    run on one thread):
    - H_eo on 16^3 x 32 -- the oracle forms the even/odd block by applying the full-lattice H to a
      field that is zero on the other parity, twice the arithmetic of an even/odd hop; `value` is
      the even/odd hop's algorithmic bytes (1536 B per output site) per second of that;
    - its even/odd CG to a residual of 1e-10 on 4^4 (Haar links, seed 1000, kappa = 0.156), whole;
    - M_oo^dag M_oo on 16^3 x 32 (one CG iteration's operator), times the iteration count of the
      GPU's 16^3 x 32 solve at kappa = 0.156: an extrapolated oracle CG time, labelled as such."""
    import numpy as np

    from oracle import dirac
    from oracle.lattice import Lattice
    from oracle.solve import cg
    from paper_1805_03560_amd import synth
    dims = (32, 16, 16, 16)
    lat = Lattice(dims)
    U = synth.smooth_links(dims, 2000)
    x = synth.gaussian_spinor(lat.Vh, 2001)
    dirac.apply_Hblock(lat, U, x, 0)
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while t < 8.0 and reps < 50:
        dirac.apply_Hblock(lat, U, x, 0)
        reps += 1
        t = time.perf_counter() - t0
    gbs = 1536 * lat.Vh * reps / t / 1e9
    log(f"[bench] oracle H_eo 16^3x32: {t / reps:.2f} s/hop, {gbs:.3f} GB/s")
    # whole CG on 4^4
    d4 = (4, 4, 4, 4)
    l4 = Lattice(d4)
    U4 = synth.haar_links(d4, 1000)
    b4 = synth.gaussian_spinor(l4.Vh, 0)
    t0 = time.perf_counter()
    _, it4, res4 = cg(lambda v: dirac.apply_MooDagMoo(l4, U4, v, 0.156), b4, tol=1e-10)
    t4 = time.perf_counter() - t0
    # operator of one CG iteration on 16^3 x 32
    t0 = time.perf_counter()
    for _ in range(2):
        dirac.apply_MooDagMoo(lat, U, x, 0.156)
    t_op = (time.perf_counter() - t0) / 2
    cg16 = {"seconds_per_iteration": round(t_op, 3)}
    if gpu_iters_16x32:
        cg16["iterations_of_the_gpu_solve"] = gpu_iters_16x32
        cg16["extrapolated_seconds"] = round(t_op * gpu_iters_16x32, 1)
    log(f"[bench] oracle CG 4^4: {it4} iters in {t4:.2f} s; 16^3x32 M^dag M: {t_op:.2f} s")
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} oracle H_eo applications on 16^3x32 (Vh={lat.Vh}, computed as a full-lattice H on "
                      f"a half-zero field), {t / reps:.2f} s each, one thread",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "cg_4x4_kappa0.156_to_1e-10": {"seconds": round(t4, 3), "iterations": it4, "true_residual": res4},
            "cg_16x32_kappa0.156_to_1e-10_extrapolated": cg16}


if __name__ == "__main__":
    main()
