"""Summaries of rocprofv3 result databases (the rocpd SQLite files of `rocprofv3 -d DIR -o NAME`).

    python -m paper_1805_03560_amd.profsum trace DB [--top N] [--match TEXT]
        markdown table of the kernels of a `--kernel-trace` run: calls, average / min / max launch
        duration, total time, share, registers.
    python -m paper_1805_03560_amd.profsum counters DB [--match TEXT] [--lds BYTES]
        per-dispatch values of every counter of a `--pmc` run (summed over the counter's instances).
    python -m paper_1805_03560_amd.profsum traffic --kernel TEXT --fetch DB --write DB --copy-fetch DB \\
            --copy-write DB --copy-bytes N [--trace DB] [--algorithmic BYTES] [--workload TEXT] [--json OUT] \\
            [--lds BYTES] [--last N] [--trace-last N]
        HBM bytes per launch of one kernel from a FETCH_SIZE and a WRITE_SIZE pass, each scaled by what
        the same counter reads for a device copy of N bytes (FETCH_SIZE counts the 128-byte read requests
        of gfx950 as 64 bytes, so its scale is 2).  --json writes the record bench.py reports as
        roofline.traffic, stamped with the digest of the stencil sources it was measured on.
"""
import argparse
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DIGEST_SOURCES = ("device.h", "stencil.h", "core.hip")


def source_digest():
    """digest of the sources the single-RHS hop kernel is built from"""
    h = hashlib.sha256()
    for f in DIGEST_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(db, table):
    con = sqlite3.connect(db)
    try:
        cols = [r[1] for r in con.execute(f"pragma table_info({table})")]
        return [dict(zip(cols, r)) for r in con.execute(f"select * from {table}").fetchall()]
    finally:
        con.close()


def kernels(db, lds=None):
    """[(name, duration_us, vgpr, agpr, lds bytes)] of every dispatch in a kernel-trace database (only
    those with that LDS allocation if lds is given)"""
    out = []
    for d in _rows(db, "kernels"):
        sz = d.get("lds_size", 0) or 0
        if lds is None or sz == lds:
            out.append((d["name"], (d["end"] - d["start"]) / 1e3, d["vgpr_count"], d["accum_vgpr_count"], sz))
    return out


def counters(db, lds=None):
    """{kernel name: [{counter: value} per dispatch]} of a --pmc database, instances summed (only the
    dispatches with that LDS allocation if lds is given)"""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for d in _rows(db, "counters_collection"):
        if lds is not None and (d.get("lds_block_size", 0) or 0) != lds:
            continue
        per[d["dispatch_id"]][d["counter_name"]] += d["value"]
        names[d["dispatch_id"]] = d["kernel_name"]
    out = collections.defaultdict(list)
    for disp in sorted(per):
        out[names[disp]].append(dict(per[disp]))
    return out


def _short(name, width=110):
    return name if len(name) <= width else name[:width - 3] + "..."


def trace_table(db, top=25, match=None):
    """kernels grouped by name and LDS allocation (a launch-time LDS reservation caps occupancy)"""
    agg = collections.defaultdict(list)
    regs = {}
    for name, us, v, a, sz in kernels(db):
        if match and match not in name:
            continue
        agg[(name, sz)].append(us)
        regs[(name, sz)] = (v, a)
    total = sum(sum(v) for v in agg.values()) or 1.0
    lines = ["| kernel | LDS B | calls | avg us | min us | max us | total ms | share | VGPR / AGPR |",
             "|---|---|---|---|---|---|---|---|---|"]
    for key, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"| `{_short(key[0])}` | {key[1]} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | "
                     f"{max(v):.1f} | {sum(v) / 1e3:.2f} | {100 * sum(v) / total:.1f}% | {regs[key][0]} / {regs[key][1]} |")
    lines.append("")
    lines.append("(VGPR / AGPR: rocprofv3's vgpr_count / accum_vgpr_count; on gfx950 vgpr_count is half the registers "
                 "allocated per lane, architectural and accumulation together, so the compiler's resource report "
                 "gives about twice it.)")
    return "\n".join(lines)


def _one(db, counter, match, lds=None, last=None):
    """average of a counter over the dispatches of the kernels matching `match` (the last `last` of
    them in dispatch order if given: a benchmark's timed launches follow its tuning launches)"""
    per = collections.defaultdict(float)
    for d in _rows(db, "counters_collection"):
        if d["counter_name"] != counter or match not in d["kernel_name"]:
            continue
        if lds is not None and (d.get("lds_block_size", 0) or 0) != lds:
            continue
        per[d["dispatch_id"]] += d["value"]
    vals = [per[k] for k in sorted(per)]
    if last:
        vals = vals[-last:]
    if not vals:
        raise SystemExit(f"{db}: no {counter} values for a kernel matching {match!r}")
    return sum(vals) / len(vals), len(vals)


def _copy_kernel(db):
    for name in counters(db):
        if "copyBuffer" in name or "copy" in name.lower():
            return name
    raise SystemExit(f"{db}: no copy kernel")


def traffic(a):
    ck_f, ck_w = _copy_kernel(a.copy_fetch), _copy_kernel(a.copy_write)
    copy_f = max(c["FETCH_SIZE"] for c in counters(a.copy_fetch)[ck_f])
    copy_w = max(c["WRITE_SIZE"] for c in counters(a.copy_write)[ck_w])
    fs = a.copy_bytes / (copy_f * 1024.0)
    ws = a.copy_bytes / (copy_w * 1024.0)
    lds = getattr(a, "lds", None)
    last = getattr(a, "last", None)
    f_kib, nf = _one(a.fetch, "FETCH_SIZE", a.kernel, lds, last)
    w_kib, nw = _one(a.write, "WRITE_SIZE", a.kernel, lds, last)
    rd, wr = f_kib * 1024.0 * fs, w_kib * 1024.0 * ws
    rec = {"kernel": next(n for n in counters(a.fetch) if a.kernel in n), "workload": a.workload,
           "fetch_kib": round(f_kib, 2), "write_kib": round(w_kib, 2), "dispatches": [nf, nw],
           "fetch_scale": fs, "write_scale": ws, "bytes_per_launch": int(round(rd + wr))}
    lines = [f"- calibration: a device copy of {a.copy_bytes} bytes reads FETCH_SIZE = {copy_f:.0f} KiB and "
             f"WRITE_SIZE = {copy_w:.0f} KiB per dispatch: scale factors {fs:.3f} (fetch) and {ws:.3f} (write)",
             f"- kernel (average over {nf} / {nw} dispatches): FETCH_SIZE {f_kib:.0f} KiB, WRITE_SIZE {w_kib:.0f} KiB "
             f"-> {rd / 1e9:.3f} GB read + {wr / 1e9:.3f} GB written = {(rd + wr) / 1e9:.3f} GB per launch"]
    if a.algorithmic:
        lines.append(f"- algorithmic bytes per launch {a.algorithmic / 1e9:.3f} GB; measured / algorithmic = "
                     f"{(rd + wr) / a.algorithmic:.3f}")
        rec["algorithmic_bytes"] = int(a.algorithmic)
    if lds is not None:
        rec["lds_bytes"] = lds
    if a.trace:
        durs = [us for name, us, _, _, _ in kernels(a.trace, lds) if a.kernel in name]
        if durs and getattr(a, "trace_last", None):
            durs = durs[-a.trace_last:]
        if durs:
            avg = sum(durs) / len(durs)
            rec["avg_launch_us"] = round(avg, 3)
            lines.append(f"- average launch {avg:.1f} us over {len(durs)} launches -> "
                         f"{(rd + wr) / (avg * 1e-6) / 1e9:.0f} GB/s counted" +
                         (f", {a.algorithmic / (avg * 1e-6) / 1e9:.0f} GB/s algorithmic" if a.algorithmic else ""))
    if a.json:
        rec["source_digest"] = source_digest()
        with open(a.json, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=25)
    t.add_argument("--match")
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--match")
    c.add_argument("--lds", type=int)
    f = sub.add_parser("traffic")
    for k in ("kernel", "fetch", "write", "copy_fetch", "copy_write"):
        f.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--trace")
    f.add_argument("--algorithmic", type=float)
    f.add_argument("--workload", default="")
    f.add_argument("--json")
    f.add_argument("--lds", type=int, help="only dispatches with this LDS allocation (bytes)")
    f.add_argument("--last", type=int, help="only the last N matching dispatches of each counter pass")
    f.add_argument("--trace-last", type=int, help="only the last N matching launches of the trace")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(a.db, a.top, a.match))
    elif a.cmd == "counters":
        for name, lst in counters(a.db, a.lds).items():
            if a.match and a.match not in name:
                continue
            print(f"{_short(name)}: {len(lst)} dispatches")
            for d in lst:
                print("   " + ", ".join(f"{k} {v:.0f}" for k, v in sorted(d.items())))
    else:
        print(traffic(a))
    return 0


if __name__ == "__main__":
    sys.exit(main())
