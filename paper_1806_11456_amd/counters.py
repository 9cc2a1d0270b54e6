"""HBM traffic from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE), and kernel statistics.

Per launch of one kernel (--kernel), or per fine-level residual of profile_residual.py (--residual R: the
dispatches of the last R residuals, delimited by the divergence kernel that ends each of them); the
statistics mode (--stats DIR) prints a per-kernel table of a --kernel-trace run.

Each counter is scaled by what it reads for a plain device copy of known size run in the same process (the
largest copy dispatch): a copy of B bytes reads B and writes B.  The result is written as JSON (read by
bench.py, which reports it only while the kernel sources still hash to the recorded value) and as a short
Markdown summary.

    python -m paper_1806_11456_amd.counters --fetch DIR --write DIR --residual 10 --alg-bytes B \\
        --out profiles/residual_plate64x32_counters.json --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


RESIDUAL_SOURCES = ("device.h", "kernels_elem.inc", "kernels_face.inc")


def source_hash() -> str:
    """SHA-256 over the device sources of the residual's kernels (element and face kernels and their device
    helpers): what the counted traffic depends on.  Setup, transfer and reduction kernels and the host
    library (launch sizes, drivers) are not hashed."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        base = os.path.basename(path)
        if base not in RESIDUAL_SOURCES:
            continue
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode())
            h.update(f.read())
    return h.hexdigest()


def _rows(path: str):
    if os.path.isdir(path):
        found = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
        if not found:
            raise SystemExit(f"no counter_collection.csv under {path}")
        path = found[0]
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _per_kernel(rows, kernel):
    vals = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].split("(")[0].split("<")[0].replace("void ", "").strip() == kernel]
    copies = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no dispatches of {kernel}")
    if not copies:
        raise SystemExit("no copy dispatch for the calibration")
    return sum(vals) / len(vals), len(vals), max(copies)[1]


RESIDUAL_KERNELS = ("k_trace", "k_face1", "k_grad", "k_face2c", "k_face2", "k_div")


def _base(name: str) -> str:
    return name.split("(")[0].split("<")[0].replace("void ", "").strip()


def _last_residuals(rows, R):
    """Rows of the dispatches of the last R fine-level residuals.  Each residual ends with its divergence
    launches (one per launch class of the level's tiles, back to back)."""
    key = (lambda r: int(r["Dispatch_Id"])) if rows and "Dispatch_Id" in rows[0] else None
    order = sorted(range(len(rows)), key=(lambda i: key(rows[i])) if key else (lambda i: i))
    is_div = [_base(rows[i]["Kernel_Name"]) == "k_div" for i in order]
    ends = [p for p in range(len(order)) if is_div[p] and (p + 1 == len(order) or not is_div[p + 1])]
    if len(ends) < R + 1:
        raise SystemExit(f"fewer than {R + 1} residuals")
    start = ends[-R - 1] + 1
    return [rows[i] for i in order[start:] if _base(rows[i]["Kernel_Name"]) in RESIDUAL_KERNELS]


def residual_traffic(fetch_dir, write_dir, R, copy_mib, out_path, command, alg_bytes):
    fr, wr = _rows(fetch_dir), _rows(write_dir)
    f_copy = max((int(r["Grid_Size"]), float(r["Counter_Value"])) for r in fr if "copyBuffer" in r["Kernel_Name"])[1]
    w_copy = max((int(r["Grid_Size"]), float(r["Counter_Value"])) for r in wr if "copyBuffer" in r["Kernel_Name"])[1]
    copy_kib = copy_mib * 1024.0
    fs, ws = copy_kib / f_copy, copy_kib / w_copy
    per = {}
    for rows, scale, col in ((_last_residuals(fr, R), fs, "fetch"), (_last_residuals(wr, R), ws, "write")):
        for r in rows:
            k = _base(r["Kernel_Name"])
            per.setdefault(k, {"fetch": 0.0, "write": 0.0})
            per[k][col] += float(r["Counter_Value"]) * scale * 1024.0 / R
    total = sum(v["fetch"] + v["write"] for v in per.values())
    out = {"residuals": R, "traffic_bytes_per_residual": total, "per_kernel_bytes": per, "fetch_scale": fs,
           "write_scale": ws, "alg_bytes_per_residual": alg_bytes, "traffic_over_alg": total / alg_bytes,
           "source_sha256": source_hash(), "command": command}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    md = os.path.splitext(out_path)[0] + ".md"
    with open(md, "w") as f:
        f.write("# HBM traffic of one fine-level residual R(u) (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n\n")
        f.write(f"Commands (repository root, on one MI355X):\n\n    {command}\n\n")
        f.write(f"Calibration: a plain device copy of {copy_mib} MiB reads FETCH_SIZE = {f_copy:.0f} KiB and "
                f"WRITE_SIZE = {w_copy:.0f} KiB; scale factors {fs:.3f} (fetch) and {ws:.3f} (write).  The last "
                f"{R} residuals of the run are counted.\n\n")
        f.write("| kernel | fetch MB | write MB |\n|---|---|---|\n")
        for k, v in per.items():
            f.write(f"| {k} | {v['fetch'] / 1e6:.2f} | {v['write'] / 1e6:.2f} |\n")
        f.write(f"\nTotal {total / 1e6:.2f} MB per residual against the surveyed algorithmic {alg_bytes / 1e6:.2f} MB "
                f"(160 B per node + 160 B per element face node): {total / alg_bytes:.2f} x.\n")
    print(json.dumps(out))


def sq_summary(dirs, R, title, command, alg_flops):
    """Per-kernel instruction and stall counters (SQ block) of the last R residuals of profile_residual.py runs,
    one directory per counter pass: waves, the fraction of wave time spent waiting and issuing VALU / LDS work,
    instructions per wave and FP64 VALU flops (the SQ_INSTS_VALU_FLOPS_FP64 count times the 64 lanes of a wave)."""
    agg = {}
    for d in dirs:
        for r in _last_residuals(_rows(d), R):
            k = _base(r["Kernel_Name"])
            agg.setdefault(k, {})
            agg[k][r["Counter_Name"]] = agg[k].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"]) / R
    g = lambda k, c: agg[k].get(c, 0.0)
    lines = [f"# SQ counters per fine-level residual: {title}", "",
             "Commands (repository root, TMPDIR=/tmp, one MI355X; two counter passes):", "", f"    {command}", "",
             "| kernel | waves | wait / wave time | VALU / wave time | LDS / wave time | VALU instr / wave | "
             "LDS instr / wave | VMEM rd / wave | FP64 VALU GFLOP | MFMA F64 instr |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    tot_fl = 0.0
    for k in sorted(agg, key=lambda k: -g(k, "SQ_WAVE_CYCLES")):
        if k not in RESIDUAL_KERNELS:
            continue
        w, wc = g(k, "SQ_WAVES"), g(k, "SQ_WAVE_CYCLES")
        fl = 64.0 * g(k, "SQ_INSTS_VALU_FLOPS_FP64")
        tot_fl += fl
        frac = lambda c: g(k, c) / wc if wc else 0.0
        per = lambda c: g(k, c) / w if w else 0.0
        lines.append(f"| {k} | {w:.0f} | {frac('SQ_WAIT_ANY'):.2f} | {frac('SQ_ACTIVE_INST_VALU'):.2f} | "
                     f"{frac('SQ_ACTIVE_INST_LDS'):.2f} | {per('SQ_INSTS_VALU'):.0f} | {per('SQ_INSTS_LDS'):.0f} | "
                     f"{per('SQ_INSTS_VMEM_RD'):.0f} | {fl / 1e9:.3f} | {g(k, 'SQ_INSTS_VALU_MFMA_F64'):.0f} |")
    lines += ["", f"FP64 VALU flops per residual as counted {tot_fl / 1e9:.3f} GFLOP (counter x 64: every lane of each "
                  f"FP64 VALU instruction, masked lanes included, an upper bound) against the surveyed model's "
                  f"{alg_flops / 1e9:.3f} GFLOP.  Counts are summed over the shader engines the profiler read; other "
                  "runs of the same command have read a subset of them (1/5 to 1/10 of the waves), so absolute counts "
                  "are not compared across runs; the ratios within a kernel (time waiting, VALU and LDS issue, "
                  "instructions per wave) are.  No FP64 MFMA instruction runs: the contractions use the FP64 vector "
                  "units, which issue in a small fraction of the wave time, so matrix cores would not shorten them."]
    return "\n".join(lines) + "\n"


def kernel_stats(path, title, command):
    """Per-kernel table (calls, total, average, share) of a --kernel-trace run: the CSV statistics when
    present, else the dispatch table of the rocpd database."""
    rows = []
    found = glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)
    if found:
        with open(found[0], newline="") as f:
            for r in csv.DictReader(f):
                rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"])))
    else:
        import sqlite3
        db = glob.glob(os.path.join(path, "**", "*results.db"), recursive=True)[0]
        con = sqlite3.connect(db)
        for name, n, tot in con.execute("select name, count(*), sum(end - start) from kernels group by name"):
            rows.append((name, int(n), float(tot)))
    tot = sum(r[2] for r in rows)
    rows.sort(key=lambda r: -r[2])
    lines = [f"# rocprofv3 kernel statistics: {title}", "#", "# command (repository root, TMPDIR=/tmp, one MI355X):",
             f"#   {command}", "#",
             f"{'kernel':58s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}"]
    for name, n, t in rows[:30]:
        nm = name.replace("void ", "").split("(")[0][:58]
        lines.append(f"{nm:58s} {n:7d} {t / 1e6:10.3f} {t / n / 1e3:10.2f} {100 * t / tot:6.2f}")
    lines.append(f"{'all kernels':58s} {sum(r[1] for r in rows):7d} {tot / 1e6:10.3f}")
    return "\n".join(lines) + "\n"


def step_breakdown(path: str, marker: str, title: str, command: str) -> str:
    """One solver step from a --kernel-trace run: in the run's longest stretch of GPU work with at least three
    dispatches of 'marker', the dispatches
    between the last two dispatches of 'marker' before the final one (a kernel launched once per step, e.g. the
    restriction out of the finest level), summed per kernel and launch size (workgroups), so that each level
    of the hierarchy shows as its own rows."""
    found = glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True)
    if not found:
        raise SystemExit(f"no kernel_trace.csv under {path}")
    rows = []
    with open(found[0], newline="") as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"],
                         int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))))
    rows.sort()
    # the run's longest stretch of GPU work (dispatches closer than 20 ms apart): the workload of interest when
    # several run one after another
    segs, cur = [], [rows[0]]
    for r in rows[1:]:
        if r[0] - cur[-1][1] > 20_000_000:
            segs.append(cur)
            cur = [r]
        else:
            cur.append(r)
    segs.append(cur)
    is_mark = lambda r: r[2].replace("void ", "").startswith(marker)
    segs = [sg for sg in segs if sum(1 for r in sg if is_mark(r)) >= 3] or segs
    rows = max(segs, key=lambda sg: sum(t1 - t0 for t0, t1, _, _ in sg))
    marks = [i for i, r in enumerate(rows) if is_mark(r)]
    if len(marks) < 3:
        raise SystemExit(f"fewer than 3 dispatches of {marker}")
    a, b = marks[-3], marks[-2]
    step = rows[a:b]
    agg = {}
    for t0, t1, name, wg in step:
        key = (name.replace("void ", "").split("(")[0], wg)
        n, t = agg.get(key, (0, 0.0))
        agg[key] = (n + 1, t + (t1 - t0) * 1e-6)
    busy = sum(v[1] for v in agg.values())
    span = (step[-1][1] - step[0][0]) * 1e-6
    lines = [f"# One solver step by kernel and launch size: {title}", "", "Command (repository root, TMPDIR=/tmp, "
             "one MI355X):", "", f"    {command}", "",
             f"The dispatches from one '{marker}' launch to the next (one step), {len(step)} dispatches, "
             f"{busy:.1f} ms of kernel time in a {span:.1f} ms span.  Launch sizes tell the levels apart "
             "(element-tile kernels: one workgroup per tile; face kernels: one per face tile).", "",
             "| kernel | workgroups | launches | ms | us per launch |", "|---|---|---|---|---|"]
    for (name, wg), (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        if t < 0.05 * busy / 100:
            continue
        lines.append(f"| {name} | {wg} | {n} | {t:.2f} | {1e3 * t / n:.1f} |")
    return "\n".join(lines) + "\n"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", default=None, help="summarise a --kernel-trace output directory")
    ap.add_argument("--step", default=None, help="one solver step of a --kernel-trace output directory")
    ap.add_argument("--marker", default="k_transfer<double, float, 10>", help="--step: a kernel launched once per step")
    ap.add_argument("--sq", nargs="+", default=None, help="SQ counter pass directories to summarise per residual")
    ap.add_argument("--alg-flops", type=float, default=0.0)
    ap.add_argument("--title", default="")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel")
    ap.add_argument("--residual", type=int, default=0, help="per residual: the last R residuals of the run")
    ap.add_argument("--alg-bytes", type=float, default=0.0)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--alg-json", default=None,
                    help="JSON with the compulsory bytes per launch of the same launches ({kind: {...}})")
    ap.add_argument("--kind", default=None, help="kernel kind in that JSON (div, grad, ...)")
    args = ap.parse_args()
    if args.sq:
        txt = sq_summary(args.sq, args.residual or 10, args.title, args.command, args.alg_flops)
        with open(args.out, "w") as f:
            f.write(txt)
        print(txt)
        return 0
    if args.step:
        txt = step_breakdown(args.step, args.marker, args.title, args.command)
        with open(args.out, "w") as f:
            f.write(txt)
        print(txt)
        return 0
    if args.stats:
        txt = kernel_stats(args.stats, args.title, args.command)
        with open(args.out, "w") as f:
            f.write(txt)
        print(txt)
        return 0
    if args.residual:
        residual_traffic(args.fetch, args.write, args.residual, args.copy_mib, args.out, args.command, args.alg_bytes)
        return 0
    f_avg, n, f_copy = _per_kernel(_rows(args.fetch), args.kernel)
    w_avg, n2, w_copy = _per_kernel(_rows(args.write), args.kernel)
    copy_kib = args.copy_mib * 1024.0
    fs, ws = copy_kib / f_copy, copy_kib / w_copy
    traffic = (f_avg * fs + w_avg * ws) * 1024.0
    out = {"kernel": args.kernel, "dispatches": n, "fetch_kib_avg": f_avg, "write_kib_avg": w_avg,
           "fetch_scale": fs, "write_scale": ws, "traffic_bytes_per_launch": traffic,
           "source_sha256": source_hash(), "command": args.command}
    if args.alg_json:
        with open(args.alg_json) as f:
            lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
        alg = json.loads(lines[0])[args.kind]
        out["alg_bytes_per_launch"] = alg["alg_bytes_per_launch"]
        out["alg_launches"] = alg["launches"]
        out["traffic_over_alg"] = traffic / alg["alg_bytes_per_launch"]
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    md = os.path.splitext(args.out)[0] + ".md"
    with open(md, "w") as f:
        f.write(f"# HBM traffic of {args.kernel} (rocprofv3 FETCH_SIZE / WRITE_SIZE)\n\n")
        f.write(f"Command (repository root, on one MI355X):\n\n    {args.command}\n\n")
        f.write(f"Calibration: a plain device copy of {args.copy_mib} MiB reads FETCH_SIZE = {f_copy:.0f} KiB and "
                f"WRITE_SIZE = {w_copy:.0f} KiB; scale factors {fs:.3f} (fetch) and {ws:.3f} (write).\n\n")
        f.write(f"{args.kernel}: {n} dispatches, average FETCH_SIZE {f_avg:.1f} KiB, WRITE_SIZE {w_avg:.1f} KiB; "
                f"HBM traffic per launch {traffic / 1e6:.2f} MB.\n")
        if "traffic_over_alg" in out:
            f.write(f"Compulsory bytes of the same launches (the library's accounting): "
                    f"{out['alg_bytes_per_launch'] / 1e6:.2f} MB per launch ({out['alg_launches']} launches); "
                    f"measured / compulsory = {out['traffic_over_alg']:.3f}.\n")
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
