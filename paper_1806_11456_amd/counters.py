"""HBM traffic per launch of one kernel from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE).

Each counter is scaled by what it reads for a plain device copy of known size run in the same process (the
largest copy dispatch): a copy of B bytes reads B and writes B.  The result is written as JSON (read by
bench.py, which reports it only while the kernel sources still hash to the recorded value) and as a short
Markdown summary.

    python -m paper_1806_11456_amd.counters --fetch DIR --write DIR --kernel k_div --copy-mib 1024 \\
        --out profiles/k_div_plate64x32_N661_counters.json --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


# host-only parts of the library that define and launch no kernel of the timed step (adaptation and the
# wall-force diagnostic): editing them does not change what the counters measured
HOST_ONLY = ("adapt.inc", "functionals.inc")


def source_hash() -> str:
    """SHA-256 over the HIP sources that define or launch the kernels of the timed step."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if os.path.basename(path) in HOST_ONLY:
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--alg-json", default=None,
                    help="output of profile_plate --alg: compulsory bytes per launch of the same launches")
    ap.add_argument("--kind", default=None, help="kernel kind in that JSON (div, grad, ...)")
    args = ap.parse_args()
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
