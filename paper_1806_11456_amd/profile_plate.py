"""Profiling workload: the flat plate (64 x 32 x 1 hexes, N = (6,6,1), 200,704 DOF) under isotropic FAS
V-cycles (levels 6..1, beta 2/2/4) and fine-level residuals, after one plain device copy of a known size
(the calibration of the HBM counters).  Run under rocprofv3:

    rocprofv3 --pmc FETCH_SIZE -- python3 paper_1806_11456_amd/profile_plate.py --cycles 20 --copy-mib 1024
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--cycles", type=int, default=20)
    ap.add_argument("--residuals", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--alg", action="store_true",
                    help="also print each kernel kind's launches and compulsory bytes (library event timers)")
    args = ap.parse_args()
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    src = torch.ones(args.copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    wl = I.config_plate()
    ctx = pmg.Context(0)
    s = pmg.Solver(ctx, pmg.Mesh(ctx, wl.mesh), wl.orders, wl.phys, pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4))
    Q = s.tensor(wl.Q)
    s.autotune()
    kinds = ["trace", "face1", "grad", "face2", "div", "dt", "transfer"]
    if args.alg:
        s.profile(kinds)
    for _ in range(args.cycles):
        s.vcycle(Q, None, n_cycles=1)
    R = s.empty()
    for _ in range(args.residuals):
        s.residual(Q, None, out=R)
    torch.cuda.synchronize()
    if args.alg:
        import json
        out = {}
        for k in kinds:
            ms, n, b = s.profile_read(k)
            out[k] = {"launches": n, "alg_bytes_per_launch": b / max(n, 1), "event_us_per_launch": 1e3 * ms / max(n, 1)}
        print(json.dumps(out), flush=True)
    print(f"{args.cycles} V-cycles and {args.residuals} residuals done; state finite: {bool(torch.isfinite(Q).all())}",
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
