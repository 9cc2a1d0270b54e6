"""Profiling workload: fine-level residuals R(u) of one configuration, after one plain device copy of a known
size (the calibration of the HBM counters).  Run under rocprofv3, e.g.

    rocprofv3 --pmc FETCH_SIZE -d DIR -- python3 paper_1806_11456_amd/profile_residual.py --config ogrid

Configurations: plate (64x32x1, N = (6,6,1)), ogrid (4,992 hexes, orders iid 1..7), batch (64 problems,
orders iid 2..5).  Prints the launches of every kernel kind per residual.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", choices=["plate", "ogrid", "batch"], required=True)
    ap.add_argument("--residuals", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()
    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    src = torch.ones(args.copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    ctx = pmg.Context(0)
    if args.config == "batch":
        wls = I.config_batch()
        s = pmg.Batch(ctx, [pmg.Mesh(ctx, w.mesh) for w in wls], [w.orders for w in wls], [w.phys for w in wls],
                      pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4, precision=1))
        Q = s.tensor(np.concatenate([w.Q for w in wls], axis=1))
    else:
        wl = I.config_plate() if args.config == "plate" else I.config_ogrid()
        s = pmg.Solver(ctx, pmg.Mesh(ctx, wl.mesh), wl.orders, wl.phys, pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4))
        Q = s.tensor(wl.Q)
    s.autotune()
    R = s.empty()
    kinds = ["trace", "face1", "grad", "face2", "div"]
    s.profile(kinds)
    for _ in range(args.residuals):
        s.residual(Q, None, out=R)
    torch.cuda.synchronize()
    launches = {k: s.profile_read(k)[1] / args.residuals for k in kinds}
    print(json.dumps({"config": args.config, "residuals": args.residuals, "launches_per_residual": launches}),
          flush=True)
    print(f"{args.residuals} residuals done; finite: {bool(torch.isfinite(R).all())}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
