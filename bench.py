#!/usr/bin/env python3
"""Throughput of the DGSEM / FAS p-multigrid hot path on one MI355X; prints one JSON line.

Workload: the flat-plate boundary layer -- 64 x 32 x 1 hexahedra stretched toward the wall (ratio 1.1),
quadratic mapping, orders N = (6, 6, 1) on Gauss nodes (200,704 DOF), Mach 0.2, Re_L = 1e5, no-slip
adiabatic wall and far field, seeded perturbation of the far-field state.

One step = one isotropic FAS V-cycle (levels 6..1, beta_1 = beta_2 = 2 RK3 sweeps, 4 on the coarsest
level) followed by the in-cycle anisotropic truncation-error estimate (3V cycle, isolated tau) on the
same state: every stage of the hot path (residual, RK3 smoothing, restriction/prolongation, V-cycle,
per-direction tau).  value = fine-level DOF-residual evaluations per second over the timed steps
(DOF x fine-level residual evaluations contained in them / wall time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KINDS = ["trace", "face1", "grad", "face2", "div", "dt", "transfer"]
KERNEL_NAME = {"trace": "k_trace", "face1": "k_face1", "grad": "k_grad", "face2": "k_face2", "div": "k_div",
               "dt": "k_dt", "transfer": "k_transfer"}


def cpu_baseline(wl, evals: int):
    """The oracle, as it is, on a bounded sample of the same workload: 'evals' fine-level residuals."""
    import numpy as np

    from oracle import oracle as O
    o = O.Oracle(wl.mesh, wl.phys)
    t0 = time.perf_counter()
    for _ in range(evals):
        R = o.residual(wl.orders, wl.Q)
    dt = time.perf_counter() - t0
    assert np.isfinite(R).all()
    return {"value": wl.n_nodes * evals / dt, "unit": "DOF-residual evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{evals} fine-level residual evaluations R(u) of the same plate state (FP64 C oracle, "
                      f"one thread, {dt:.1f} s)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--beta", type=int, nargs=3, default=[2, 2, 4], metavar=("PRE", "POST", "COARSE"))
    ap.add_argument("--residual-loops", type=int, default=200)
    ap.add_argument("--cpu-evals", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
                  f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    if args.copy_mib:
        src = torch.ones(args.copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = I.config_plate()
    ctx = pmg.Context(0)
    b1, b2, bc = args.beta
    s = pmg.Solver(ctx, pmg.Mesh(ctx, wl.mesh), wl.orders, wl.phys, pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc))
    dof = s.n_nodes
    Q = s.tensor(wl.Q)

    def step():
        s.vcycle(Q, None, n_cycles=1)
        s.tau_estimate(Q, None, isolated=True)

    # fine-level residual evaluations per step: each V-cycle on its top level runs 3 (beta_1 + beta_2) RK
    # stages plus the residual it restricts; tau runs one such cycle per direction with more than one level
    per_cycle = 3 * (b1 + b2) + 1
    tau_dirs = sum(1 for d in range(3) if int(wl.orders[:, d].max()) > 1)
    evals_per_step = per_cycle * (1 + tau_dirs)

    # warm-up; the first step times every kernel kind to find the dominant one
    s.profile(KINDS)
    step()
    torch.cuda.synchronize()
    per_kind = {k: s.profile_read(k) for k in KINDS}
    dominant = max(KINDS, key=lambda k: per_kind[k][0])
    s.profile([])
    for _ in range(max(args.warmup - 1, 0)):
        step()
    torch.cuda.synchronize()

    # timed region: the dominant kernel's launches are bracketed by events on their stream
    s.profile([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n, k_bytes = s.profile_read(dominant)
    s.profile([])
    if not torch.isfinite(Q).all():
        print("non-finite state after the timed steps", file=sys.stderr)
        return 1
    wall = t1 - t0
    value = dof * evals_per_step * args.steps / wall
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0

    # residual-only rate (fine-level R(u) back to back) for comparison with the CPU oracle
    R = s.empty()
    for _ in range(10):
        s.residual(Q, None, out=R)
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    for _ in range(args.residual_loops):
        s.residual(Q, None, out=R)
    torch.cuda.synchronize()
    r_wall = time.perf_counter() - r0

    out = {
        "metric": "fine-level DOF-residual evals/s",
        "value": value,
        "unit": "DOF-residual evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "flat-plate boundary layer: 64x32x1 stretched hexes (ratio 1.1), quadratic mapping, "
                        "N=(6,6,1) Gauss, Mach 0.2, Re_L 1e5, wall + far field",
            "dof": dof,
            "step": f"isotropic FAS V-cycle (levels 6..1, beta {b1}/{b2}/{bc}) + anisotropic 3V isolated tau",
            "fine_residual_evals_per_step": evals_per_step,
        },
        "roofline": {
            "kernel": KERNEL_NAME[dominant],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": 1e3 * k_ms / max(k_n, 1),
            "launches": k_n,
            "alg_bytes_per_launch": k_bytes / max(k_n, 1),
        },
        "residual_only": {"value": dof * args.residual_loops / r_wall, "unit": "DOF-residual evals/s",
                          "us_per_residual": 1e6 * r_wall / args.residual_loops},
        "kernel_ms_first_step": {KERNEL_NAME[k]: round(v[0], 3) for k, v in per_kind.items()},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_evals)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
