#!/usr/bin/env python3
"""Throughput of the DGSEM / FAS p-multigrid hot path on one MI355X; prints one JSON line.

Headline workload (the largest single-GPU configuration): 64 independent steady problems solved together --
random stretched boxes of 2k..20k hexahedra with a no-slip wall, orders iid in {2..5} per direction, Mach
U[0.1, 0.4], Re U[1e2, 1e4] (63.9M DOF) -- in one batched solver: union mesh, one launch per kernel kind,
captured V-cycle graphs, autotuned tiles, FP32 coarse-level smoothing inside the FP64 defect correction.  One
step = one iteration of the batched solve driver: the FP64 fine-level residual check of every problem (with
the divergence guard), then one FAS V-cycle (levels 5..1, beta 2/2/4).  value = fine-level DOF-residual
evaluations per second over the timed steps (DOF x fine-level operator evaluations / wall time).

Secondary lines, each with its own roofline of the fine-level residual: the anisotropic O-grid around a
sphere (4,992 curved hexes, orders iid {1..7}^3, 620,512 DOF; FP64 and mixed; step = a solve-driver
iteration + the isolated 3V truncation-error estimate) and the flat plate (200,704 DOF; step = V-cycle +
3V estimate).  roofline = the surveyed algorithmic bytes of one fine-level residual over its time measured
with events on the launch stream; flops likewise from the surveyed flop model.
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

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (and matrix) peak
KINDS = ["trace", "face1", "grad", "face2", "div", "dt", "transfer"]
# the library's kernel kinds; "face2" is the numerical-flux pass (k_face2c on conforming and boundary faces,
# k_face2 on p-nonconforming ones)
KERNEL_NAME = {"trace": "k_trace", "face1": "k_face1", "grad": "k_grad", "face2": "k_face2c+k_face2",
               "div": "k_div", "dt": "k_dt", "transfer": "k_transfer"}
CPU_SHARE = 16  # host threads one GPU's share of the box allows


def alg_model(orders_list):
    """(nodes, element face nodes, algorithmic bytes, flops) of one fine-level residual R(u), the surveyed
    minimum: per node read Q (40 B) and the metric terms (80 B) and write R (40 B); per element face node its
    traces of q and F^v . n (10 values) written by one side and read by the other (160 B); flops 34 sum_d n_d
    + 650 per node and 125 per element face node (for isotropic order N: 102 (N+1) + 650 + 750 / (N+1) per
    node, the gradient and divergence contractions, pointwise fluxes, lifts and face work)."""
    import numpy as np
    nn = nf = fl = 0
    for o in orders_list:
        n = np.asarray(o, dtype=np.int64) + 1
        npe = n.prod(axis=1)
        fpe = 2 * (n[:, 1] * n[:, 2] + n[:, 0] * n[:, 2] + n[:, 0] * n[:, 1])
        nn += int(npe.sum())
        nf += int(fpe.sum())
        fl += int((npe * (34 * n.sum(axis=1) + 650) + 125 * fpe).sum())
    return nn, nf, 160.0 * (nn + nf), float(fl)


_CPU_WORK = []  # (mesh, orders, phys, Q) of the sampled problems, shared with forked workers


def _cpu_one(i):
    from oracle import oracle as O
    mesh, orders, phys, Q = _CPU_WORK[i]
    R = O.Oracle(mesh, phys).residual(orders, Q)
    return int(Q.shape[1]), bool(__import__("numpy").isfinite(R).all())


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(works, single_budget_s: float, pool_rounds: int) -> dict:
    """The oracle, as it is, on a bounded sample of the same workload, before the GPU is touched: one thread
    over the sampled problems' fine-level residuals until the budget is spent; then every host thread of the
    GPU's share (at most 16), one process per thread, each evaluating whole problems' residuals (the batch's
    problems are independent), over pool_rounds x threads problems."""
    import multiprocessing as mp

    _CPU_WORK[:] = works
    t0 = time.perf_counter()
    dof = 0
    n1 = 0
    while n1 < len(works) and time.perf_counter() - t0 < single_budget_s:
        d, ok = _cpu_one(n1)
        assert ok
        dof += d
        n1 += 1
    t1 = time.perf_counter() - t0
    single = dof / t1
    affinity = len(os.sched_getaffinity(0))
    threads = max(1, min(CPU_SHARE, affinity))
    idx = [i % len(works) for i in range(pool_rounds * threads)]
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS",)}
    os.environ["OMP_NUM_THREADS"] = "1"
    t2 = time.perf_counter()
    with mp.get_context("fork").Pool(threads) as pool:
        res = pool.map(_cpu_one, idx, chunksize=1)
    t3 = time.perf_counter() - t2
    for k, v in env.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    assert all(ok for _, ok in res)
    allc = sum(d for d, _ in res) / t3
    return {"value": allc, "unit": "DOF-residual evals/s", "cores": threads, "kind": "oracle",
            "sample": f"fine-level residuals R(u) of whole problems of the same batch (FP64 C oracle): "
                      f"{len(idx)} problem residuals on {threads} processes of one thread each in {t3:.1f} s; "
                      f"one thread: {n1} problem residuals in {t1:.1f} s",
            "single_thread": {"value": single, "cores": 1, "problems": n1, "seconds": t1},
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity": affinity}}


def residual_roofline(s, Q, orders_list, loops: int, counters_name: str):
    """Fine-level R(u) back to back, timed with events on the stream the library launches on: its algorithmic
    bytes and flops over that time (roofline), and each kernel's share (every launch bracketed by the
    library's own events, in a separate shorter loop)."""
    import torch

    nn, nf, B, F = alg_model(orders_list)
    R = s.empty()
    for _ in range(3):
        s.residual(Q, None, out=R)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(loops):
        s.residual(Q, None, out=R)
    e1.record(st)
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / loops
    s.profile(KINDS)
    nk = max(3, loops // 10)
    for _ in range(nk):
        s.residual(Q, None, out=R)
    torch.cuda.synchronize()
    per = {k: s.profile_read(k) for k in KINDS}
    s.profile([])
    kern = {KERNEL_NAME[k]: {"us": round(1e3 * v[0] / nk, 2), "launches": v[1] // nk}
            for k, v in per.items() if v[1]}
    dominant = max(kern, key=lambda k: kern[k]["us"])
    traffic, ratio = None, None
    cpath = os.path.join(ROOT, "profiles", f"residual_{counters_name}_counters.json")
    if os.path.exists(cpath):
        from paper_1806_11456_amd import counters
        with open(cpath) as f:
            c = json.load(f)
        if c.get("source_sha256") == counters.source_hash():
            traffic = c["traffic_bytes_per_residual"]
            ratio = traffic / B
    achieved = B / t / 1e9
    return {
        "roofline": {"kernel": "fine-level residual R(u): " + ", ".join(kern), "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_over_alg": ratio, "alg_bytes_per_launch": B,
                     "alg_bytes_model": "160 B per node + 160 B per element face node",
                     "avg_launch_us": 1e6 * t, "nodes": nn, "element_face_nodes": nf,
                     "dominant_kernel": dominant, "per_kernel_us": kern},
        "flops": {"achieved_tflops": F / t / 1e12, "peak_tflops": FP64_PEAK_TFLOPS,
                  "frac": F / t / 1e12 / FP64_PEAK_TFLOPS, "flops_per_residual": F},
        "residual_only": {"value": nn / t, "unit": "DOF-residual evals/s", "us_per_residual": 1e6 * t},
    }


def timed(step, steps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def tile_desc(s):
    """The autotuned element tiles of each level, finest first: node target, and which kernels launch once
    per tile-size class."""
    out = []
    for l in reversed(range(s.level_info(-1))):  # level 0 is the coarsest
        t, sp = s.level_tile_choice(-1, l)
        per = [k for k, bit in (("grad", 1), ("div", 2)) if sp & bit]
        out.append(f"{t}" + (f" split({','.join(per)})" if per else ""))
    return "autotuned per level, finest first: " + ", ".join(out)


def batch_line(args, wls) -> dict:
    """Configuration of 64 independent problems: batched solve-driver iterations (mixed precision, graph
    replay, autotuned tiles, divergence guard)."""
    import numpy as np
    import torch

    from paper_1806_11456_amd import pmg

    ctx = pmg.Context(0)
    t0 = time.perf_counter()
    meshes = [pmg.Mesh(ctx, w.mesh) for w in wls]
    b1, b2, bc = args.beta
    mg = pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc, precision=1, guard=8)
    b = pmg.Batch(ctx, meshes, [w.orders for w in wls], [w.phys for w in wls], mg)
    Q = b.tensor(np.concatenate([w.Q for w in wls], axis=1))
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    b.autotune()
    b.set_graph(True)
    roof = residual_roofline(b, Q, [w.orders for w in wls], args.residual_loops_batch, "batch64")
    # one call per phase: each driver iteration is a residual check (+ guard) and a V-cycle; the call ends with
    # one more check
    b.solve_all(Q, None, tol=0.0, max_cycles=args.warmup, raise_not_converged=False, raise_failed=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc, r = b.solve_all(Q, None, tol=0.0, max_cycles=args.steps, raise_not_converged=False, raise_failed=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    halv, _ = b.guard_stats()
    print(f"batch: guard halvings per problem {halv.tolist()}; given up: {np.flatnonzero(np.isnan(r)).tolist()}; "
          f"cycles on FP32 coarse levels per problem {b.fp32_cycles().tolist()}", file=sys.stderr, flush=True)
    per_cycle = 3 * (b1 + b2) + 1
    # fine-level evaluations done: every problem's cycles (a problem the guard gave up on stops cycling) and the
    # batched residual checks, which cover every problem
    dofs = np.diff(b.problem_offsets).astype(np.float64)
    done = float(np.sum(dofs * per_cycle * cyc) + b.n_nodes * (args.steps + 1))
    fp32 = b.fp32_cycles()
    tiles = tile_desc(b)
    n_nodes = b.n_nodes
    fp64 = None
    if not args.no_batch_fp64:
        # the same calls on an FP64 batch from the same start: the mixed precision's saving and its state error
        Qm = Q.detach().cpu().numpy()
        del b, Q
        torch.cuda.synchronize()
        b64 = pmg.Batch(ctx, meshes, [w.orders for w in wls], [w.phys for w in wls],
                        pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc, precision=0, guard=8))
        Q64 = b64.tensor(np.concatenate([w.Q for w in wls], axis=1))
        b64.autotune()
        b64.set_graph(True)
        b64.solve_all(Q64, None, tol=0.0, max_cycles=args.warmup, raise_not_converged=False, raise_failed=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b64.solve_all(Q64, None, tol=0.0, max_cycles=args.steps, raise_not_converged=False, raise_failed=False)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t0
        h64, _ = b64.guard_stats()
        Qd = Q64.detach().cpu().numpy()
        err = np.abs(Qm - Qd).max(axis=1) / np.abs(Qd).max(axis=1)
        fp64 = {"ms_per_step": 1e3 * wall64 / args.steps, "mixed_speedup": wall64 / wall,
                "guard_halvings": int(h64.sum()), "state_error_of_mixed": [float(x) for x in err],
                "state_error_meaning": "after the same warm-up and timed steps from the same start: "
                                       "max |Q_mixed - Q_fp64| / max |Q_fp64| per variable over the batch"}
        print(f"batch FP64: {fp64['ms_per_step']:.1f} ms/step, mixed {fp64['mixed_speedup']:.2f}x faster, state "
              f"error {np.array2string(err, precision=2)}", file=sys.stderr, flush=True)
        del b64, Q64
    return {"value": done / wall, "ms_per_step": 1e3 * wall / args.steps,
            "config": {"workload": "64 independent steady problems (seed 4): random boxes of 2k..20k hexes "
                                   "stretched toward a no-slip wall, orders iid U{2..5}^3, Mach U[0.1,0.4], "
                                   "Re U[1e2,1e4], trilinear mapping, Gauss nodes",
                       "dof": n_nodes, "problems": len(wls),
                       "step": f"batched solve-driver iteration: FP64 residual check + divergence guard + one FAS "
                               f"V-cycle (levels 5..1, beta {b1}/{b2}/{bc}), FP32 coarse levels, graph replay",
                       "tiles": tiles, "fine_residual_evals_per_step": per_cycle + 1,
                       "setup_s": round(setup, 2)},
            "guard_halvings": int(halv.sum()), "problems_halved": int((halv > 0).sum()),
            "problems_given_up": int(np.isnan(r).sum()), "cycles_run": int(np.sum(cyc)),
            "fp32_cycles_min": int(fp32.min()), "residual_max": float(np.nanmax(r)), "fp64": fp64, **roof}


def ogrid_line(args) -> dict:
    """Anisotropic O-grid around a sphere, random orders 1..7: solve-driver iteration + isolated 3V tau."""
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    wl = I.config_ogrid()
    ctx = pmg.Context(0)
    mesh = pmg.Mesh(ctx, wl.mesh)
    b1, b2, bc = args.beta
    out = {}
    states = {}
    for prec in (0, 1):
        s = pmg.Solver(ctx, mesh, wl.orders, wl.phys, pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc,
                                                              precision=prec, guard=8))
        Q = s.tensor(wl.Q)
        Qc = torch.empty_like(Q)
        tau = s.tau_estimate(Q.clone(), None, isolated=True)  # builds every level
        s.autotune()
        s.set_graph(True)

        def step():
            s.solve(Q, None, tol=0.0, max_cycles=1, raise_not_converged=False)
            Qc.copy_(Q)
            s.tau_estimate(Qc, None, isolated=True, out=tau)

        wall = timed(step, args.ogrid_steps, 1)
        halv, _ = s.guard_stats()
        states[prec] = Q.detach().cpu().numpy()
        if prec == 0:
            per_cycle = 3 * (b1 + b2) + 1
            evals = per_cycle + 2 + 3 * per_cycle  # cycle, two checks, one V-cycle per direction (3V)
            out = {"value": s.n_nodes * evals * args.ogrid_steps / wall, "ms_per_step": 1e3 * wall / args.ogrid_steps,
                   "config": {"workload": "O-grid around a unit sphere: 6 panels of 8x8 x 13 radial cells (4,992 "
                                          "hexes, r in [1,20], ratio 1.25), quadratic mapping, rotated element "
                                          "frames, orders iid U{1..7}^3 (seed 3), Mach 0.2, Re 200, Gauss nodes",
                              "dof": s.n_nodes,
                              "step": f"solve-driver iteration (residual checks + guard + FAS V-cycle, levels 7..1, "
                                      f"beta {b1}/{b2}/{bc}) + isolated anisotropic 3V tau estimate of the state",
                              "tiles": tile_desc(s), "fine_residual_evals_per_step": evals},
                   "guard_halvings": int(halv.sum()),
                   **residual_roofline(s, Q, [wl.orders], args.residual_loops, "ogrid8x13")}
        else:
            import numpy as np
            d = np.abs(states[1] - states[0]).max(axis=1) / np.abs(states[0]).max(axis=1)
            out["mixed"] = {"ms_per_step": 1e3 * wall / args.ogrid_steps, "guard_halvings": int(halv.sum()),
                            "speedup_vs_fp64": out["ms_per_step"] / (1e3 * wall / args.ogrid_steps),
                            "state_error_vs_fp64": [float(x) for x in d],
                            "state_error_meaning": "after the same warm-up and timed steps from the same start: "
                                                   "max |Q_mixed - Q_fp64| / max |Q_fp64| per variable"}
        del s, Q, Qc
    return out


def plate_line(args) -> dict:
    """Flat plate: isotropic V-cycle + isolated 3V tau estimate on the same state."""
    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    wl = I.config_plate()
    ctx = pmg.Context(0)
    b1, b2, bc = args.beta
    s = pmg.Solver(ctx, pmg.Mesh(ctx, wl.mesh), wl.orders, wl.phys, pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc))
    Q = s.tensor(wl.Q)
    s.tau_estimate(s.tensor(wl.Q), None, isolated=True)  # builds every level
    s.autotune()

    def step():
        s.vcycle(Q, None, n_cycles=1)
        s.tau_estimate(Q, None, isolated=True)

    wall = timed(step, args.plate_steps, 2)
    per_cycle = 3 * (b1 + b2) + 1
    evals = per_cycle * 3  # the V-cycle and one cycle per direction with more than one level (x, y)
    return {"value": s.n_nodes * evals * args.plate_steps / wall, "ms_per_step": 1e3 * wall / args.plate_steps,
            "config": {"workload": "flat-plate boundary layer: 64x32x1 stretched hexes (ratio 1.1), quadratic "
                                   "mapping, N=(6,6,1) Gauss, Mach 0.2, Re_L 1e5, wall + far field",
                       "dof": s.n_nodes,
                       "step": f"isotropic FAS V-cycle (levels 6..1, beta {b1}/{b2}/{bc}) + anisotropic 3V "
                               f"isolated tau", "tiles": tile_desc(s), "fine_residual_evals_per_step": evals},
            **residual_roofline(s, Q, [wl.orders], args.residual_loops, "plate64x32")}


def serve_bench(args) -> dict:
    """Served stream (reduced sizes): Poisson arrivals at 20/s of steady-solve
    requests on random stretched boxes with a wall, solved to ||r||_inf < 1e-9 by the continuous-batching
    server, per-request solvers on several streams and union solvers (batched); baseline: the same list
    solved one after another with pmg_solve (plain FP64) on the same GPU, queued first come, first served at
    the same arrival times.  All include solver construction."""
    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    reqs = I.config_serve(n=args.serve_n, seed=5, rate=20.0, kmin=args.serve_kmin, kmax=args.serve_kmax, lo=1,
                          hi=4, re_lo=1e3, re_hi=1e4, ogrid_frac=0.0)
    ctx = pmg.Context(0)
    mg = pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4, precision=args.serve_precision)
    meshes = [pmg.Mesh(ctx, w.mesh) for _, w, _ in reqs]
    max_cycles = 20000
    pct = lambda x, q: float(np.percentile(x, q))

    def served_run(batched: bool) -> dict:
        states = [torch.tensor(w.Q, dtype=torch.float64, device="cuda") for _, w, _ in reqs]
        torch.cuda.synchronize()
        sv = pmg.Server(ctx, int(args.serve_budget_gib * 2 ** 30), n_streams=args.serve_streams, use_graph=True,
                        batched=batched)
        t0 = time.perf_counter()
        tickets = []
        for (arr, w, tol), m, Q in zip(reqs, meshes, states):
            dt = t0 + arr - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append(sv.submit(m, w.orders, w.phys, mg, Q, tol=tol, max_cycles=max_cycles))
        done = {}
        last = t0
        while len(done) < len(tickets):
            for t in tickets:
                if t not in done:
                    r = sv.poll(t)
                    if r is not None:
                        done[t] = r
                        last = time.perf_counter()
                        print(f"served{' batched' if batched else ''} {len(done)}/{len(tickets)}: {r}",
                              file=sys.stderr, flush=True)
            time.sleep(0.001)
        stats = sv.stats()
        sv.close()
        served = [done[t] for t in tickets]
        lat = np.array([r["latency_s"] for r in served])
        return {"p50_s": pct(lat, 50), "p99_s": pct(lat, 99), "solves_per_s": len(reqs) / (last - t0),
                "makespan_s": last - t0, "converged": int(sum(r["status"] == 0 for r in served)),
                "cycles_total": int(sum(r["cycles"] for r in served)), "max_resident": stats["max_resident"],
                "peak_bytes": stats["peak_bytes"], "iterations": stats["iterations"]}

    modes = [m for m in args.serve_modes.split(",") if m]
    out_served = {}
    for m in modes:
        assert m in ("per-request", "batched"), m
        out_served[m] = served_run(m == "batched")

    # baseline: sequential plain FP64 solves
    seq = None
    if not args.serve_no_sequential:
        solve_t = []
        base_ok = 0
        for (arr, w, tol), m in zip(reqs, meshes):
            torch.cuda.synchronize()
            a = time.perf_counter()
            s = pmg.Solver(ctx, m, w.orders, w.phys, pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4))
            s.set_graph(True)
            Q = s.tensor(w.Q)
            cyc, r = s.solve(Q, None, tol=tol, max_cycles=max_cycles, raise_not_converged=False)
            torch.cuda.synchronize()
            solve_t.append(time.perf_counter() - a)
            base_ok += r < tol
            print(f"sequential {len(solve_t)}/{len(reqs)}: {cyc} cycles, {solve_t[-1]:.2f} s", file=sys.stderr,
                  flush=True)
            del s, Q
        end = 0.0
        blat = []
        for (arr, _, _), d in zip(reqs, solve_t):
            start = max(arr, end)
            end = start + d
            blat.append(end - arr)
        blat = np.array(blat)
        seq = {"p50_s": pct(blat, 50), "p99_s": pct(blat, 99), "solves_per_s": len(reqs) / end, "makespan_s": end,
               "converged": int(base_ok), "solve_s_mean": float(np.mean(solve_t))}
    head = out_served[modes[0]]
    return {
        "metric": "p50/p99 latency (arrival to result); solves/s",
        "value": head["p50_s"],
        "unit": "s",
        "higher_is_better": False,
        "n_gpus": 1,
        "dtype": "f64" if args.serve_precision == 0 else "mixed f32/f64",
        "data": "synthetic",
        "config": {"workload": f"served stream: {len(reqs)} requests, Poisson arrivals 20/s (seed 5), random "
                               f"stretched boxes K {args.serve_kmin}..{args.serve_kmax} with a no-slip wall and far "
                               "field, orders U{1..4} per direction, Mach U[0.1,0.4], Re U[1e3,1e4], tol 1e-9, "
                               "V-cycles beta 2/2/4",
                   "dof_total": int(sum(w.n_nodes for _, w, _ in reqs)), "streams": args.serve_streams,
                   "hbm_budget_gib": args.serve_budget_gib, "value_from": modes[0]},
        "served": out_served,
        "sequential_fp64": seq,
    }


def solve_batch_bench(args) -> dict:
    """The 64-problem batch solved toward ||r||_inf < tol per problem with the headline's batched solve driver
    (mixed precision, divergence guard, graph replay), in calls of 'chunk' cycles until the time limit: after
    every call, how many problems have converged, the spread of the residuals, the guard's halvings and the
    problems it gave up on."""
    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    wls = I.config_batch()
    ctx = pmg.Context(0)
    b1, b2, bc = args.beta
    t_setup = time.perf_counter()
    meshes = [pmg.Mesh(ctx, w.mesh) for w in wls]
    b = pmg.Batch(ctx, meshes, [w.orders for w in wls], [w.phys for w in wls],
                  pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc, precision=1, guard=8))
    Q = b.tensor(np.concatenate([w.Q for w in wls], axis=1))
    b.autotune()
    b.set_graph(True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t_setup
    tol = args.solve_tol
    r = np.asarray(b.norms(Q))
    hist = []
    cycles = np.zeros(len(wls), dtype=np.int64)
    t0 = time.perf_counter()

    def record():
        halv, _ = b.guard_stats()
        ok = r[np.isfinite(r)]
        row = {"t_s": round(time.perf_counter() - t0, 1), "cycles_max": int(cycles.max()),
               "converged": int(np.sum(r < tol)), "given_up": int(np.sum(~np.isfinite(r))),
               "r_min": float(ok.min()) if ok.size else None, "r_median": float(np.median(ok)) if ok.size else None,
               "r_max": float(ok.max()) if ok.size else None, "guard_halvings": int(halv.sum())}
        hist.append(row)
        print("solve-batch: " + json.dumps(row), file=sys.stderr, flush=True)

    record()
    while time.perf_counter() - t0 < args.solve_batch_s and np.sum(r < tol) + np.sum(~np.isfinite(r)) < len(wls):
        cyc, r = b.solve_all(Q, None, tol=tol, max_cycles=args.solve_batch_chunk, raise_not_converged=False,
                             raise_failed=False)
        cycles += np.asarray(cyc)
        r = np.asarray(r)
        record()
    torch.cuda.synchronize()
    return {"metric": "batched solve progress", "value": hist[-1]["converged"], "unit": "problems converged",
            "higher_is_better": True, "n_gpus": 1, "dtype": "f64/f32 (FP64 finest level and checks, FP32 coarse "
            "levels until the switch)", "data": "synthetic",
            "config": {"workload": "64 independent steady problems (seed 4), the headline batch", "dof": b.n_nodes,
                       "tol": tol, "vcycle": f"levels 5..1, beta {b1}/{b2}/{bc}, guard 8 halvings",
                       "chunk_cycles": args.solve_batch_chunk, "time_limit_s": args.solve_batch_s,
                       "setup_s": round(setup, 2)},
            "cycles_per_problem": cycles.tolist(), "final_residual": [float(x) for x in r],
            "fp32_cycles_last_call": b.fp32_cycles().tolist(), "history": hist}


def solve_bench(args) -> dict:
    """Time to a converged solve: the flat plate from the far-field state to ||r||_inf < tol with FP64 FAS
    V-cycles (beta 2/2/4, captured graphs), the norm read every 'chunk' cycles; the oracle's time is
    extrapolated as (cycles) x (one oracle V-cycle on the same plate, measured)."""
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    wl = I.config_plate()
    ctx = pmg.Context(0)
    b1, b2, bc = args.solve_beta
    paper = args.solve_tuning or args.solve_fmg > 0
    mg = pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc, precision=args.solve_precision,
                tuning=int(args.solve_tuning), max_repeats=args.solve_max_repeats)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    mesh = pmg.Mesh(ctx, wl.mesh)
    s = pmg.Solver(ctx, mesh, wl.orders, wl.phys, mg)
    s.set_graph(True)
    Q = s.freestream()
    torch.cuda.synchronize()
    setup = time.perf_counter() - t_setup
    r0 = s.residual(Q, None, norm=True)[1]
    chunk = args.solve_chunk
    cycles, r = 0, r0
    hist = [(0, r0)]
    t0 = time.perf_counter()
    if args.solve_fmg > 0:
        # the FMG start (Sec. 3.1.1) with the same smoothing, once, on a solver that has it
        sf = pmg.Solver(ctx, mesh, wl.orders, wl.phys, pmg.MG(beta_pre=b1, beta_post=b2, beta_coarse=bc, fmg=1,
                                                             fmg_threshold=args.solve_fmg, tuning=int(args.solve_tuning),
                                                             max_repeats=args.solve_max_repeats))
        # the solve stops on the finest level as soon as its residual is below the FMG threshold
        c, r = sf.solve(Q, None, tol=args.solve_fmg, max_cycles=args.solve_max_cycles, raise_not_converged=False)
        del sf
        cycles += c
        hist.append((cycles, r))
        print(f"solve: FMG start, {cycles} cycles, residual {r:.3e}, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    while r >= args.solve_tol and cycles < args.solve_max_cycles and time.perf_counter() - t0 < args.solve_max_s:
        if args.solve_precision == 1 or paper:
            # the solve driver: mixed precision switch, residual-based smoothing tuning
            c, r = s.solve(Q, None, tol=args.solve_tol, max_cycles=chunk, raise_not_converged=False)
        else:
            r = s.vcycle(Q, None, n_cycles=chunk, norm=True)
            c = chunk
        cycles += c
        hist.append((cycles, r))
        print(f"solve: {cycles} cycles, residual {r:.3e}, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"metric": "time to converged solve", "value": wall if r < args.solve_tol else None, "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64" if args.solve_precision == 0 else "mixed f32/f64",
           "data": "synthetic",
           "config": {"workload": "flat-plate boundary layer: 64x32x1 stretched hexes (ratio 1.1), quadratic "
                                  "mapping, N=(6,6,1) Gauss, Mach 0.2, Re_L 1e5, wall + far field; far-field start",
                      "dof": s.n_nodes, "tol": args.solve_tol,
                      "vcycle": f"levels 6..1, beta {b1}/{b2}/{bc}" + (" (tuned, Sec. 3.1.2, at most "
                                f"{args.solve_max_repeats} repetitions)" if args.solve_tuning else ", graph replay")
                                + (f", FMG start to {args.solve_fmg}" if args.solve_fmg > 0 else ""),
                      "norm_every": chunk},
           "converged": bool(r < args.solve_tol), "cycles": cycles, "wall_s": wall, "residual": r,
           "initial_residual": r0, "setup_s": setup, "ms_per_cycle": 1e3 * wall / max(cycles, 1),
           "history": hist}
    if not args.no_cpu:
        from oracle import oracle as O
        o = O.Oracle(wl.mesh, wl.phys)
        Qf = I.freestream_state(wl.n_nodes, wl.phys.mach)
        c0 = time.perf_counter()
        o.vcycles(wl.orders, Qf, None, ncycles=1, beta_pre=2, beta_post=2, beta_coarse=4)
        oc = time.perf_counter() - c0
        out["cpu_baseline"] = {"kind": "oracle", "cores": 1, "oracle_s_per_cycle": oc,
                               "extrapolated_s": oc * cycles,
                               "sample": "one oracle V-cycle on the same plate state (FP64 C oracle, one thread); "
                                         "time to solve = cycles x that, extrapolated"}
    return out


def compare_bench(args) -> dict:
    """Pure explicit RK3 against the FAS p-multigrid solve driver as solvers of one steady problem from the
    far-field state on the GPU (the paper's comparison of Tables 1 and 2, without adaptation): FAS with the
    paper's smoothing (beta^0 = 100/100/400 with the residual-based tuning of Sec. 3.1.2 and the FMG start of
    Sec. 3.1.1) and with fixed beta 2/2/4; each method runs for a bounded time, the residual read after every
    chunk.  Reported: the time each first reaches the lowest residual all of them reach (measured); each
    method's time to the tolerance, measured where reached, else extrapolated from the log-linear rate over the
    last third of its history (labelled); their ratios to RK3."""
    import math

    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    ctx = pmg.Context(0)
    if args.compare_case == "plate":
        wl = I.config_plate()
        mesh_h, orders, phys, top, coarse, fmg_thr = wl.mesh, wl.orders, wl.phys, 6, 1, 0.1
        workload = ("flat-plate boundary layer: 64x32x1 stretched hexes (ratio 1.1), quadratic mapping, N=(6,6,1) "
                    "Gauss, Mach 0.2, Re_L 1e5, wall + far field; far-field start")
    else:
        mesh_h = I.ogrid_mesh(8, 13, r_out=20.0, ratio=1.25)
        N = args.sphere_order
        orders = I.uniform_orders(mesh_h.K, (N, N, N))
        phys = I.Physics(mach=0.2, reynolds=100.0, family=I.FAMILY_LG, cfl_adv=args.sphere_cfl,
                         cfl_visc=args.sphere_cfl)
        top, coarse, fmg_thr = N, 2, 1.0
        workload = (f"sphere, Re_D 200, Mach 0.2: six-panel O-grid 8x8x13 per panel (4992 hexes), outer radius 20, "
                    f"quadratic mapping, uniform order {N}; far-field start")
    mesh = pmg.Mesh(ctx, mesh_h)
    caps = list(range(top, coarse - 1, -1))
    tol = args.compare_tol

    def mg(**k):
        return pmg.MG(level_caps=caps, guard=8, **k)

    def run(name, chunk, advance, setup=None):
        s = pmg.Solver(ctx, mesh, orders, phys, mg(beta_pre=2, beta_post=2, beta_coarse=4))
        s.set_graph(True)
        Q = s.freestream()
        r0 = s.residual(Q, None, norm=True)[1]
        hist = [(0.0, 0, r0)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, last = 0, t0
        if setup is not None:
            n, r = setup(s, Q)
            hist.append((time.perf_counter() - t0, n, r))
        while time.perf_counter() - t0 < args.compare_s and hist[-1][2] >= tol:
            n += advance(s, Q, chunk)
            r = s.residual(Q, None, norm=True)[1]
            hist.append((time.perf_counter() - t0, n, r))
            if r != r:
                break
            if time.perf_counter() - last > 10.0:
                last = time.perf_counter()
                print(f"compare {args.compare_case} {name}: {n} after {hist[-1][0]:.1f} s, residual {r:.3e}",
                      file=sys.stderr, flush=True)
        del s, Q
        return hist

    b0 = args.compare_paper_beta
    paper = pmg.Solver(ctx, mesh, orders, phys, mg(beta_pre=b0[0], beta_post=b0[1], beta_coarse=b0[2], tuning=1,
                                                    max_repeats=10))
    fmg = pmg.Solver(ctx, mesh, orders, phys, mg(beta_pre=b0[0], beta_post=b0[1], beta_coarse=b0[2], tuning=1,
                                                  max_repeats=10, fmg=1, fmg_threshold=fmg_thr))

    def paper_setup(s, Q):
        c, r = fmg.solve(Q, None, tol=fmg_thr, max_cycles=100000, raise_not_converged=False)
        return c, r

    def paper_advance(s, Q, c):
        cyc, _ = paper.solve(Q, None, tol=tol, max_cycles=c, raise_not_converged=False)
        return cyc

    hist = {
        "rk3": run("rk3", args.compare_rk_chunk, lambda s, Q, c: (s.smooth(Q, None, sweeps=c), c)[1]),
        "fas_paper": run("fas_paper", args.compare_paper_chunk, paper_advance, paper_setup),
        "fas_fixed": run("fas_fixed", args.compare_fas_chunk, lambda s, Q, c: (s.vcycle(Q, None, n_cycles=c), c)[1]),
    }
    best = {m: min(r for _, _, r in h if r == r) for m, h in hist.items()}
    level = max(best.values())

    def first(h, lv):
        return next(((t, n) for t, n, r in h if r <= lv), (None, None))

    def to_tol(h):
        t, n = first(h, tol)
        if t is not None:
            return {"seconds": t, "work": n, "measured": True}
        tail = [(t, r) for t, _, r in h[len(h) * 2 // 3:] if r == r and r > 0]
        if len(tail) < 3:
            return {"seconds": None, "measured": False}
        tt = np.array([x[0] for x in tail])
        lr = np.log10([x[1] for x in tail])
        slope = np.polyfit(tt, lr, 1)[0]
        if slope >= 0:
            return {"seconds": None, "measured": False, "rate_decades_per_s": float(slope)}
        return {"seconds": float(tt[-1] + (math.log10(tol) - lr[-1]) / slope), "measured": False,
                "rate_decades_per_s": float(slope)}

    reach = {m: first(h, level) for m, h in hist.items()}
    tol_t = {m: to_tol(h) for m, h in hist.items()}
    t_rk = reach["rk3"][0]
    speed = {m: (t_rk / t if t and t_rk else None) for m, (t, _) in reach.items()}
    rk_tol = tol_t["rk3"]["seconds"]
    speed_tol = {m: (rk_tol / v["seconds"] if v["seconds"] and rk_tol else None) for m, v in tol_t.items()}
    return {"metric": "speed-up over RK3 (equal residual; time to tolerance)", "value": speed["fas_paper"],
            "unit": "x", "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": workload, "dof": int(I.node_offsets(orders)[-1]), "levels": caps, "tol": tol,
                       "seconds_per_method": args.compare_s,
                       "fas_paper": f"solve driver, beta^0 {b0[0]}/{b0[1]}/{b0[2]}, tuning (at most 10 repetitions), "
                                    f"FMG start to {fmg_thr}", "fas_fixed": "V-cycles, beta 2/2/4, graph replay",
                       "units": {"rk3": "sweeps", "fas_paper": "V-cycles", "fas_fixed": "V-cycles"}},
            "level": level, "speedup_at_level": speed,
            "time_to_level_s": {m: t for m, (t, _) in reach.items()},
            "time_to_tol": tol_t, "speedup_to_tol": speed_tol,
            "paper_ratio": {"plate": 71.51, "sphere": 27.41}[args.compare_case],
            "best_residual": best,
            "history": {m: [(round(t, 3), n, r) for t, n, r in h[:: max(1, len(h) // 40)]] + [h[-1]]
                        for m, h in hist.items()}}


def sphere_bench(args) -> dict:
    """Soft physics check (not parity): steady flow past the unit sphere at Re_D = 200, Mach 0.2 (Re = 100 on
    the radius), the six-panel O-grid (8 x 8 x 13 hexes per panel, outer radius 20, quadratic mapping) at
    uniform order N, FAS V-cycles on levels N..2 from the far-field state; the drag coefficient
    C_d = 2 F_x / (pi r^2) after every chunk of cycles, for comparison with the paper's 0.7771."""
    import math

    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    N = args.sphere_order
    mesh = I.ogrid_mesh(8, 13, r_out=20.0, ratio=1.25)
    orders = I.uniform_orders(mesh.K, (N, N, N))
    phys = I.Physics(mach=0.2, reynolds=100.0, family=I.FAMILY_LG, cfl_adv=args.sphere_cfl,
                     cfl_visc=args.sphere_cfl)
    ctx = pmg.Context(0)
    s = pmg.Solver(ctx, pmg.Mesh(ctx, mesh), orders, phys,
                   pmg.MG(level_caps=list(range(N, 1, -1)), beta_pre=2, beta_post=2, beta_coarse=4))
    s.set_graph(True)
    Q = s.freestream()
    area = math.pi
    hist = []
    t0 = time.perf_counter()
    cycles = 0
    r = s.residual(Q, None, norm=True)[1]
    while time.perf_counter() - t0 < args.sphere_s and r > args.sphere_tol:
        r = s.vcycle(Q, None, n_cycles=args.sphere_chunk, norm=True)
        cycles += args.sphere_chunk
        if r != r:
            break
        F = s.wall_force(Q)
        cd, cl = pmg.force_coefficients(F, area)
        hist.append((cycles, round(time.perf_counter() - t0, 2), r, cd, cl, float(2 * F[0] / area),
                     float(2 * F[3] / area)))
        print(f"sphere: {cycles} cycles, {hist[-1][1]:.1f} s, residual {r:.3e}, C_d {cd:.5f} "
              f"(pressure {hist[-1][5]:.5f}, viscous {hist[-1][6]:.5f}), C_l {cl:.2e}", file=sys.stderr, flush=True)
    last = hist[-1] if hist else None
    return {"metric": "sphere drag coefficient (soft physics check)", "value": last[3] if last else None,
            "unit": "C_d", "higher_is_better": None, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "sphere, Re_D 200, Mach 0.2: six-panel O-grid 8x8x13 per panel (4992 hexes), "
                                   "outer radius 20, radial ratio 1.25, quadratic mapping, far-field start",
                       "order": N, "dof": s.n_nodes, "levels": list(range(N, 1, -1)), "beta": [2, 2, 4],
                       "cfl": args.sphere_cfl},
            "paper_cd": 0.7771, "cycles": cycles, "residual": r,
            "history": hist[:: max(1, len(hist) // 30)] + ([last] if last else [])}


def sphere_adapt_bench(args) -> dict:
    """The structure of the paper's single-stage adaptation of the sphere (Sec. 4.2): the sphere of
    sphere_bench converged at uniform P = 4, its isolated truncation-error map estimated by the anisotropic
    3V cycle (on a copy of the state), new orders for a few tau_max with the 3-D rules (the floor(2N/3)
    order-jump rule, conforming orders on the wall, n_max = 6) and n_min = 4: with the quadratic mapping
    (M = 2) the curl-form metric keeps the free stream on p-nonconforming faces only for N >= 2M; the state
    carried over and the adapted problem converged; C_d of each against a uniform order-6 reference solved the
    same way (or given by --sphere-ref-cd from an earlier run)."""
    import math

    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    mesh_h = I.ogrid_mesh(8, 13, r_out=20.0, ratio=1.25)
    phys = I.Physics(mach=0.2, reynolds=100.0, family=I.FAMILY_LG, cfl_adv=args.sphere_cfl,
                     cfl_visc=args.sphere_cfl)
    ctx = pmg.Context(0)
    mesh = pmg.Mesh(ctx, mesh_h)
    area = math.pi

    def solver(orders):
        top = int(orders.max())
        s = pmg.Solver(ctx, mesh, orders, phys,
                       pmg.MG(level_caps=list(range(top, 1, -1)), beta_pre=2, beta_post=2, beta_coarse=4))
        s.set_graph(True)
        return s

    def converge(s, Q, label):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cycles, r = 0, s.residual(Q, None, norm=True)[1]
        while r > args.sphere_tol and time.perf_counter() - t0 < args.sphere_s and r == r:
            r = s.vcycle(Q, None, n_cycles=args.sphere_chunk, norm=True)
            cycles += args.sphere_chunk
            if cycles % (10 * args.sphere_chunk) == 0:
                print(f"sphere-adapt {label}: {cycles} cycles, {time.perf_counter() - t0:.1f} s, residual {r:.3e}",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        cd = pmg.force_coefficients(s.wall_force(Q), area)[0]
        out = {"label": label, "dof": s.n_nodes, "cycles": cycles, "residual": r,
               "solve_s": round(time.perf_counter() - t0, 2), "cd": cd}
        print(f"sphere-adapt {label}: {out}", file=sys.stderr, flush=True)
        return out

    K = mesh_h.K
    runs = []
    if args.sphere_ref_cd:
        ref = {"label": "uniform N=6 (reference, earlier run)", "dof": 1712256, "cd": args.sphere_ref_cd}
    else:
        ref_orders = I.uniform_orders(K, (6, 6, 6))
        sr = solver(ref_orders)
        ref = converge(sr, sr.freestream(), "uniform N=6 (reference)")
        del sr
    P = I.uniform_orders(K, (4, 4, 4))
    s4 = solver(P)
    Q4 = s4.freestream()
    runs.append(converge(s4, Q4, "uniform N=4"))
    tau = s4.tau_estimate(Q4.clone(), None, isolated=True).cpu().numpy()
    vals = tau[np.isfinite(tau) & (tau > 0)]
    for q in args.sphere_quantiles:
        tau_max = float(np.quantile(vals, q))
        t0 = time.perf_counter()
        N, req = pmg.adapt_orders(mesh_h, P, tau, tau_max, (6, 6, 6), args.sphere_nmin, 2, True,
                                  with_required=True)
        sa = solver(N)
        Qa = pmg.remap_state(s4, Q4, sa)
        torch.cuda.synchronize()
        prep = time.perf_counter() - t0
        run = converge(sa, Qa, f"adapted tau_max={tau_max:.3e}")
        run.update({"tau_max": tau_max, "quantile": q, "max_required": req, "adapt_s": round(prep, 3),
                    "orders_hist": np.bincount(N.ravel(), minlength=8)[1:].tolist()})
        runs.append(run)
        del sa, Qa
    for r in runs + [ref]:
        r["cd_error"] = abs(r["cd"] - ref["cd"]) / ref["cd"]
    return {"metric": "sphere drag error vs DOF after tau-based adaptation", "value": None, "unit": "relative",
            "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "sphere, Re_D 200, Mach 0.2, six-panel O-grid 8x8x13 per panel (4992 hexes), "
                                   "outer radius 20, quadratic mapping", "tol": args.sphere_tol,
                       "adapt": f"isolated 3V map at P=4, n_min {args.sphere_nmin}, n_max 6, jump rule "
                                "floor(2N/3), wall conforming",
                       "levels": "max order .. 2, beta 2/2/4"},
            "reference": ref, "runs": runs}


def sphere_multistage_bench(args) -> dict:
    """The structure of the paper's multi-stage comparison on the sphere (Sec. 4.2, its Table 3), both runs
    through the library's driver (pmg_adapt_multistage): single-stage, converging uniform P = 6 before the one
    estimate and adaptation; multi-stage, stages (4, 6) from uniform 4 (orders capped at 6 after the first
    estimate, a second estimate and adaptation at the stage-6 orders when some element asks for more).  Same
    tau_max, n_max (6 by default), n_min = 4 (N >= 2M for the quadratic mapping), floor(2N/3) jump rule,
    conforming wall orders, stage solves to tau_max / 10, FMG start, levels down to order 2, final solve to
    the tolerance;
    wall time of each driver call and C_d of its result."""
    import math

    import numpy as np
    import torch

    from paper_1806_11456_amd import inputs as I
    from paper_1806_11456_amd import pmg

    mesh_h = I.ogrid_mesh(8, 13, r_out=20.0, ratio=1.25)
    phys = I.Physics(mach=0.2, reynolds=100.0, family=I.FAMILY_LG, cfl_adv=args.sphere_cfl,
                     cfl_visc=args.sphere_cfl)
    ctx = pmg.Context(0)
    mesh = pmg.Mesh(ctx, mesh_h)
    mg = pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4, fmg=1, fmg_threshold=1.0)
    K = mesh_h.K
    out = {}
    cases = (("single-stage", 6, (6,)), ("multi-stage", 4, (4, 6)))
    for label, first, stages in cases:
        print(f"sphere-multistage {label}: start", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the driver runs the stages and the carry-over (final_tol out of reach from above: no final cycles);
        # the final solve continues here in chunks, with progress lines, on a solver like the driver's
        N, Q, reps, _, _ = pmg.adapt_multistage(
            ctx, mesh, I.uniform_orders(K, (first,) * 3), phys, mg, stages, args.sphere_tau_max,
            (6, 6, 6), 4, 2,
            True, conv=0.1, final_tol=1e30, max_cycles=args.sphere_max_cycles, raise_not_converged=False,
            n_coarse=2)
        torch.cuda.synchronize()
        t_stages = time.perf_counter() - t0
        print(f"sphere-multistage {label}: stages done in {t_stages:.1f} s: {reps}", file=sys.stderr, flush=True)
        top = int(N.max())
        s = pmg.Solver(ctx, mesh, N, phys, pmg.MG(level_caps=list(range(top, 1, -1)), beta_pre=2, beta_post=2,
                                                beta_coarse=4))
        Q = Q.clone()
        cyc, res = 0, s.residual(Q, None, norm=True)[1]
        while res > args.sphere_tol and cyc < args.sphere_max_cycles and res == res:
            res = s.vcycle(Q, None, n_cycles=args.sphere_chunk, norm=True)
            cyc += args.sphere_chunk
            if cyc % (10 * args.sphere_chunk) == 0 or cyc <= 5 * args.sphere_chunk:
                print(f"sphere-multistage {label}: final solve {cyc} cycles, {time.perf_counter() - t0:.1f} s, "
                      f"residual {res:.3e}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cd = pmg.force_coefficients(s.wall_force(Q), math.pi)[0]
        out[label] = {"wall_s": round(wall, 2), "stages_s": round(t_stages, 2), "cd": cd, "final_cycles": cyc,
                      "final_residual": res,
                      "dof": int(Q.shape[1]), "orders_hist": np.bincount(N.ravel(), minlength=8)[1:].tolist(),
                      "stages": [{k: (int(v) if isinstance(v, (int, np.integer)) else float(v))
                                  for k, v in r.items()} for r in reps]}
        print(f"sphere-multistage {label}: {out[label]}", file=sys.stderr, flush=True)
        del s, Q
    ref = args.sphere_ref_cd or None
    for v in out.values():
        v["cd_error_vs_order6"] = abs(v["cd"] - ref) / ref if ref else None
    both = "single-stage" in out and "multi-stage" in out
    return {"metric": "multi-stage vs single-stage adaptation, sphere", "unit": "s", "higher_is_better": False,
            "value": (out["single-stage"]["wall_s"] / out["multi-stage"]["wall_s"]) if both else None,
            "value_meaning":
                "speed-up of the multi-stage run over the single-stage run (wall time of the driver calls)",
            "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "sphere, Re_D 200, Mach 0.2, six-panel O-grid 8x8x13 per panel (4992 hexes)",
                       "tau_max": args.sphere_tau_max, "tol": args.sphere_tol, "n_max": 6, "n_min": 4,
                       "jump_rule": "floor(2N/3)", "wall_conforming": True, "levels": "max .. 2",
                       "mg": "beta 2/2/4, FMG start (threshold 1.0)"},
            "order6_reference_cd": ref, "runs": out}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--beta", type=int, nargs=3, default=[2, 2, 4], metavar=("PRE", "POST", "COARSE"))
    ap.add_argument("--residual-loops", type=int, default=200)
    ap.add_argument("--residual-loops-batch", type=int, default=20)
    ap.add_argument("--ogrid-steps", type=int, default=10)
    ap.add_argument("--plate-steps", type=int, default=20)
    ap.add_argument("--lines", default="batch,ogrid,plate",
                    help="workloads, the first one is the headline: batch, ogrid, plate")
    ap.add_argument("--cpu-single-s", type=float, default=12.0)
    ap.add_argument("--cpu-rounds", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch-fp64", action="store_true", help="skip the FP64 run of the batch beside the mixed one")
    ap.add_argument("--serve", action="store_true", help="served-stream latency benchmark instead of the plate")
    ap.add_argument("--serve-n", type=int, default=24)
    ap.add_argument("--serve-kmin", type=int, default=64)
    ap.add_argument("--serve-kmax", type=int, default=400)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-precision", type=int, default=0)
    ap.add_argument("--serve-modes", default="per-request,batched",
                    help="served runs, in order: per-request (a solver per request, several streams), batched "
                         "(union solvers)")
    ap.add_argument("--serve-no-sequential", action="store_true")
    ap.add_argument("--solve", action="store_true", help="time to a converged plate solve instead of throughput")
    ap.add_argument("--solve-batch", action="store_true", help="progress of the 64-problem batch toward the tolerance")
    ap.add_argument("--solve-batch-chunk", type=int, default=25)
    ap.add_argument("--solve-batch-s", type=float, default=480.0)
    ap.add_argument("--solve-tol", type=float, default=1e-9)
    ap.add_argument("--solve-chunk", type=int, default=2000)
    ap.add_argument("--solve-max-cycles", type=int, default=400000)
    ap.add_argument("--solve-max-s", type=float, default=1000.0)
    ap.add_argument("--solve-precision", type=int, default=0)
    ap.add_argument("--solve-beta", type=int, nargs=3, default=[2, 2, 4], metavar=("PRE", "POST", "COARSE"))
    ap.add_argument("--solve-tuning", action="store_true", help="residual-based smoothing tuning (Sec. 3.1.2)")
    ap.add_argument("--solve-max-repeats", type=int, default=10)
    ap.add_argument("--solve-fmg", type=float, default=0.0, help="FMG start to this residual (Sec. 3.1.1)")
    ap.add_argument("--compare", action="store_true", help="RK3 against FAS: speed-up at equal residual")
    ap.add_argument("--sphere", action="store_true", help="sphere drag at Re_D 200 (soft physics check)")
    ap.add_argument("--sphere-order", type=int, default=4)
    ap.add_argument("--sphere-cfl", type=float, default=0.3)
    ap.add_argument("--sphere-s", type=float, default=240.0)
    ap.add_argument("--sphere-chunk", type=int, default=200)
    ap.add_argument("--sphere-tol", type=float, default=1e-7)
    ap.add_argument("--sphere-adapt", action="store_true", help="sphere drag error vs DOF after adaptation")
    ap.add_argument("--sphere-quantiles", type=float, nargs="+", default=[0.3, 0.6, 0.9])
    ap.add_argument("--sphere-nmin", type=int, default=4)
    ap.add_argument("--sphere-ref-cd", type=float, default=0.0)
    ap.add_argument("--sphere-multistage", action="store_true", help="multi-stage vs single-stage adaptation")
    ap.add_argument("--sphere-tau-max", type=float, default=2.761e-2)
    ap.add_argument("--sphere-max-cycles", type=int, default=40000)
    ap.add_argument("--compare-s", type=float, default=40.0)
    ap.add_argument("--compare-case", default="plate", choices=["plate", "sphere"])
    ap.add_argument("--compare-tol", type=float, default=1e-9)
    ap.add_argument("--compare-paper-beta", type=int, nargs=3, default=[100, 100, 400])
    ap.add_argument("--compare-paper-chunk", type=int, default=5)
    ap.add_argument("--compare-rk-chunk", type=int, default=1000)
    ap.add_argument("--compare-fas-chunk", type=int, default=20)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
                  f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        return 2

    if args.serve:
        print(json.dumps(serve_bench(args)), flush=True)
        return 0
    if args.solve:
        print(json.dumps(solve_bench(args)), flush=True)
        return 0
    if args.solve_batch:
        print(json.dumps(solve_batch_bench(args)), flush=True)
        return 0
    if args.compare:
        print(json.dumps(compare_bench(args)), flush=True)
        return 0
    if args.sphere:
        print(json.dumps(sphere_bench(args)), flush=True)
        return 0
    if args.sphere_adapt:
        print(json.dumps(sphere_adapt_bench(args)), flush=True)
        return 0
    if args.sphere_multistage:
        print(json.dumps(sphere_multistage_bench(args)), flush=True)
        return 0

    from paper_1806_11456_amd import inputs as I

    lines = [x for x in args.lines.split(",") if x]
    assert lines and all(x in ("batch", "ogrid", "plate") for x in lines), args.lines
    head = lines[0]
    wls = I.config_batch() if "batch" in lines else None
    cpu = None
    if not args.no_cpu and head == "batch":
        # before the GPU is touched: forked oracle workers
        cpu = cpu_baseline([(w.mesh, w.orders, w.phys, w.Q) for w in wls], args.cpu_single_s, args.cpu_rounds)
    elif not args.no_cpu:
        wl = I.config_ogrid() if head == "ogrid" else I.config_plate()
        cpu = cpu_baseline([(wl.mesh, wl.orders, wl.phys, wl.Q)], args.cpu_single_s, args.cpu_rounds)

    import torch

    results = {}
    for name in lines:
        fn = {"batch": lambda: batch_line(args, wls), "ogrid": lambda: ogrid_line(args), "plate": lambda: plate_line(args)}
        results[name] = fn[name]()
        print(f"{name}: {results[name]['value']:.4g} DOF-residual evals/s, {results[name]['ms_per_step']:.2f} ms/step, "
              f"roofline frac {results[name]['roofline']['frac']:.3f}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    h = results[head]
    dtype = {"batch": "f64/f32 (FP64 finest level and checks, FP32 coarse-level smoothing)", "ogrid": "f64",
             "plate": "f64"}[head]
    steps = args.steps if head == "batch" else (args.ogrid_steps if head == "ogrid" else args.plate_steps)
    out = {
        "metric": "fine-level DOF-residual evals/s",
        "value": h["value"],
        "unit": "DOF-residual evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup if head == "batch" else (1 if head == "ogrid" else 2),
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": h["config"],
        "roofline": h["roofline"],
        "flops": h["flops"],
        "residual_only": h["residual_only"],
        "lines": {k: v for k, v in results.items() if k != head},
    }
    for k in ("guard_halvings", "problems_halved", "problems_given_up", "cycles_run", "fp32_cycles_min",
              "residual_max", "mixed", "fp64"):
        if k in h:
            out[k] = h[k]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
