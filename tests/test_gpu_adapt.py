"""p-adaptation on the GPU: the adapted orders in use, the carry-over and the multi-stage driver against the
oracle (the host selection against random maps is in test_adapt_host.py).

* The maps of the GPU's own anisotropic 3V cycle (a curved random-order box; the full-size plate): both
  adapt them to the same orders.
* A solver built on the adapted, p-nonconforming orders reproduces the oracle's residual (the parity bar).
"""
import time

import numpy as np
import pytest

from paper_1806_11456_amd import inputs as I
from tests.gpu_util import check, derived_bar, gpu_pair, np_, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1806_11456_amd import pmg
    assert torch.cuda.is_available()
    return pmg.Context(0)


def test_gpu_map_adapted_and_used(ctx):
    """Map of the GPU 3V cycle -> the same orders on both sides -> a solver on them at parity."""
    from oracle import adapt as A
    from paper_1806_11456_amd import pmg
    wl = CASES["curved_lg"]
    mg = pmg.MG(beta_pre=1, beta_post=1, beta_coarse=2)
    s, _ = gpu_pair(ctx, wl, mg)
    rng = np.random.default_rng(7)
    S = 0.1 * rng.uniform(-1, 1, size=wl.Q.shape)
    tau = np_(s.tau_estimate(s.tensor(wl.Q), s.tensor(S), isolated=True))
    vals = tau[np.isfinite(tau) & (tau > 0)]
    tau_max = float(np.quantile(vals, 0.5)) * 3.0
    got = pmg.adapt_orders(wl.mesh, wl.orders, tau, tau_max, (7, 7, 7), 1, 1)
    want = A.adapt_orders(wl.mesh, wl.orders, tau, tau_max, (7, 7, 7), 1, 1)
    assert np.array_equal(got, want)
    assert (got != wl.orders).any()  # the orders did change
    # the adapted discretisation: residual of a perturbed state against the oracle
    nn = int(I.node_offsets(got)[-1])
    new = I.Workload(wl.name + "_adapted", wl.mesh, got.astype(np.int32), wl.phys,
                     I.perturbed_freestream(nn, wl.phys.mach, 0.02, 29))
    s2, o2 = gpu_pair(ctx, new)
    S2 = rng.uniform(-1, 1, size=new.Q.shape)
    Rg = np_(s2.residual(s2.tensor(new.Q), s2.tensor(S2)))
    A2, scale = o2.operator_scale(new.orders, new.Q)
    check(Rg, S2 - A2, scale, 1e-12, "residual on the adapted orders")


def test_full_size_plate_adaptation(ctx):
    """The full plate (2048 elements, P = (6, 6, 1)): the map of one isolated 3V cycle adapted on both sides."""
    from oracle import adapt as A
    from paper_1806_11456_amd import pmg
    wl = I.config_plate()
    s = pmg.Solver(ctx, pmg.Mesh(ctx, wl.mesh), wl.orders, wl.phys, pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4))
    tau = np_(s.tau_estimate(s.tensor(wl.Q), None, isolated=True))
    assert np.isnan(tau[:, 2]).all() and np.isfinite(tau[:, :2, :5]).all()
    vals = tau[np.isfinite(tau) & (tau > 0)]
    for q in (0.1, 0.5, 0.9):
        tau_max = float(np.quantile(vals, q))
        t0 = time.perf_counter()
        got = pmg.adapt_orders(wl.mesh, wl.orders, tau, tau_max, (7, 7, 7), 2, 1)
        t_lib = time.perf_counter() - t0
        want = A.adapt_orders(wl.mesh, wl.orders, tau, tau_max, (7, 7, 7), 2, 1)
        assert np.array_equal(got, want), q
        assert (got[:, 2] == 1).all()
        dof = int(I.node_offsets(got)[-1])
        print(f"plate adaptation tau_max={tau_max:.3e}: {1e3 * t_lib:.2f} ms, DOF {dof} (was {s.n_nodes})")


# ---- the state carried over to new orders, and the multi-stage driver ----------------------------------------

def _min_margin(P, tau, tau_max, n_max, n_min):
    """Smallest |sum - tau_max| / tau_max over every candidate sum the selection compares (oracle tables): a
    decision both sides take from maps that differ by round-off is safe when this is far above it."""
    import itertools
    from oracle import adapt as A
    worst = np.inf
    for e in range(P.shape[0]):
        inner, full = A.directional_table([int(v) for v in P[e]], tau[e], list(n_max), n_min)
        for tables in (inner, full):
            c = [[(int(P[e][d]), 0.0)] if tables[d] is None else sorted(tables[d].items()) for d in range(3)]
            for x, y, z in itertools.product(*c):
                worst = min(worst, abs(x[1] + y[1] + z[1] - tau_max) / tau_max)
    return worst


@pytest.mark.parametrize("name", ["curved_lg", "plate_full"])
def test_remap_matches_oracle(ctx, name):
    """Random new orders (rising in some directions and falling in others inside one element): every value."""
    from oracle import oracle as O
    from paper_1806_11456_amd import pmg
    wl = I.config_plate() if name == "plate_full" else CASES[name]
    rng = np.random.default_rng(17)
    K = wl.mesh.K
    B = rng.integers(1, 8, size=(K, 3)).astype(np.int32)
    if name == "plate_full":
        B[:, 2] = 1
    mesh = pmg.Mesh(ctx, wl.mesh)
    sa = pmg.Solver(ctx, mesh, wl.orders, wl.phys, pmg.MG(level_caps=[int(wl.orders.max())]))
    sb = pmg.Solver(ctx, mesh, B, wl.phys, pmg.MG(level_caps=[int(B.max())]))
    Q = rng.uniform(0.5, 1.5, size=wl.Q.shape) * wl.Q
    got = np_(pmg.remap_state(sa, sa.tensor(Q), sb))
    want = O.Oracle(wl.mesh, wl.phys).remap(wl.orders, B, Q)
    check(got, want, None, 1e-13, f"{name} remap")


def test_remap_mesh_checks(ctx):
    """Two handles of identical mesh data count as one mesh (same result as one handle); a different mesh is
    rejected."""
    from paper_1806_11456_amd import pmg
    wl = CASES["curved_lg"]
    B = np.random.default_rng(3).integers(1, 8, size=(wl.mesh.K, 3)).astype(np.int32)
    m1, m2 = pmg.Mesh(ctx, wl.mesh), pmg.Mesh(ctx, wl.mesh)
    sa = pmg.Solver(ctx, m1, wl.orders, wl.phys, pmg.MG(level_caps=[7]))
    sb1 = pmg.Solver(ctx, m1, B, wl.phys, pmg.MG(level_caps=[7]))
    sb2 = pmg.Solver(ctx, m2, B, wl.phys, pmg.MG(level_caps=[7]))
    Q = sa.tensor(wl.Q)
    assert np.array_equal(np_(pmg.remap_state(sa, Q, sb1)), np_(pmg.remap_state(sa, Q, sb2)))
    other = CASES["ogrid2x2"]
    so = pmg.Solver(ctx, pmg.Mesh(ctx, other.mesh), other.orders, other.phys, pmg.MG(level_caps=[7]))
    with pytest.raises(pmg.PmgError, match="same mesh"):
        pmg.remap_state(sa, Q, so)


def test_multistage_matches_oracle(ctx):
    """Small plate, stages (3, 5, 6) from free stream with FMG: the orders of every stage, the reports and the
    final state equal the oracle's driver.  Each solve runs its max_cycles (tolerances out of reach), so both
    sides take the same steps; the decision margins are checked on the oracle's maps.  n_min = 2: with
    order-1 elements next to the wall the smoother's transient amplifies round-off by orders of magnitude (a
    1e-13 change of the start moves the stage residuals by 1e-5 .. 1e-3 in the oracle alone), so no parity bar
    holds there; with n_min = 2 the same change stays below 1e-12 in the final state."""
    from oracle import adapt as A
    from oracle import oracle as O
    from paper_1806_11456_amd import pmg
    wl = CASES["plate8x4"]
    K = wl.mesh.K
    first = I.uniform_orders(K, (3, 3, 1))
    stages, tau_max, n_max, n_min = (3, 5, 6), 1.0, (6, 6, 6), 2
    mg = dict(beta_pre=2, beta_post=2, beta_coarse=4, fmg=1, fmg_threshold=1e30)
    o = O.Oracle(wl.mesh, wl.phys)
    maps, solved = [], []
    select, solve = A.select_orders, o.solve

    def recording(mesh, N, tau, *a, **k):
        maps.append((N.copy(), tau.copy()))
        return select(mesh, N, tau, *a, **k)

    total = [0]  # oracle operator evaluations so far

    def recording_solve(N, *a, **k):
        out = solve(N, *a, **k)
        total[0] += o.take_eval_count()
        solved.append((np.array(N), out[0].copy(), total[0]))
        return out

    A.select_orders, o.solve = recording, recording_solve
    o.take_eval_count()
    try:
        Q0 = I.freestream_state(int(np.prod(first + 1, axis=1).sum()), wl.phys.mach)
        No, Qo, ro, co, reso = A.multistage(o, wl.mesh, first, stages, tau_max, n_max, n_min=n_min, rule=1,
                                            conv=1e-9, final_tol=1e-30, max_cycles=2, Q0=Q0, **mg)
    finally:
        A.select_orders, o.solve = select, solve
    total[0] += o.take_eval_count()
    for P, tau in maps:
        assert _min_margin(P, tau, tau_max, n_max, n_min) > 1e-6
    # the first stage's carry-over lowers some elements and raises others (to the next stage's cap)
    assert (maps[1][0] < 3).any() and (maps[1][0] == 5).any()
    Ng, Qg, rg, cg, resg = pmg.adapt_multistage(ctx, pmg.Mesh(ctx, wl.mesh), first, wl.phys, pmg.MG(**mg), stages,
                                                tau_max, n_max, n_min, 1, False, conv=1e-9, final_tol=1e-30,
                                                max_cycles=2, raise_not_converged=False)
    assert np.array_equal(Ng, No)
    assert len(rg) == len(ro) >= 2 and cg == co

    def bars(N, Q, n_evals):
        """(per-variable state scale, bar of a residual entry) of a state after the oracle's n_evals operator
        evaluations so far (an upper bound for each stage)."""
        return derived_bar(o, I.Workload("stage", wl.mesh, N, wl.phys, Q), n_evals)

    for i, (g, w) in enumerate(zip(rg, ro)):
        assert (g["stage_order"], g["cycles"], g["max_required"], bool(g["last"]), g["nodes_before"],
                g["nodes_after"]) == (w["order"], w["cycles"], w["max_required"], w["last"], w["dof_before"],
                                      w["dof_after"])
        _, rbar = bars(*solved[i])
        print(f"[parity] multi-stage stage {i} residual: error / bar {abs(g['res_inf'] - w['res']) / rbar:.2e}")
        assert abs(g["res_inf"] - w["res"]) <= rbar, (i, g["res_inf"], w["res"], rbar)
    ss, rbar = bars(No, Qo, total[0])
    check(np_(Qg), Qo, ss, 1e-12, "multi-stage final state")
    print(f"[parity] multi-stage final residual: error / bar {abs(resg - reso) / rbar:.2e}")
    assert abs(resg - reso) <= rbar


def test_multistage_invalid_arguments(ctx):
    from paper_1806_11456_amd import pmg
    wl = CASES["plate8x4"]
    mesh = pmg.Mesh(ctx, wl.mesh)
    first = I.uniform_orders(wl.mesh.K, (2, 2, 1))
    with pytest.raises(pmg.PmgError, match="increase"):
        pmg.adapt_multistage(ctx, mesh, first, wl.phys, pmg.MG(), (4, 2), 1.0)
    with pytest.raises(pmg.PmgError, match="level_caps"):
        pmg.adapt_multistage(ctx, mesh, first, wl.phys, pmg.MG(level_caps=[2, 1]), (2, 4), 1.0)


def test_full_size_plate_multistage(ctx):
    """The full plate from (3, 3, 1) through stages (3, 5, 6) with n_min = 2: stage caps, the jump rule across
    every face and a finite final state; prints the time of the whole run and each stage's report."""
    from oracle import adapt as A
    from paper_1806_11456_amd import pmg
    import torch
    wl = I.config_plate()
    mesh = pmg.Mesh(ctx, wl.mesh)
    first = I.uniform_orders(wl.mesh.K, (3, 3, 1))
    mg = pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4, fmg=1, fmg_threshold=1e30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    N, Q, reps, cyc, res = pmg.adapt_multistage(ctx, mesh, first, wl.phys, mg, (3, 5, 6), 1.0, (6, 6, 6), 2, 1,
                                                False, conv=1e-9, final_tol=1e-30, max_cycles=3,
                                                raise_not_converged=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    assert (N[:, 2] == 1).all() and N.max() <= 6 and N[:, :2].min() >= 2
    assert A.enforce_jumps(wl.mesh, N, 1).tolist() == N.tolist()  # already a fixed point of the rule
    assert torch.isfinite(Q).all()
    for r in reps:
        print(f"stage P={r['stage_order']}: cycles {r['cycles']}, |r| {r['res_inf']:.3e}, nodes "
              f"{r['nodes_before']} -> {r['nodes_after']}, max required {r['max_required']}, last {r['last']}")
    print(f"plate multi-stage: {1e3 * t:.1f} ms in all, final cycles {cyc}, |r| {res:.3e}, nodes {Q.shape[1]}")
