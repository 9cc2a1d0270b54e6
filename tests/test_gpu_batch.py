"""Batching, graph capture and tile autotuning on the GPU.

A batch advances independent problems together in one union solver; every problem's arithmetic is the
same as in its own solve, so results must agree bitwise with solving each problem alone.  Captured-graph
replays must agree bitwise with eager launches, replay after replay.
"""
import numpy as np
import pytest

from paper_1806_11456_amd import inputs as I
from tests.gpu_util import check, np_

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1806_11456_amd import pmg
    assert torch.cuda.is_available()
    return pmg.Context(0)


@pytest.fixture(scope="module")
def problems():
    return I.config_batch(n=4, kmin=20, kmax=60, seed=7)


MG = dict(beta_pre=2, beta_post=1, beta_coarse=3)


@pytest.fixture(scope="module")
def batch(ctx, problems):
    from paper_1806_11456_amd import pmg
    meshes = [pmg.Mesh(ctx, w.mesh) for w in problems]
    b = pmg.Batch(ctx, meshes, [w.orders for w in problems], [w.phys for w in problems], pmg.MG(**MG))
    singles = [pmg.Solver(ctx, m, w.orders, w.phys, pmg.MG(**MG)) for m, w in zip(meshes, problems)]
    return b, singles


def batch_state(b, problems):
    return b.tensor(np.concatenate([w.Q for w in problems], axis=1))


def test_batch_layout(batch, problems):
    b, singles = batch
    assert b.n == len(problems)
    assert b.n_nodes == sum(w.n_nodes for w in problems)
    assert list(np.diff(b.problem_offsets)) == [w.n_nodes for w in problems]


def test_batch_residual_equals_single(batch, problems):
    b, singles = batch
    Q = batch_state(b, problems)
    R = b.residual(Q)
    norms = b.norms(Q)
    for p, (s, w) in enumerate(zip(singles, problems)):
        Rs, ns = s.residual(s.tensor(w.Q), norm=True)
        assert np.array_equal(np_(b.part(R, p)), np_(Rs)), p
        assert norms[p] == ns


def test_batch_residual_parity_oracle(batch, problems):
    from oracle import oracle as O
    b, _ = batch
    R = np_(b.residual(batch_state(b, problems)))
    for p, w in enumerate(problems):
        A, sc = O.Oracle(w.mesh, w.phys).operator_scale(w.orders, w.Q)
        check(R[:, b.problem_offsets[p]:b.problem_offsets[p + 1]], -A, sc, 1e-12, f"batch problem {p}")


def test_batch_vcycle_and_tau_equal_single(batch, problems):
    b, singles = batch
    Q = batch_state(b, problems)
    b.vcycle(Q, None, n_cycles=2)
    Qt = batch_state(b, problems)
    tau = np_(b.tau_estimate(Qt, None, isolated=True))
    K0 = 0
    for p, (s, w) in enumerate(zip(singles, problems)):
        Qs = s.tensor(w.Q)
        s.vcycle(Qs, None, n_cycles=2)
        assert np.array_equal(np_(b.part(Q, p)), np_(Qs)), p
        Qs2 = s.tensor(w.Q)
        ts = np_(s.tau_estimate(Qs2, None, isolated=True))
        tb = tau[K0:K0 + w.mesh.K, :, :ts.shape[2]]
        assert np.array_equal(np.isnan(tb), np.isnan(ts))
        assert np.array_equal(tb[~np.isnan(ts)], ts[~np.isnan(ts)]), p
        assert np.array_equal(np_(b.part(Qt, p)), np_(Qs2)), p
        K0 += w.mesh.K


def test_batch_solve_freezes_converged_problems(batch, problems):
    """Each problem stops at its own tolerance crossing, exactly as when solved alone."""
    b, singles = batch
    Q = batch_state(b, problems)
    r0 = b.norms(Q)
    tol = float(np.median(r0)) * 0.3
    cyc, r = b.solve_all(Q, None, tol=tol, max_cycles=6, raise_not_converged=False)
    for p, (s, w) in enumerate(zip(singles, problems)):
        Qs = s.tensor(w.Q)
        cs, rs = s.solve(Qs, None, tol=tol, max_cycles=6, raise_not_converged=False)
        assert cs == cyc[p], (p, cs, cyc[p])
        assert rs == r[p]
        assert np.array_equal(np_(b.part(Q, p)), np_(Qs)), p


def test_graph_replays_equal_eager(ctx, problems):
    import torch
    from paper_1806_11456_amd import pmg
    w = problems[0]
    mesh = pmg.Mesh(ctx, w.mesh)
    eager = pmg.Solver(ctx, mesh, w.orders, w.phys, pmg.MG(**MG))
    graph = pmg.Solver(ctx, mesh, w.orders, w.phys, pmg.MG(**MG))
    graph.set_graph(True)
    Qe = eager.tensor(w.Q)
    Qg = graph.tensor(w.Q)
    for rep in range(3):
        eager.vcycle(Qe, None, n_cycles=1)
        graph.vcycle(Qg, None, n_cycles=1)
        torch.cuda.synchronize()
        # eager work between replays
        eager.residual(Qe)
        torch.cuda.synchronize()
        assert np.array_equal(np_(Qe), np_(Qg)), rep
    te = np_(eager.tau_estimate(Qe, None, isolated=True))
    for rep in range(2):
        Qg2 = Qg.clone()
        tg = np_(graph.tau_estimate(Qg2, None, isolated=True))
        torch.cuda.synchronize()
        assert np.array_equal(np.isnan(te), np.isnan(tg))
        assert np.array_equal(te[~np.isnan(te)], tg[~np.isnan(tg)]), rep
    # a batch in graph mode
    b = pmg.Batch(ctx, [mesh, pmg.Mesh(ctx, problems[1].mesh)], [w.orders, problems[1].orders],
                  [w.phys, problems[1].phys], pmg.MG(**MG))
    b.set_graph(True)
    Qb = b.tensor(np.concatenate([w.Q, problems[1].Q], axis=1))
    b.vcycle(Qb, None, n_cycles=2)
    Qs = eager.tensor(w.Q)
    eager.vcycle(Qs, None, n_cycles=2)
    assert np.array_equal(np_(b.part(Qb, 0)), np_(Qs))


def test_autotune_keeps_results(ctx, problems):
    from paper_1806_11456_amd import pmg
    w = problems[2]
    s = pmg.Solver(ctx, pmg.Mesh(ctx, w.mesh), w.orders, w.phys, pmg.MG(**MG))
    R0 = np_(s.residual(s.tensor(w.Q)))
    s.autotune()
    for l in range(s.level_info(-1)):
        assert s.level_tiles(-1, l) in (32, 64, 128, 256, 512)
    R1 = np_(s.residual(s.tensor(w.Q)))
    assert np.array_equal(R0, R1)


def _set_all_tiles(s, target, split, hierarchies=(-1,)):
    for h in hierarchies:
        for l in range(s.level_info(h)):
            s.set_tiles(h, l, target, split)
            assert s.level_tile_choice(h, l) == (target, split)


TILE_CHOICES = [(t, sp) for t in (32, 64, 128, 256, 512) for sp in range(4)]


def test_tile_choices_bitwise_batch(ctx, problems):
    """Every element-tile node target, launched as one grid or per size class, gives bitwise the same residual,
    per-problem norms (per-tile partials reduced per problem over every class) and V-cycle of a batch."""
    from paper_1806_11456_amd import pmg
    meshes = [pmg.Mesh(ctx, w.mesh) for w in problems]
    b = pmg.Batch(ctx, meshes, [w.orders for w in problems], [w.phys for w in problems], pmg.MG(**MG))
    ref = None
    for target, split in TILE_CHOICES:
        _set_all_tiles(b, target, split)
        Q = batch_state(b, problems)
        R = np_(b.residual(Q))
        norms = np.asarray(b.norms(Q))
        b.vcycle(Q, None, n_cycles=1)
        out = (R, norms, np_(Q))
        print(f"[tiles] batch target {target} split {split}", flush=True)
        if ref is None:
            assert all(np.isfinite(x).all() for x in out)
            ref = out
            continue
        for a, r, what in zip(out, ref, ("residual", "norms", "state after a V-cycle")):
            assert np.array_equal(a, r), (target, split, what, float(np.nanmax(np.abs(a - r))))


def test_tile_choices_bitwise_ogrid(ctx):
    """The same on an O-grid with orders 1..7 (tiles up to 512 nodes: 512-thread blocks), including the
    truncation-error estimate of the anisotropic hierarchies."""
    from paper_1806_11456_amd import pmg
    w = I.config_ogrid(nt=2, nr=3, r_out=3.0, ratio=1.2)
    s = pmg.Solver(ctx, pmg.Mesh(ctx, w.mesh), w.orders, w.phys,
                   pmg.MG(beta_pre=1, beta_post=1, beta_coarse=2))
    ref = None
    for target, split in TILE_CHOICES:
        _set_all_tiles(s, target, split)
        Q = s.tensor(w.Q)
        R = np_(s.residual(Q))
        s.vcycle(Q, None, n_cycles=1)
        tau = np_(s.tau_estimate(Q, None, isolated=False))
        _set_all_tiles(s, target, split, hierarchies=(0, 1, 2))
        tau2 = np_(s.tau_estimate(Q, None, isolated=True))
        out = (R, np_(Q), tau, tau2)
        print(f"[tiles] ogrid target {target} split {split}", flush=True)
        if ref is None:
            assert np.isfinite(R).all() and np.isfinite(out[1]).all()
            assert np.isfinite(tau).any() and np.isfinite(tau2).any()
            ref = out
            continue
        # unrecorded truncation-error entries are NaN on every choice
        for a, r, what in zip(out, ref, ("residual", "state after a V-cycle", "tau", "isolated tau")):
            assert np.array_equal(a, r, equal_nan=True), (target, split, what, float(np.nanmax(np.abs(a - r))))


def test_determinism_run_twice(ctx, problems):
    """The same calls from the same state give bitwise the same results, on the same solver and on a second
    one built alike (no atomics in floating-point accumulations; reductions in a fixed order)."""
    from paper_1806_11456_amd import pmg
    meshes = [pmg.Mesh(ctx, w.mesh) for w in problems]
    out = []
    for run in range(3):
        if run in (0, 2):  # runs 0 and 1 on one solver, run 2 on a second one
            b = pmg.Batch(ctx, meshes, [w.orders for w in problems], [w.phys for w in problems],
                          pmg.MG(precision=1, **MG))
        Q = batch_state(b, problems)
        R = np_(b.residual(Q))
        b.vcycle(Q, None, n_cycles=2)
        tau = np_(b.tau_estimate(Q.clone(), None, isolated=False))
        out.append((R, np_(Q), tau, np.asarray(b.norms(Q))))
        print(f"[determinism] run {run}", flush=True)
    for run in (1, 2):
        for a, r, what in zip(out[run], out[0], ("residual", "state", "tau map", "norms")):
            assert np.array_equal(a, r, equal_nan=True), (run, what)
