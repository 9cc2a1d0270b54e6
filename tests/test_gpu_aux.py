"""Nodal truncation error, residual history and checkpoint / resume on the GPU.

* The pointwise truncation error of one anisotropic level matches the oracle's (isolated and not), on a
  Lobatto box and on a rotated curved box with random orders (mortars).
* The residual history of a solve starts at the initial residual and ends at the returned one.
* A state restored from a checkpoint continues bitwise like the one that was saved; a damaged or foreign
  checkpoint is refused.
"""
import numpy as np
import pytest

from paper_1806_11456_amd import inputs as I
from tests.gpu_util import derived_bar, np_, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()
MG = dict(beta_pre=1, beta_post=1, beta_coarse=2)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1806_11456_amd import pmg
    assert torch.cuda.is_available()
    return pmg.Context(0)


@pytest.mark.parametrize("isolated", [False, True])
@pytest.mark.parametrize("name", ["box_lgl", "curved_lg"])
def test_tau_nodal_parity(ctx, name, isolated):
    from oracle import oracle as O
    from paper_1806_11456_amd import pmg
    wl = CASES[name]
    s = pmg.Solver(ctx, pmg.Mesh(ctx, wl.mesh), wl.orders, wl.phys, pmg.MG(**MG))
    o = O.Oracle(wl.mesh, wl.phys)
    rng = np.random.default_rng(4)
    S = 0.1 * rng.uniform(-1, 1, size=wl.Q.shape)
    for d in range(3):
        pmax = int(wl.orders[:, d].max())
        for order in sorted({1, pmax - 1}):
            if order < 1 or order >= pmax:
                continue
            Q = s.tensor(wl.Q)
            tg = np_(s.tau_nodal(Q, s.tensor(S), d=d, order=order, isolated=isolated))
            o.take_eval_count()
            to, Qo = o.tau_nodal(wl.orders, wl.Q, S, d=d, cap=order, isolated=int(isolated), **MG)
            # tau = S - A(I Q~): the operator bar plus the state bar carried through A
            _, tbar = derived_bar(o, wl, o.take_eval_count())
            err = np.abs(tg - to).max()
            print(f"[parity] {name} tau nodal d={d} order={order} iso={isolated}: error / bar {err / tbar:.2e}")
            assert err <= tbar, (d, order, err, tbar)


def test_history_and_checkpoint(ctx, tmp_path):
    import torch
    from paper_1806_11456_amd import pmg
    wl = I.config_batch(n=1, kmin=30, kmax=40, seed=13)[0]
    mesh = pmg.Mesh(ctx, wl.mesh)
    mg = pmg.MG(beta_pre=2, beta_post=2, beta_coarse=4)
    a = pmg.Solver(ctx, mesh, wl.orders, wl.phys, mg)
    Q = a.tensor(wl.Q)
    r0 = a.residual(Q, None, norm=True)[1]
    cyc, r = a.solve(Q, None, tol=1e-30, max_cycles=7, raise_not_converged=False)
    h = a.history()
    assert len(h) == cyc + 1 and h[0] == r0 and h[-1] == r
    assert a.cycle_count() == 7
    path = tmp_path / "state.ckpt"
    a.checkpoint(path, Q)
    saved = Q.clone()
    a.vcycle(Q, None, n_cycles=3)
    # another solver of the same problem resumes from the file
    b = pmg.Solver(ctx, mesh, wl.orders, wl.phys, mg)
    Qb = torch.zeros_like(Q)
    b.restore(path, Qb)
    assert torch.equal(Qb, saved)
    assert b.cycle_count() == 7 and np.array_equal(b.history(), h)
    b.vcycle(Qb, None, n_cycles=3)
    assert np.array_equal(np_(Qb), np_(Q))
    # damaged file
    raw = bytearray(path.read_bytes())
    raw[100] ^= 1
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(bytes(raw))
    with pytest.raises(pmg.PmgError, match="checksum"):
        b.restore(bad, Qb)
    # a checkpoint of another problem
    other = CASES["box_lgl"]
    c = pmg.Solver(ctx, pmg.Mesh(ctx, other.mesh), other.orders, other.phys, mg)
    with pytest.raises(pmg.PmgError, match="another problem"):
        c.restore(path, c.tensor(other.Q))
