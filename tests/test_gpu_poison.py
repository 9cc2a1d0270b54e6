"""Debug mode PMG_POISON=1: every device allocation starts as all-ones bytes (NaN in FP64 and FP32).  Results
computed with poisoned allocations equal those without, bitwise -- no kernel reads memory that nothing has
written (residual, smoothing, FP64 and mixed V-cycles, the truncation-error map, a guarded batched solve).
"""
import os

import numpy as np
import pytest

from paper_1806_11456_amd import inputs as I
from tests.gpu_util import np_, small_cases

pytestmark = pytest.mark.gpu

MG = dict(beta_pre=2, beta_post=1, beta_coarse=3)


def _run(ctx, poison):
    from paper_1806_11456_amd import pmg
    old = os.environ.get("PMG_POISON")
    os.environ["PMG_POISON"] = "1" if poison else "0"
    try:
        out = []
        for name in ("ogrid2x2", "curved_lg", "plate8x4"):
            wl = small_cases()[name]
            mesh = pmg.Mesh(ctx, wl.mesh)
            for prec in (0, 1):
                s = pmg.Solver(ctx, mesh, wl.orders, wl.phys, pmg.MG(precision=prec, **MG))
                Q = s.tensor(wl.Q)
                out.append(np_(s.residual(Q)))
                s.smooth(Q, None, sweeps=1)
                s.vcycle(Q, None, n_cycles=2)
                out.append(np_(Q))
                out.append(np_(s.tau_estimate(Q.clone(), None, isolated=False)))
        probs = I.config_batch(n=3, kmin=20, kmax=60, seed=7)
        b = pmg.Batch(ctx, [pmg.Mesh(ctx, w.mesh) for w in probs], [w.orders for w in probs],
                      [w.phys for w in probs], pmg.MG(precision=1, guard=4, **MG))
        Qb = b.tensor(np.concatenate([w.Q for w in probs], axis=1))
        cyc, r = b.solve_all(Qb, None, tol=1e-30, max_cycles=4, raise_not_converged=False)
        out += [np_(Qb), np.asarray(r)]
        return out
    finally:
        if old is None:
            os.environ.pop("PMG_POISON", None)
        else:
            os.environ["PMG_POISON"] = old


def test_poisoned_allocations_change_nothing():
    import torch
    from paper_1806_11456_amd import pmg
    assert torch.cuda.is_available()
    ctx = pmg.Context(0)
    clean = _run(ctx, False)
    poisoned = _run(ctx, True)
    assert len(clean) == len(poisoned)
    for k, (a, b) in enumerate(zip(clean, poisoned)):
        assert np.array_equal(a, b, equal_nan=True), k
        assert np.isfinite(a[~np.isnan(a)]).all()
