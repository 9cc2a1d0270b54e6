"""Shared helpers of the GPU parity tests: solver/oracle pairs on the same seeded inputs and the parity bar.

The bar (FP64): for every variable v, max |X_gpu - X_oracle| <= tol * max(max |X_oracle,v|, s_v), with
s_v the largest round-off scale of that variable -- for an operator output the sum of the magnitudes of the
terms that make it up (from the oracle), for a state max |Q_v|.
"""
from __future__ import annotations

import numpy as np

from paper_1806_11456_amd import inputs as I


def gpu_pair(ctx, wl, mg=None):
    from oracle import oracle as O
    from paper_1806_11456_amd import pmg
    mesh = pmg.Mesh(ctx, wl.mesh)
    s = pmg.Solver(ctx, mesh, wl.orders, wl.phys, mg or pmg.MG())
    return s, O.Oracle(wl.mesh, wl.phys)


def np_(t):
    return t.detach().cpu().numpy()


def check(got, ref, scale=None, tol=1e-12, what=""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    g = got.reshape(got.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    nv = g.shape[0]
    dens = np.abs(r).max(axis=1)
    if scale is not None:
        dens = np.maximum(dens, np.asarray(scale).reshape(nv, -1).max(axis=1))
    if nv == 5:
        # momentum is one vector: round-off of the metric terms (curl form of absolute coordinates) moves
        # error between its Cartesian components, so they share the momentum scale
        dens[1:4] = dens[1:4].max()
    worst = 0.0
    for v in range(nv):
        den = dens[v]
        err = np.abs(g[v] - r[v]).max()
        rel = err / den if den > 0 else err
        worst = max(worst, rel)
        assert rel <= tol, f"{what}: variable {v} relative error {rel:.3e} > {tol:.0e} (err {err:.3e}, den {den:.3e})"
    return worst


def small_cases():
    """Small workloads spanning the code paths: Lobatto periodic box; Gauss stretched plate with walls and
    self-periodic faces; rotated cubed-sphere O-grid with random orders 1..7 (mortars, every orientation
    code, wall and far field); rotated curved periodic box with random orders (Gauss and Lobatto)."""
    cases = {}
    cases["box_lgl"] = I.config_box()
    cases["plate8x4"] = I.config_plate(8, 4)
    cases["ogrid2x2"] = I.config_ogrid(nt=2, nr=3, r_out=3.0, ratio=1.2)
    base = I.box_mesh((3, 3, 3), (-1, -1, -1), (1, 1, 1), M=(2, 2, 2), wobble=0.12)
    for fam, name in ((I.FAMILY_LG, "curved_lg"), (I.FAMILY_LGL, "curved_lgl")):
        mesh, orders = I.reorient(base, 21, period=(2, 2, 2), orders=I.random_orders(base.K, 1, 7, 22))
        ph = I.Physics(mach=0.3, reynolds=150.0, family=fam, cfl_adv=0.2, cfl_visc=0.2)
        nn = int(I.node_offsets(orders)[-1])
        Q = I.perturbed_freestream(nn, 0.3, 0.02, 23)
        cases[name] = I.Workload(name, mesh, orders, ph, Q)
    return cases
