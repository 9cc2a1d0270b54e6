"""Pins of the oracle's wall force and of the subsonic-outflow boundary condition (CPU), against closed forms
and exact invariants.

* Couette flow u = 2y, p = p_inf, rho = 1 between a no-slip wall (y = 0) and the far field (y = 0.5, where it
  equals the far-field state) on a stretched, quadratically mapped channel, periodic in x and z: every BR1
  interface state equals the trace, so the gradient is exact and the force is the closed form
  F = (2 A / Re, -p_inf A, 0) with A the wall area (mu = 1 at T = 1).  The same on rotated element frames.
* A uniform state on the plate: the pressure part is (0, -p A, 0) whatever the gradient.
* Outflow: the ghost state keeps the interior density and velocity with the far-field pressure, so a uniform
  state with p = p_inf is an exact solution on a box whose faces are all outflow (any density and velocity),
  and a uniform (1, (1, 0, 0), p) state sees the far-field state as its ghost (outflow residual = far-field
  residual); the far-field state is exact on the plate with inflow, free slip and outflow.
"""
import dataclasses

import numpy as np

from oracle import oracle as O
from paper_1806_11456_amd import inputs as I


def channel(nx=4, ny=3):
    return I.box_mesh((nx, ny, 1), (0.0, 0.0, 0.0), (1.0, 0.5, 0.05), M=(2, 2, 2),
                      periodic=(True, False, True), ratio=(1.0, 1.1, 1.0),
                      bc_lo=(I.BC_NONE, I.BC_WALL, I.BC_NONE), bc_hi=(I.BC_NONE, I.BC_FARFIELD, I.BC_NONE))


def mapped_coords(mesh, orders):
    """Solution-node coordinates of the polynomial element mapping (what the discretisation sees): tensor
    Lagrange interpolation of the equispaced mapping nodes at numpy's Gauss-Legendre nodes, node i fastest."""
    out = []
    for e in range(mesh.K):
        g = mesh.gnodes[e]  # (M3+1, M2+1, M1+1, 3)
        L = []
        for d in range(3):
            xe = np.linspace(-1.0, 1.0, mesh.M[d] + 1)
            xs = np.polynomial.legendre.leggauss(int(orders[e, d]) + 1)[0]
            L.append(np.array([[np.prod([(x - xe[m]) / (xe[k] - xe[m]) for m in range(len(xe)) if m != k])
                                for k in range(len(xe))] for x in xs]))
        X = np.einsum("ak,bj,ci,kjid->abcd", L[2], L[1], L[0], g)  # (n3, n2, n1, 3)
        out.append(X.reshape(-1, 3))
    return np.concatenate(out).T


def couette_state(mesh, orders, phys):
    x, y, z = mapped_coords(mesh, orders)
    one = np.ones_like(x)
    pinf = 1.0 / (phys.gamma * phys.mach ** 2)
    return I.conserved(one, 2.0 * y, 0 * one, 0 * one, pinf * one, phys.gamma)


def test_couette_force_closed_form():
    phys = I.Physics(mach=0.2, reynolds=500.0, family=I.FAMILY_LG)
    pinf = 1.0 / (phys.gamma * phys.mach ** 2)
    A = 1.0 * 0.05
    base = channel()
    o0 = I.uniform_orders(base.K, (4, 4, 4))  # N >= 2M: the curl-form metric is exact
    for mesh, orders in ((base, o0), I.reorient(base, 41, period=(1.0, None, 0.05), orders=o0)):
        Q = couette_state(mesh, orders, phys)
        F, sc = O.Oracle(mesh, phys).wall_force(orders, Q)
        want = np.array([0.0, -pinf * A, 0.0, 2.0 * A / phys.reynolds, 0.0, 0.0])
        assert np.all(np.abs(F - want) <= 1e-12 * np.maximum(sc, 1.0)), (F, want)


def test_uniform_state_pressure_force():
    wl = I.config_plate(8, 4, amp=0.0)
    F, sc = O.Oracle(wl.mesh, wl.phys).wall_force(wl.orders, wl.Q)
    pinf = 1.0 / (wl.phys.gamma * wl.phys.mach ** 2)
    assert np.all(np.abs(F[:3] - np.array([0.0, -pinf * 0.05, 0.0])) <= 1e-13 * sc[:3].max())


def test_outflow_keeps_uniform_states_with_far_field_pressure():
    mesh = I.box_mesh((2, 2, 2), (-1, -1, -1), (1, 1, 1), M=(1, 1, 1), periodic=(False, False, False),
                      bc_lo=(I.BC_OUTFLOW,) * 3, bc_hi=(I.BC_OUTFLOW,) * 3)
    phys = I.Physics(mach=0.3, reynolds=100.0, family=I.FAMILY_LG)
    orders = I.uniform_orders(mesh.K, (3, 3, 3))
    nn = int(I.node_offsets(orders)[-1])
    pinf = 1.0 / (phys.gamma * phys.mach ** 2)
    o = O.Oracle(mesh, phys)
    one = np.ones(nn)
    for rho, vel in ((1.3, (0.4, -0.2, 0.1)), (0.7, (-0.5, 0.3, 0.6))):
        Q = I.conserved(rho * one, vel[0] * one, vel[1] * one, vel[2] * one, pinf * one, phys.gamma)
        _, sc = o.operator_scale(orders, Q)
        assert np.abs(o.residual(orders, Q)).max() <= 1e-12 * sc.max()
    # a pressure that differs from the far field's: the boundary now acts
    Q = I.conserved(1.3 * one, 0.4 * one, 0 * one, 0 * one, 1.2 * pinf * one, phys.gamma)
    assert np.abs(o.residual(orders, Q)).max() > 1e-6


def test_outflow_ghost_equals_far_field_for_unit_flow():
    mk = lambda bc: I.box_mesh((2, 2, 1), (-1, -1, -1), (1, 1, 1), M=(1, 1, 1), periodic=(False, False, True),
                               bc_lo=(bc, bc, I.BC_NONE), bc_hi=(bc, bc, I.BC_NONE))
    phys = I.Physics(mach=0.3, reynolds=100.0, family=I.FAMILY_LG)
    orders = I.uniform_orders(4, (3, 3, 2))
    nn = int(I.node_offsets(orders)[-1])
    one = np.ones(nn)
    pinf = 1.0 / (phys.gamma * phys.mach ** 2)
    Q = I.conserved(one, one, 0 * one, 0 * one, 1.1 * pinf * one, phys.gamma)
    Rout = O.Oracle(mk(I.BC_OUTFLOW), phys).residual(orders, Q)
    Rff = O.Oracle(mk(I.BC_FARFIELD), phys).residual(orders, Q)
    assert np.abs(Rff).max() > 1e-6
    assert np.abs(Rout - Rff).max() <= 1e-13 * np.abs(Rff).max()


def test_far_field_state_exact_with_inflow_freeslip_outflow():
    mesh = I.plate_mesh_inflow_outflow(8, 4, x_lead=2.0)  # free slip along all of y = 0, no wall
    assert set(np.unique(mesh.bc[mesh.nbr_elem < 0]).tolist()) == {I.BC_FARFIELD, I.BC_FREESLIP, I.BC_OUTFLOW}
    wl = I.config_plate(8, 4, amp=0.0)
    o = O.Oracle(mesh, wl.phys)
    _, sc = o.operator_scale(wl.orders, wl.Q)
    assert np.abs(o.residual(wl.orders, wl.Q)).max() <= 1e-12 * sc.max()
