"""pmg_force_coefficients, a host entry point of the library (CPU; no device is used).

Drag and lift coefficients are the wall force over the dynamic pressure times the reference area (Secs. 4.1 and
4.2).  In the non-dimensional far field rho_inf = |v_inf| = 1 the dynamic pressure is 1/2.  Pinned on the
Couette channel's closed-form force, whose coefficients are known in closed form too, and on a force that
separates the drag (x) and lift (y) directions and the pressure and viscous parts.
"""
import numpy as np
import pytest

from paper_1806_11456_amd import pmg


def test_couette_force_closed_form():
    # u = 2 y over a wall of area A: viscous traction mu du/dy / Re = 2/Re along x, pressure p_inf into the wall
    re, mach, gamma, A = 500.0, 0.2, 1.4, 0.05
    pinf = 1.0 / (gamma * mach ** 2)
    F = np.array([0.0, -pinf * A, 0.0, 2.0 * A / re, 0.0, 0.0])
    cd, cl = pmg.force_coefficients(F, A)
    assert cd == pytest.approx(4.0 / re, rel=1e-15)
    assert cl == pytest.approx(-2.0 * pinf, rel=1e-15)


def test_directions_and_parts():
    F = np.array([3.0, 5.0, 7.0, 11.0, 13.0, 17.0])
    out = np.zeros(4)
    lib = pmg.lib()
    import ctypes as C
    pmg._check(lib.pmg_force_coefficients(F.ctypes.data_as(C.POINTER(C.c_double)), 2.0,
                                          out.ctypes.data_as(C.POINTER(C.c_double))))
    # dynamic pressure x area = 1/2 x 2 = 1: the coefficients are the force components themselves
    assert out.tolist() == [14.0, 18.0, 3.0, 11.0]  # drag = x (pressure + viscous), lift = y; z never enters


def test_rejects_bad_arguments():
    with pytest.raises(pmg.PmgError):
        pmg.force_coefficients(np.zeros(6), 0.0)
    with pytest.raises(pmg.PmgError):
        pmg.force_coefficients(np.zeros(6), -1.0)
