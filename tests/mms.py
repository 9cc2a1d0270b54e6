"""Manufactured solutions for the oracle pins: the exact source s = div(F^a - F^v)(q) of a smooth field,
derived symbolically (SymPy) from the non-dimensional Navier-Stokes equations of the paper's Appendix A.

This is an independent, symbolic statement of the PDE used only to pin the oracle; it shares nothing with
the oracle's C code or the HIP library.
"""
from __future__ import annotations

import numpy as np
import sympy as sp


def source_function(rho, u, v, w, p, mach, reynolds, prandtl=0.72, gamma=1.4, suth=110.4 / 288.15,
                    constant_mu=False):
    """rho, u, v, w, p: SymPy expressions in x, y, z.  Returns (q_fn, s_fn) evaluating the conserved state
    and the exact steady source on arrays of coordinates."""
    x, y, z = sp.symbols("x y z")
    X = (x, y, z)
    vel = (u, v, w)
    E = p / (gamma - 1) + sp.Rational(1, 2) * rho * (u ** 2 + v ** 2 + w ** 2)
    q = [rho, rho * u, rho * v, rho * w, E]
    T = gamma * mach ** 2 * p / rho
    mu = sp.Integer(1) if constant_mu else T * sp.sqrt(T) * (1 + suth) / (T + suth)
    div = sum(sp.diff(vel[i], X[i]) for i in range(3))
    tau = [[mu * (sp.diff(vel[i], X[j]) + sp.diff(vel[j], X[i])) - (sp.Rational(2, 3) * mu * div if i == j else 0)
            for j in range(3)] for i in range(3)]
    kap = mu / ((gamma - 1) * prandtl * mach ** 2)
    s = [sp.Integer(0)] * 5
    for c in range(3):
        Fa = [rho * vel[c], rho * u * vel[c], rho * v * vel[c], rho * w * vel[c], vel[c] * (E + p)]
        Fa[1 + c] = Fa[1 + c] + p
        Fv = [0, tau[c][0], tau[c][1], tau[c][2],
              u * tau[c][0] + v * tau[c][1] + w * tau[c][2] + kap * sp.diff(T, X[c])]
        for k in range(5):
            s[k] = s[k] + sp.diff(Fa[k] - Fv[k] / reynolds, X[c])
    qf = sp.lambdify(X, q, "numpy")
    sf = sp.lambdify(X, s, "numpy")

    def ev(f, pts):
        out = f(pts[0], pts[1], pts[2])
        return np.stack([np.broadcast_to(np.asarray(o, dtype=float), pts[0].shape) for o in out])

    return (lambda pts: ev(qf, pts)), (lambda pts: ev(sf, pts))
