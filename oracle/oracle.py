"""Python face of the plain FP64 CPU oracle (test infrastructure only).

The oracle is the slow, obviously-correct implementation of the DGSEM / FAS p-multigrid hot path that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library; both only read the seeded inputs of
``paper_1806_11456_amd.inputs``.
"""
from __future__ import annotations

import ctypes as C
import glob
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "*.c")))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, fixed summation order."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class Phys(C.Structure):
    _fields_ = [("mach", C.c_double), ("reynolds", C.c_double), ("prandtl", C.c_double), ("gamma", C.c_double),
                ("suth", C.c_double), ("cfl_adv", C.c_double), ("cfl_visc", C.c_double),
                ("family", C.c_int32), ("viscosity", C.c_int32)]


class MGParams(C.Structure):
    _fields_ = [("beta_pre", C.c_int32), ("beta_post", C.c_int32), ("beta_coarse", C.c_int32),
                ("tuning", C.c_int32), ("eta", C.c_double), ("max_repeats", C.c_int32), ("fmg", C.c_int32),
                ("fmg_threshold", C.c_double), ("isolated", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P, D, I32, I64 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.ora_create.restype = P
        L.ora_create.argtypes = [C.c_int64, I32, D, I64, I32, I32, I32, C.POINTER(Phys)]
        L.ora_destroy.argtypes = [P]
        L.ora_basis.argtypes = [C.c_int, C.c_int, D, D, D, D, D]
        L.ora_projection.argtypes = [C.c_int, C.c_int, C.c_int, D]
        L.ora_interp.argtypes = [C.c_int, C.c_int, C.c_int, D]
        L.ora_level_sizes.restype = C.c_int64
        L.ora_level_sizes.argtypes = [P, I32, I64]
        L.ora_geometry.argtypes = [P, I32, D, D, D, D]
        L.ora_operator.argtypes = [P, I32, C.c_int, D, D]
        L.ora_residual.argtypes = [P, I32, C.c_int, D, D, D]
        L.ora_timestep.restype = C.c_double
        L.ora_timestep.argtypes = [P, I32, D]
        L.ora_smooth.argtypes = [P, I32, D, D, C.c_int]
        L.ora_transfer.argtypes = [P, I32, I32, C.c_int, D, D]
        L.ora_roe.argtypes = [C.POINTER(Phys), D, D, D, D]
        L.ora_flux.argtypes = [C.POINTER(Phys), D, D, D, D]
        L.ora_vcycles.restype = C.c_double
        L.ora_vcycles.argtypes = [P, I32, C.c_int, I32, C.c_int, C.POINTER(MGParams), D, D, C.c_int]
        L.ora_tau_3v.argtypes = [P, I32, C.POINTER(MGParams), D, D, D, C.c_int]
        L.ora_tau_nodal.argtypes = [P, I32, C.POINTER(MGParams), D, D, C.c_int, C.c_int, D]
        L.ora_rk3_linear.restype = C.c_double
        L.ora_rk3_linear.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_gradient.argtypes = [P, I32, C.c_int, D, D]
        L.ora_wall_force.argtypes = [P, I32, D, D]
        L.ora_operator_scale.argtypes = [P, I32, C.c_int, D, D, D]
        L.ora_take_eval_count.restype = C.c_int64
        L.ora_take_eval_count.argtypes = []
        L.ora_solve.restype = C.c_int
        L.ora_solve.argtypes = [P, I32, C.c_int, I32, C.POINTER(MGParams), D, D, C.c_double, C.c_int, D, D]
        L.ora_solve_ex.restype = C.c_int
        L.ora_solve_ex.argtypes = [P, I32, C.c_int, I32, C.POINTER(MGParams), D, D, C.c_double, C.c_int, D, D, I32,
                                   I32]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def phys_struct(ph) -> Phys:
    return Phys(ph.mach, ph.reynolds, ph.prandtl, ph.gamma, ph.sutherland, ph.cfl_adv, ph.cfl_visc,
                int(ph.family), int(ph.viscosity))


def mg_params(beta_pre=3, beta_post=3, beta_coarse=3, tuning=0, eta=1.1, max_repeats=10, fmg=0,
              fmg_threshold=0.1, isolated=1) -> MGParams:
    return MGParams(beta_pre, beta_post, beta_coarse, tuning, eta, max_repeats, fmg, fmg_threshold, isolated)


def basis(order: int, family: int):
    n = order + 1
    x, w, lm, lp = (np.zeros(n) for _ in range(4))
    D = np.zeros((n, n))
    lib().ora_basis(order, family, _d(x), _d(w), _d(D), _d(lm), _d(lp))
    return x, w, D, lm, lp


def projection(coarse_order: int, fine_order: int, family: int) -> np.ndarray:
    R = np.zeros((coarse_order + 1, fine_order + 1))
    lib().ora_projection(coarse_order, fine_order, family, _d(R))
    return R


def interpolation(from_order: int, to_order: int, family: int) -> np.ndarray:
    I = np.zeros((to_order + 1, from_order + 1))
    lib().ora_interp(from_order, to_order, family, _d(I))
    return I


def rk3_linear(lam: float, dt: float, q0: float) -> float:
    return float(lib().ora_rk3_linear(lam, dt, q0))


def roe(ph, qL, qR, n) -> np.ndarray:
    F = np.zeros(5)
    p = phys_struct(ph)
    lib().ora_roe(C.byref(p), _d(_f64(qL)), _d(_f64(qR)), _d(_f64(n)), _d(F))
    return F


def fluxes(ph, q, gW):
    Fa = np.zeros((3, 5))
    Fv = np.zeros((3, 5))
    p = phys_struct(ph)
    lib().ora_flux(C.byref(p), _d(_f64(q)), _d(_f64(gW).reshape(-1)), _d(Fa), _d(Fv))
    return Fa, Fv


class Oracle:
    """One mesh + physics; every call takes the order tensor of the level it works on."""

    def __init__(self, mesh, phys):
        self.mesh = mesh
        self.phys = phys
        self._ph = phys_struct(phys)
        self._keep = [np.ascontiguousarray(mesh.gnodes, dtype=np.float64),
                      np.ascontiguousarray(mesh.nbr_elem, dtype=np.int64),
                      np.ascontiguousarray(mesh.nbr_face, dtype=np.int32),
                      np.ascontiguousarray(mesh.orient, dtype=np.int32),
                      np.ascontiguousarray(mesh.bc, dtype=np.int32)]
        M = np.asarray(mesh.M, dtype=np.int32)
        g, nb, nf, o, bc = self._keep
        self.h = lib().ora_create(mesh.K, _i32(M), _d(g), _i64(nb), _i32(nf), _i32(o), _i32(bc), C.byref(self._ph))
        self.K = mesh.K

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ora_destroy(self.h)
            self.h = None

    @staticmethod
    def _ord(orders):
        return np.ascontiguousarray(orders, dtype=np.int32)

    def sizes(self, orders):
        nf = np.zeros(1, dtype=np.int64)
        nn = lib().ora_level_sizes(self.h, _i32(self._ord(orders)), _i64(nf))
        return int(nn), int(nf[0])

    def geometry(self, orders):
        nn, nf = self.sizes(orders)
        X, Ja, J, N = np.zeros((3, nn)), np.zeros((3, 3, nn)), np.zeros(nn), np.zeros((3, nf))
        lib().ora_geometry(self.h, _i32(self._ord(orders)), _d(X), _d(Ja), _d(J), _d(N))
        return X, Ja, J, N

    def gradient(self, orders, Q, isolated=False):
        Q = _f64(Q)
        g = np.zeros((12, Q.shape[1]))
        lib().ora_gradient(self.h, _i32(self._ord(orders)), int(isolated), _d(Q), _d(g))
        return g.reshape(4, 3, -1)

    def wall_force(self, orders, Q):
        """(force on the no-slip walls: pressure part (3), viscous part (3); the round-off scale of each
        component (6): the sum over the wall nodes of the length of the node's vector term)."""
        out = np.zeros(12)
        lib().ora_wall_force(self.h, _i32(self._ord(orders)), _d(_f64(Q)), _d(out))
        return out[:6], out[6:]

    def operator(self, orders, Q, isolated=False):
        Q = _f64(Q)
        A = np.zeros_like(Q)
        lib().ora_operator(self.h, _i32(self._ord(orders)), int(isolated), _d(Q), _d(A))
        return A

    @staticmethod
    def take_eval_count() -> int:
        """Operator evaluations the oracle made since the previous call (all levels)."""
        return int(lib().ora_take_eval_count())

    def operator_scale(self, orders, Q, isolated=False):
        """(A, scale): scale[v, node] = sum of |terms| entering A[v, node] (its round-off scale)."""
        Q = _f64(Q)
        A = np.zeros_like(Q)
        sc = np.zeros_like(Q)
        lib().ora_operator_scale(self.h, _i32(self._ord(orders)), int(isolated), _d(Q), _d(A), _d(sc))
        return A, sc

    def residual(self, orders, Q, S=None, isolated=False):
        Q = _f64(Q)
        R = np.zeros_like(Q)
        Sp = _d(_f64(S)) if S is not None else None
        lib().ora_residual(self.h, _i32(self._ord(orders)), int(isolated), _d(Q), Sp, _d(R))
        return R

    def timestep(self, orders, Q):
        return float(lib().ora_timestep(self.h, _i32(self._ord(orders)), _d(_f64(Q))))

    def smooth(self, orders, Q, S=None, sweeps=1):
        Q = np.array(Q, dtype=np.float64, copy=True)
        Sp = _d(_f64(S)) if S is not None else None
        lib().ora_smooth(self.h, _i32(self._ord(orders)), _d(Q), Sp, int(sweeps))
        return Q

    def transfer(self, ord_from, ord_to, U, prolong: bool):
        U = _f64(U)
        nn, _ = self.sizes(ord_to)
        V = np.zeros((U.shape[0], nn))
        assert U.shape[0] == 5
        lib().ora_transfer(self.h, _i32(self._ord(ord_from)), _i32(self._ord(ord_to)), int(prolong), _d(U), _d(V))
        return V

    def remap(self, ord_from, ord_to, U):
        """State on new orders (after an adaptation): per element and direction, interpolation where the order
        rises, L2 projection where it falls."""
        U = _f64(U)
        nn, _ = self.sizes(ord_to)
        V = np.zeros((U.shape[0], nn))
        assert U.shape[0] == 5
        lib().ora_transfer(self.h, _i32(self._ord(ord_from)), _i32(self._ord(ord_to)), 2, _d(U), _d(V))
        return V

    def vcycles(self, orders, Q, S=None, caps=None, ncycles=1, dir=-1, **prm):
        orders = self._ord(orders)
        if caps is None:
            pmax = int(orders.max())
            caps = list(range(pmax, 0, -1))
        caps = np.asarray(caps, dtype=np.int32)
        Q = np.array(Q, dtype=np.float64, copy=True)
        Sp = _d(_f64(S)) if S is not None else None
        p = mg_params(**prm)
        r = lib().ora_vcycles(self.h, _i32(orders), len(caps), _i32(caps), int(dir), C.byref(p), _d(Q), Sp, ncycles)
        return Q, float(r)

    def tau_3v(self, orders, Q, S=None, **prm):
        orders = self._ord(orders)
        nt = max(int(orders.max()) - 1, 1)
        tau = np.zeros((self.K, 3, nt))
        Q = np.array(Q, dtype=np.float64, copy=True)
        Sp = _d(_f64(S)) if S is not None else None
        p = mg_params(**prm)
        lib().ora_tau_3v(self.h, _i32(orders), C.byref(p), _d(Q), Sp, _d(tau), nt)
        return tau, Q

    def tau_nodal(self, orders, Q, S=None, d=0, cap=1, **prm):
        """One anisotropic V-cycle in direction d; returns (pointwise tau [5][nn] of the level whose order in d
        is capped at 'cap', state after the cycle)."""
        orders = self._ord(orders)
        o = orders.copy()
        o[:, d] = np.minimum(o[:, d], cap)
        nn = int(np.prod(o + 1, axis=1).sum())
        tau = np.full((5, nn), np.nan)
        Q = np.array(Q, dtype=np.float64, copy=True)
        Sp = _d(_f64(S)) if S is not None else None
        p = mg_params(**prm)
        lib().ora_tau_nodal(self.h, _i32(orders), C.byref(p), _d(Q), Sp, int(d), int(cap), _d(tau))
        return tau, Q

    def solve(self, orders, Q, S=None, caps=None, tol=1e-9, max_cycles=100, **prm):
        orders = self._ord(orders)
        if caps is None:
            caps = list(range(int(orders.max()), 0, -1))
        caps = np.asarray(caps, dtype=np.int32)
        Q = np.array(Q, dtype=np.float64, copy=True)
        Sp = _d(_f64(S)) if S is not None else None
        p = mg_params(**prm)
        res = np.zeros(1)
        hist = np.zeros(max_cycles + 1)
        cyc = lib().ora_solve(self.h, _i32(orders), len(caps), _i32(caps), C.byref(p), _d(Q), Sp, float(tol),
                              int(max_cycles), _d(res), _d(hist))
        return Q, int(cyc), float(res[0]), hist[:cyc + 1]

    def solve_record(self, orders, Q, S=None, caps=None, tol=1e-9, max_cycles=100, **prm):
        """solve() that also returns the smoothing blocks of the last visit of each level (reps[l] = (pre, post),
        level 0 the coarsest) and the V-cycles the FMG start ran on each level."""
        orders = self._ord(orders)
        if caps is None:
            caps = list(range(int(orders.max()), 0, -1))
        caps = np.asarray(caps, dtype=np.int32)
        Q = np.array(Q, dtype=np.float64, copy=True)
        Sp = _d(_f64(S)) if S is not None else None
        p = mg_params(**prm)
        res = np.zeros(1)
        hist = np.zeros(max_cycles + 1)
        reps = np.zeros((len(caps), 2), dtype=np.int32)
        fmg = np.zeros(len(caps), dtype=np.int32)
        cyc = lib().ora_solve_ex(self.h, _i32(orders), len(caps), _i32(caps), C.byref(p), _d(Q), Sp, float(tol),
                                 int(max_cycles), _d(res), _d(hist), _i32(reps), _i32(fmg))
        return Q, int(cyc), float(res[0]), reps, fmg
