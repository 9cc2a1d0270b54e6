"""Thin Python binding of the pmg C-ABI (include/pmg.h): argument marshalling only.

Device arrays are torch tensors on the solver's GPU (float64, contiguous, shape (5, n_nodes) for states);
every call is enqueued on torch's current stream.  All computation happens in the HIP library; if it is
not built this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PMG_LIB names another build of the same library (the host-sanitizer build of the CPU checks); there is no
# fallback when the file is missing
LIB_PATH = os.environ.get("PMG_LIB") or os.path.join(HERE, "libpmg.so")

STATUS = {0: "PMG_OK", 1: "PMG_ERR_INVALID_ARG", 2: "PMG_ERR_OOM", 3: "PMG_ERR_HIP", 4: "PMG_ERR_NONPHYSICAL",
          5: "PMG_ERR_NOT_CONVERGED", 6: "PMG_ERR_BUSY", 7: "PMG_ERR_UNIMPLEMENTED"}

# every entry point the header declares (checked by the CPU test suite)
EXPORTS = ["pmg_last_error", "pmg_ctx_create", "pmg_ctx_destroy", "pmg_mesh_create", "pmg_mesh_destroy",
           "pmg_solver_create", "pmg_solver_destroy", "pmg_state_layout", "pmg_init_freestream", "pmg_residual",
           "pmg_timestep", "pmg_smooth", "pmg_level_info", "pmg_restrict", "pmg_prolong", "pmg_vcycle",
           "pmg_solve", "pmg_tau_estimate", "pmg_profile_enable", "pmg_profile_read", "pmg_profile_stride", "pmg_adapt_orders",
           "pmg_remap_state", "pmg_adapt_multistage", "pmg_wall_force", "pmg_wall_force_noalloc",
           "pmg_force_coefficients", "pmg_batch_create",
           "pmg_batch_layout", "pmg_batch_norms", "pmg_batch_solve", "pmg_set_graph", "pmg_autotune",
           "pmg_level_tiles", "pmg_set_tiles", "pmg_solve_stats", "pmg_guard_stats", "pmg_footprint", "pmg_device_bytes", "pmg_server_create",
           "pmg_server_submit", "pmg_server_poll", "pmg_server_stats", "pmg_server_destroy", "pmg_tau_nodal",
           "pmg_solve_history", "pmg_cycle_count", "pmg_checkpoint", "pmg_restore"]

# kernel kinds of pmg_profile_enable / pmg_profile_read
KINDS = {"trace": 0, "face1": 1, "grad": 2, "face2": 3, "div": 4, "dt": 5, "transfer": 6}


class PmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Physics(C.Structure):
    _fields_ = [("mach", C.c_double), ("reynolds", C.c_double), ("prandtl", C.c_double), ("gamma", C.c_double),
                ("sutherland", C.c_double), ("cfl_adv", C.c_double), ("cfl_visc", C.c_double),
                ("node_family", C.c_int32), ("viscosity_model", C.c_int32)]


class MGParams(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level_caps", C.POINTER(C.c_int32)), ("beta_pre", C.c_int32),
                ("beta_post", C.c_int32), ("beta_coarse", C.c_int32), ("tuning", C.c_int32), ("eta", C.c_double),
                ("max_repeats", C.c_int32), ("fmg", C.c_int32), ("fmg_threshold", C.c_double),
                ("precision", C.c_int32), ("mixed_patience", C.c_int32), ("guard", C.c_int32)]


@dataclasses.dataclass
class MG:
    level_caps: Optional[Sequence[int]] = None
    beta_pre: int = 3
    beta_post: int = 3
    beta_coarse: int = 3
    tuning: int = 0
    eta: float = 1.1
    max_repeats: int = 10
    fmg: int = 0
    fmg_threshold: float = 0.1
    precision: int = 0  # 0 all FP64; 1 mixed (FP32 coarse-level smoothing, FP64 finest level)
    mixed_patience: int = 0  # mixed: cycles without a new residual minimum before FP64 coarse levels (0 = 4)
    guard: int = 0  # divergence guard of the solve drivers: at most this many halvings of the step constants


_lib = None


def lib():
    """Load libpmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1806_11456_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    # torch first: the library's HIP runtime dependency then resolves to the runtime torch already holds,
    # so the process has one HIP runtime whichever call (host-only or device) loads the library first
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, D, I32, I64, V = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_void_p
    pp = C.POINTER(C.c_void_p)
    L.pmg_last_error.restype = C.c_char_p
    L.pmg_ctx_create.argtypes = [C.c_int, pp]
    L.pmg_ctx_destroy.argtypes = [P]
    L.pmg_mesh_create.argtypes = [P, C.c_int64, I32, D, I64, I32, I32, I32, pp]
    L.pmg_mesh_destroy.argtypes = [P]
    L.pmg_solver_create.argtypes = [P, P, I32, C.POINTER(Physics), C.POINTER(MGParams), pp]
    L.pmg_solver_destroy.argtypes = [P]
    L.pmg_state_layout.argtypes = [P, I64, I64]
    L.pmg_init_freestream.argtypes = [P, V, V]
    L.pmg_residual.argtypes = [P, C.c_int, V, V, V, D, V]
    L.pmg_timestep.argtypes = [P, V, D, V]
    L.pmg_smooth.argtypes = [P, V, V, C.c_int, V]
    L.pmg_level_info.argtypes = [P, C.c_int, C.c_int, I32, I64, I32]
    L.pmg_restrict.argtypes = [P, C.c_int, C.c_int, V, V, V]
    L.pmg_prolong.argtypes = [P, C.c_int, C.c_int, V, V, V]
    L.pmg_vcycle.argtypes = [P, V, V, C.c_int, D, V]
    L.pmg_solve.argtypes = [P, V, V, C.c_double, C.c_int, I32, D, V]
    L.pmg_tau_estimate.argtypes = [P, V, V, C.c_int, V, V]
    L.pmg_tau_nodal.argtypes = [P, C.c_int, C.c_int, V, V, C.c_int, V, V]
    L.pmg_solve_history.argtypes = [P, D, C.c_int32, I32]
    L.pmg_cycle_count.argtypes = [P, I64]
    L.pmg_checkpoint.argtypes = [P, C.c_char_p, V, V]
    L.pmg_restore.argtypes = [P, C.c_char_p, V, V]
    L.pmg_profile_enable.argtypes = [P, C.c_uint32]
    L.pmg_profile_read.argtypes = [P, C.c_int, D, I64, D]
    L.pmg_profile_stride.argtypes = [P, C.c_int32]
    L.pmg_adapt_orders.argtypes = [C.c_int64, I64, I32, I32, I32, I32, D, C.c_int32, C.POINTER(AdaptParams), I32,
                                   I32]
    L.pmg_remap_state.argtypes = [P, V, P, V, V]
    L.pmg_wall_force.argtypes = [P, V, D, V]
    L.pmg_wall_force_noalloc.argtypes = [P, V, D, V]
    L.pmg_force_coefficients.argtypes = [D, C.c_double, D]
    L.pmg_adapt_multistage.argtypes = [P, P, I32, C.POINTER(Physics), C.POINTER(MGParams),
                                       C.POINTER(MultistageParams), V, C.c_int64, I32, I64,
                                       C.POINTER(StageReport), I32, I32, D, V]
    L.pmg_batch_create.argtypes = [P, C.c_int, C.POINTER(C.c_void_p), C.POINTER(I32), C.POINTER(Physics),
                                   C.POINTER(MGParams), pp]
    L.pmg_batch_layout.argtypes = [P, I32, I64]
    L.pmg_batch_norms.argtypes = [P, V, V, D, V]
    L.pmg_batch_solve.argtypes = [P, V, V, C.c_double, C.c_int, I32, D, V]
    L.pmg_set_graph.argtypes = [P, C.c_int]
    L.pmg_autotune.argtypes = [P, V]
    L.pmg_level_tiles.argtypes = [P, C.c_int, C.c_int, I32, I32]
    L.pmg_set_tiles.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int]
    L.pmg_solve_stats.argtypes = [P, I32]
    L.pmg_guard_stats.argtypes = [P, I32, D]
    L.pmg_footprint.argtypes = [P, I32, C.POINTER(MGParams), I64, I64, I64]
    L.pmg_device_bytes.argtypes = [I64]
    L.pmg_server_create.argtypes = [P, C.c_int64, C.c_int, C.c_int, C.c_int, pp]
    L.pmg_server_submit.argtypes = [P, P, I32, C.POINTER(Physics), C.POINTER(MGParams), V, C.c_double, C.c_int,
                                    C.POINTER(C.c_uint64)]
    L.pmg_server_poll.argtypes = [P, C.c_uint64, I32, I32, I32, I32, D, D, D]
    L.pmg_server_stats.argtypes = [P, I32, I32, I64, I64, I64, I64, I32]
    L.pmg_server_destroy.argtypes = [P]
    L.pmg_server_destroy.restype = None
    for name in EXPORTS:
        if name not in ("pmg_last_error", "pmg_ctx_destroy", "pmg_mesh_destroy", "pmg_solver_destroy",
                        "pmg_server_destroy"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise PmgError(rc, lib().pmg_last_error().decode())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous(), "expected a contiguous CUDA tensor"
    return C.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(lib().pmg_ctx_create(device, C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pmg_ctx_destroy(self.h)
            self.h = None


class Mesh:
    def __init__(self, ctx: Context, mesh):
        self.ctx = ctx
        self.K = int(mesh.K)
        M = np.asarray(mesh.M, dtype=np.int32)
        self._arrs = [np.ascontiguousarray(mesh.gnodes, dtype=np.float64), np.ascontiguousarray(mesh.nbr_elem, dtype=np.int64),
                      np.ascontiguousarray(mesh.nbr_face, dtype=np.int32), np.ascontiguousarray(mesh.orient, dtype=np.int32),
                      np.ascontiguousarray(mesh.bc, dtype=np.int32)]
        g, nb, nf, o, bc = self._arrs
        h = C.c_void_p()
        _check(lib().pmg_mesh_create(ctx.h, self.K, M.ctypes.data_as(C.POINTER(C.c_int32)),
                                     g.ctypes.data_as(C.POINTER(C.c_double)), nb.ctypes.data_as(C.POINTER(C.c_int64)),
                                     nf.ctypes.data_as(C.POINTER(C.c_int32)), o.ctypes.data_as(C.POINTER(C.c_int32)),
                                     bc.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h)))
        self.h = h
        self._arrs = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pmg_mesh_destroy(self.h)
            self.h = None


def mg_struct(mg):
    """(pmg_mg_params, level-caps array that must outlive the call)."""
    caps = None if mg.level_caps is None else np.asarray(mg.level_caps, dtype=np.int32)
    p = MGParams(0 if caps is None else len(caps),
                 None if caps is None else caps.ctypes.data_as(C.POINTER(C.c_int32)),
                 mg.beta_pre, mg.beta_post, mg.beta_coarse, mg.tuning, mg.eta, mg.max_repeats, mg.fmg,
                 mg.fmg_threshold, mg.precision, mg.mixed_patience, mg.guard)
    return p, caps


def footprint(mesh: "Mesh", orders, mg: "MG" = None):
    """(device bytes as built, construction transient, precision-switch hierarchy) of a single-problem
    solver (pmg_footprint)."""
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    p, caps = mg_struct(mg or MG())
    b, t, sw = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().pmg_footprint(mesh.h, orders.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(p), C.byref(b),
                               C.byref(t), C.byref(sw)))
    return int(b.value), int(t.value), int(sw.value)


class AdaptParams(C.Structure):
    _fields_ = [("tau_max", C.c_double), ("n_max", C.c_int32 * 3), ("n_min", C.c_int32), ("jump_rule", C.c_int32),
                ("wall_conforming", C.c_int32), ("n_cap", C.c_int32)]


class MultistageParams(C.Structure):
    _fields_ = [("stages", C.POINTER(C.c_int32)), ("n_stages", C.c_int32), ("adapt", AdaptParams),
                ("conv", C.c_double), ("final_tol", C.c_double), ("max_cycles", C.c_int32),
                ("n_coarse", C.c_int32)]


class StageReport(C.Structure):
    _fields_ = [("stage_order", C.c_int32), ("cycles", C.c_int32), ("res_inf", C.c_double),
                ("converged", C.c_int32), ("max_required", C.c_int32), ("last", C.c_int32), ("pad", C.c_int32),
                ("nodes_before", C.c_int64), ("nodes_after", C.c_int64)]


def adapt_orders(mesh, orders, tau_map, tau_max: float, n_max=(7, 7, 7), n_min: int = 1, jump_rule: int = 1,
                 wall_conforming: bool = False, n_cap: int = 0, with_required: bool = False):
    """New element orders (K, 3) from the reference orders and the directional truncation-error map
    [K][3][nt] (pmg_adapt_orders: a host function; ``mesh`` is the host-side mesh description of
    paper_1806_11456_amd.inputs); with ``with_required`` also the largest order selected before the cap."""
    K = int(mesh.K)
    tau = np.ascontiguousarray(tau_map, dtype=np.float64)
    assert tau.ndim == 3 and tau.shape[0] == K and tau.shape[1] == 3
    nbr = np.ascontiguousarray(mesh.nbr_elem, dtype=np.int64)
    nbf = np.ascontiguousarray(mesh.nbr_face, dtype=np.int32)
    ori = np.ascontiguousarray(mesh.orient, dtype=np.int32)
    bc = np.ascontiguousarray(mesh.bc, dtype=np.int32)
    P = np.ascontiguousarray(orders, dtype=np.int32)
    out = np.zeros((K, 3), dtype=np.int32)
    prm = adapt_params(tau_max, n_max, n_min, jump_rule, wall_conforming, n_cap)
    i32, i64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    req = C.c_int32()
    _check(lib().pmg_adapt_orders(K, nbr.ctypes.data_as(i64), nbf.ctypes.data_as(i32), ori.ctypes.data_as(i32),
                                  bc.ctypes.data_as(i32), P.ctypes.data_as(i32),
                                  tau.ctypes.data_as(C.POINTER(C.c_double)), int(tau.shape[2]), C.byref(prm),
                                  out.ctypes.data_as(i32), C.byref(req)))
    return (out, int(req.value)) if with_required else out


def adapt_params(tau_max, n_max=(7, 7, 7), n_min=1, jump_rule=1, wall_conforming=False, n_cap=0) -> AdaptParams:
    return AdaptParams(float(tau_max), (C.c_int32 * 3)(*[int(v) for v in n_max]), int(n_min), int(jump_rule),
                       int(bool(wall_conforming)), int(n_cap))


def force_coefficients(F, area: float):
    """(drag, lift) coefficients of a wall force F (the 6 values of Solver.wall_force), pmg_force_coefficients."""
    f = np.ascontiguousarray(F, dtype=np.float64)
    assert f.shape == (6,)
    c = np.zeros(4)
    _check(lib().pmg_force_coefficients(f.ctypes.data_as(C.POINTER(C.c_double)), float(area),
                                        c.ctypes.data_as(C.POINTER(C.c_double))))
    return float(c[0]), float(c[1])


def remap_state(src: "Solver", Q_src, dst: "Solver", Q_dst=None):
    """The state of ``src`` carried over to the orders of ``dst`` (pmg_remap_state); returns Q_dst."""
    Q_dst = dst.empty() if Q_dst is None else Q_dst
    _check(lib().pmg_remap_state(src.h, _ptr(Q_src), dst.h, _ptr(Q_dst), _stream()))
    return Q_dst


def adapt_multistage(ctx: "Context", mesh: "Mesh", orders, phys, mg: "MG", stages, tau_max: float,
                     n_max=(7, 7, 7), n_min: int = 1, jump_rule: int = 1, wall_conforming: bool = False,
                     conv: float = 0.1, final_tol: float = 1e-8, max_cycles: int = 100,
                     raise_not_converged: bool = True, n_coarse: int = 1):
    """Multi-stage adaptation from free stream on the first stage's ``orders`` (pmg_adapt_multistage).
    Returns (orders (K, 3), state [5][nn] as a torch tensor, per-stage reports, final cycles, final residual)."""
    import torch
    K = int(mesh.K)
    orders = np.ascontiguousarray(orders, dtype=np.int32)
    st = np.ascontiguousarray(stages, dtype=np.int32)
    top = [max(int(n_max[d]), int(orders[:, d].max())) + 1 for d in range(3)]
    cap = K * top[0] * top[1] * top[2]
    Q = torch.empty(5 * cap, dtype=torch.float64, device=torch.device("cuda", ctx.device))
    p, caps_keep = mg_struct(mg)
    ph = physics_struct(phys)
    prm = MultistageParams(st.ctypes.data_as(C.POINTER(C.c_int32)), len(st),
                           adapt_params(tau_max, n_max, n_min, jump_rule, wall_conforming, 0), float(conv),
                           float(final_tol), int(max_cycles), int(n_coarse))
    out = np.zeros((K, 3), dtype=np.int32)
    nn = C.c_int64()
    reps = (StageReport * len(st))()
    nrep, cyc, res = C.c_int32(), C.c_int32(), C.c_double()
    i32 = C.POINTER(C.c_int32)
    rc = lib().pmg_adapt_multistage(ctx.h, mesh.h, orders.ctypes.data_as(i32), C.byref(ph), C.byref(p),
                                    C.byref(prm), _ptr(Q), cap, out.ctypes.data_as(i32), C.byref(nn), reps,
                                    C.byref(nrep), C.byref(cyc), C.byref(res), _stream())
    if rc != 0 and not (rc == 5 and not raise_not_converged):
        _check(rc)
    n = int(nn.value)
    reports = [{f: getattr(reps[i], f) for f, _ in StageReport._fields_ if f != "pad"} for i in range(nrep.value)]
    return out, Q[:5 * n].view(5, n), reports, int(cyc.value), float(res.value)


def device_bytes() -> int:
    """Device bytes currently allocated by the library."""
    b = C.c_int64()
    _check(lib().pmg_device_bytes(C.byref(b)))
    return int(b.value)


def physics_struct(ph) -> Physics:
    return Physics(ph.mach, ph.reynolds, ph.prandtl, ph.gamma, ph.sutherland, ph.cfl_adv, ph.cfl_visc,
                   int(ph.family), int(ph.viscosity))


class Solver:
    """mesh + orders + physics + multigrid hierarchy on one GPU."""

    def __init__(self, ctx: Context, mesh: Mesh, orders, phys, mg: MG = MG()):
        orders = np.ascontiguousarray(orders, dtype=np.int32)
        p = self._params(mg)
        ph = physics_struct(phys)
        h = C.c_void_p()
        _check(lib().pmg_solver_create(ctx.h, mesh.h, orders.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(ph),
                                       C.byref(p), C.byref(h)))
        self._setup(ctx, h, mesh.K, orders, mg)
        self.mesh, self.phys = mesh, phys

    def _params(self, mg):
        p, self._caps = mg_struct(mg)
        return p

    def _setup(self, ctx, h, K, orders, mg):
        import torch
        self.ctx, self.mg, self.h, self.K = ctx, mg, h, K
        self.torch = torch
        self.device = torch.device("cuda", ctx.device)
        self.orders = orders
        nn = C.c_int64()
        off = np.zeros(K + 1, dtype=np.int64)
        _check(lib().pmg_state_layout(h, C.byref(nn), off.ctypes.data_as(C.POINTER(C.c_int64))))
        self.n_nodes = int(nn.value)
        self.offsets = off
        self.nmax = int(orders.max())

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pmg_solver_destroy(self.h)
            self.h = None

    # -- helpers --------------------------------------------------------------------------------------
    def empty(self, n: Optional[int] = None):
        return self.torch.empty((5, self.n_nodes if n is None else n), dtype=self.torch.float64, device=self.device)

    def tensor(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)

    # -- entry points -----------------------------------------------------------------------------------
    def freestream(self):
        Q = self.empty()
        _check(lib().pmg_init_freestream(self.h, _ptr(Q), _stream()))
        return Q

    def residual(self, Q, S=None, isolated=False, out=None, norm=False):
        out = self.empty() if out is None else out
        r = C.c_double()
        _check(lib().pmg_residual(self.h, int(bool(isolated)), _ptr(Q), _ptr(S), _ptr(out),
                                  C.byref(r) if norm else None, _stream()))
        return (out, r.value) if norm else out

    def wall_force(self, Q) -> np.ndarray:
        """Force on the no-slip walls (pmg_wall_force): pressure part x, y, z, then viscous part x, y, z."""
        F = np.zeros(6)
        _check(lib().pmg_wall_force(self.h, _ptr(Q), F.ctypes.data_as(C.POINTER(C.c_double)), _stream()))
        return F

    def wall_force_noalloc(self, Q) -> np.ndarray:
        """The same force without device allocation (pmg_wall_force_noalloc): partials in the library's static
        per-GPU scratch; calls that overlap on one GPU race."""
        F = np.zeros(6)
        _check(lib().pmg_wall_force_noalloc(self.h, _ptr(Q), F.ctypes.data_as(C.POINTER(C.c_double)), _stream()))
        return F

    def timestep(self, Q) -> float:
        dt = C.c_double()
        _check(lib().pmg_timestep(self.h, _ptr(Q), C.byref(dt), _stream()))
        return dt.value

    def smooth(self, Q, S=None, sweeps=1):
        _check(lib().pmg_smooth(self.h, _ptr(Q), _ptr(S), int(sweeps), _stream()))
        return Q

    def level_info(self, hierarchy: int, level: int = -1):
        nl = C.c_int32()
        nn = C.c_int64()
        if level < 0:
            _check(lib().pmg_level_info(self.h, hierarchy, -1, C.byref(nl), None, None))
            return int(nl.value)
        orders = np.zeros((self.K, 3), dtype=np.int32)
        _check(lib().pmg_level_info(self.h, hierarchy, level, C.byref(nl), C.byref(nn),
                                    orders.ctypes.data_as(C.POINTER(C.c_int32))))
        return int(nn.value), orders

    def restrict(self, hierarchy: int, level: int, U):
        nn, _ = self.level_info(hierarchy, level - 1)
        out = self.empty(nn)
        _check(lib().pmg_restrict(self.h, hierarchy, level, _ptr(U), _ptr(out), _stream()))
        return out

    def prolong(self, hierarchy: int, level: int, U):
        nn, _ = self.level_info(hierarchy, level + 1)
        out = self.empty(nn)
        _check(lib().pmg_prolong(self.h, hierarchy, level, _ptr(U), _ptr(out), _stream()))
        return out

    def vcycle(self, Q, S=None, n_cycles=1, norm=False):
        r = C.c_double()
        _check(lib().pmg_vcycle(self.h, _ptr(Q), _ptr(S), int(n_cycles), C.byref(r) if norm else None, _stream()))
        return r.value if norm else None

    def solve(self, Q, S=None, tol=1e-9, max_cycles=100, raise_not_converged=True):
        cyc = C.c_int32()
        r = C.c_double()
        rc = lib().pmg_solve(self.h, _ptr(Q), _ptr(S), float(tol), int(max_cycles), C.byref(cyc), C.byref(r), _stream())
        if rc != 0 and (rc != 5 or raise_not_converged):
            _check(rc)
        return int(cyc.value), float(r.value)

    def fp32_cycles(self):
        """Per problem: cycles of the last solve that ran with FP32 coarse levels (mixed precision)."""
        n = getattr(self, "n", 1)
        out = np.zeros(n, dtype=np.int32)
        _check(lib().pmg_solve_stats(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def guard_stats(self):
        """Per problem: (step-constant halvings of the divergence guard, current (C^a, C^nu))."""
        n = getattr(self, "n", 1)
        h = np.zeros(n, dtype=np.int32)
        c = np.zeros((n, 2))
        _check(lib().pmg_guard_stats(self.h, h.ctypes.data_as(C.POINTER(C.c_int32)),
                                     c.ctypes.data_as(C.POINTER(C.c_double))))
        return h, c

    def profile(self, kinds, stride: int = 1):
        """Bracket every stride-th launch of the given kernel kinds with HIP events (empty = off)."""
        mask = 0
        for k in kinds:
            mask |= 1 << KINDS[k]
        _check(lib().pmg_profile_stride(self.h, int(stride)))
        _check(lib().pmg_profile_enable(self.h, mask))

    def profile_read(self, kind: str):
        """(summed milliseconds, launches, summed compulsory bytes) of one kind since its last read."""
        ms = C.c_double()
        n = C.c_int64()
        b = C.c_double()
        _check(lib().pmg_profile_read(self.h, KINDS[kind], C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, int(n.value), b.value

    def tau_estimate(self, Q, S=None, isolated=True, out=None):
        nt = max(self.nmax - 1, 1)
        tau = self.torch.empty((self.K, 3, nt), dtype=self.torch.float64, device=self.device) if out is None else out
        _check(lib().pmg_tau_estimate(self.h, _ptr(Q), _ptr(S), int(bool(isolated)), _ptr(tau), _stream()))
        return tau

    def history(self):
        """||r||_inf at every check of the last solve()."""
        n = C.c_int32()
        _check(lib().pmg_solve_history(self.h, None, 0, C.byref(n)))
        out = np.zeros(n.value)
        _check(lib().pmg_solve_history(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n.value, C.byref(n)))
        return out

    def cycle_count(self) -> int:
        c = C.c_int64()
        _check(lib().pmg_cycle_count(self.h, C.byref(c)))
        return int(c.value)

    def checkpoint(self, path: str, Q):
        _check(lib().pmg_checkpoint(self.h, str(path).encode(), _ptr(Q), _stream()))

    def restore(self, path: str, Q):
        _check(lib().pmg_restore(self.h, str(path).encode(), _ptr(Q), _stream()))

    def tau_nodal(self, Q, S=None, d=0, order=1, isolated=True):
        """Pointwise tau [5][nn] of the level of hierarchy d capped at 'order' (one anisotropic cycle on Q)."""
        import torch
        nl = self.level_info(d)
        lev = [l for l in range(nl - 1) if int(self.level_info(d, l)[1][:, d].max()) == order]
        assert lev, "no such level"
        nn = self.level_info(d, lev[0])[0]
        out = torch.empty((5, nn), dtype=torch.float64, device=self.device)
        _check(lib().pmg_tau_nodal(self.h, int(d), int(order), _ptr(Q), _ptr(S), int(bool(isolated)), _ptr(out),
                                   _stream()))
        return out

    def set_graph(self, enable: bool):
        _check(lib().pmg_set_graph(self.h, int(bool(enable))))

    def autotune(self):
        _check(lib().pmg_autotune(self.h, _stream()))

    def level_tiles(self, hierarchy: int, level: int) -> int:
        """The level's element-tile node target (32, 64, 128, 256 or 512)."""
        return self.level_tile_choice(hierarchy, level)[0]

    def set_tiles(self, hierarchy: int, level: int, target: int, split: int = 0):
        """Rebuild one level's element tiles for a node target and launch split bits (bit 0 the gradient,
        bit 1 the divergence launched per tile-size class; pmg_set_tiles)."""
        _check(lib().pmg_set_tiles(self.h, hierarchy, level, int(target), int(split)))

    def level_tile_choice(self, hierarchy: int, level: int):
        """(node target, split bits): bit 0 / bit 1 set when the gradient / divergence launches per size class."""
        t, sp = C.c_int32(), C.c_int32()
        _check(lib().pmg_level_tiles(self.h, hierarchy, level, C.byref(t), C.byref(sp)))
        return int(t.value), int(sp.value)


class Batch(Solver):
    """n independent problems advanced together (one union solver; per-problem step, norms, freezing)."""

    def __init__(self, ctx: Context, meshes, orders_list, phys_list, mg: MG = MG()):
        n = len(meshes)
        ords = [np.ascontiguousarray(o, dtype=np.int32) for o in orders_list]
        self._ords = ords
        mesh_arr = (C.c_void_p * n)(*[m.h.value for m in meshes])
        ord_arr = (C.POINTER(C.c_int32) * n)(*[o.ctypes.data_as(C.POINTER(C.c_int32)) for o in ords])
        ph_arr = (Physics * n)(*[physics_struct(p) for p in phys_list])
        p = self._params(mg)
        h = C.c_void_p()
        _check(lib().pmg_batch_create(ctx.h, n, mesh_arr, ord_arr, ph_arr, C.byref(p), C.byref(h)))
        K = sum(m.K for m in meshes)
        self._setup(ctx, h, K, np.concatenate(ords), mg)
        self.meshes, self.phys_list, self.n = meshes, phys_list, n
        npb = C.c_int32()
        off = np.zeros(n + 1, dtype=np.int64)
        _check(lib().pmg_batch_layout(h, C.byref(npb), off.ctypes.data_as(C.POINTER(C.c_int64))))
        self.problem_offsets = off

    def norms(self, Q, S=None):
        r = np.zeros(self.n)
        _check(lib().pmg_batch_norms(self.h, _ptr(Q), _ptr(S), r.ctypes.data_as(C.POINTER(C.c_double)), _stream()))
        return r

    def solve_all(self, Q, S=None, tol=1e-9, max_cycles=100, raise_not_converged=True, raise_failed=True):
        """Batched solve (pmg_batch_solve): per-problem cycles and residuals.  raise_failed=False returns the
        outputs also when the divergence guard gave up on some problems (their residual NaN)."""
        cyc = np.zeros(self.n, dtype=np.int32)
        r = np.zeros(self.n)
        rc = lib().pmg_batch_solve(self.h, _ptr(Q), _ptr(S), float(tol), int(max_cycles),
                                   cyc.ctypes.data_as(C.POINTER(C.c_int32)), r.ctypes.data_as(C.POINTER(C.c_double)),
                                   _stream())
        if rc != 0 and not (rc == 5 and not raise_not_converged) and not (rc == 4 and not raise_failed
                                                                        and self.mg.guard > 0):
            _check(rc)
        return cyc, r

    def part(self, U, p: int):
        """View of problem p's nodes in a batch array [5][n_nodes]."""
        return U[:, int(self.problem_offsets[p]):int(self.problem_offsets[p + 1])]


class Server:
    """Continuous-batching steady-solve server on one GPU (pmg_server_* in include/pmg.h).

    submit() hands over a problem and a CUDA state tensor solved in place; poll() returns None while the
    request is queued or resident, then a dict with status, cycles, fp32_cycles, residual, latency_s and
    queue_s (seconds from submission to admission)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, n_streams: int = 4, use_graph: bool = True,
                 batched: bool = False):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().pmg_server_create(ctx.h, int(hbm_budget_bytes), int(n_streams), int(bool(use_graph)),
                                       int(bool(batched)), C.byref(h)))
        self.h = h
        self._alive = {}  # ticket -> (mesh, state): kept alive until the request is done

    def submit(self, mesh: Mesh, orders, phys, mg: MG, Q, tol: float, max_cycles: int) -> int:
        import torch
        orders = np.ascontiguousarray(orders, dtype=np.int32)
        p, caps = mg_struct(mg)
        ph = physics_struct(phys)
        torch.cuda.current_stream().synchronize()  # the initial state is complete before the server reads it
        t = C.c_uint64()
        _check(lib().pmg_server_submit(self.h, mesh.h, orders.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(ph),
                                       C.byref(p), _ptr(Q), float(tol), int(max_cycles), C.byref(t)))
        self._alive[t.value] = (mesh, Q)
        return int(t.value)

    def poll(self, ticket: int):
        done, st, cyc, f32 = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        r, lat, qs = C.c_double(), C.c_double(), C.c_double()
        _check(lib().pmg_server_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(st), C.byref(cyc),
                                     C.byref(f32), C.byref(r), C.byref(lat), C.byref(qs)))
        if not done.value:
            return None
        self._alive.pop(ticket, None)
        return {"status": int(st.value), "cycles": int(cyc.value), "fp32_cycles": int(f32.value),
                "residual": float(r.value), "latency_s": float(lat.value), "queue_s": float(qs.value)}

    def stats(self):
        res, q, mres = C.c_int32(), C.c_int32(), C.c_int32()
        comp, it, used, peak = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().pmg_server_stats(self.h, C.byref(res), C.byref(q), C.byref(comp), C.byref(it), C.byref(used),
                                      C.byref(peak), C.byref(mres)))
        return {"resident": res.value, "queued": q.value, "completed": comp.value, "iterations": it.value,
                "bytes_in_use": used.value, "peak_bytes": peak.value, "max_resident": mres.value}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pmg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
