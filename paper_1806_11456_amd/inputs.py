"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module only *describes problems*: it places the geometry nodes of each hexahedron, links the faces
(neighbour, neighbour face, orientation code, boundary tag), draws order tensors and samples initial or
perturbed states at the solution nodes.  It computes nothing the method computes (no metrics, fluxes,
operators or transfers), so both implementations can consume it without sharing any of the method.

Conventions (they are the ones the C-ABI documents in include/pmg.h):

* Element e has reference coordinates (xi, eta, zeta) in [-1, 1]^3 and orders (N1, N2, N3).  Its nodes are
  the tensor product of the 1-D node sets, node index i + n1*(j + n2*k) with n_d = N_d + 1 (xi fastest).
* A state is stored variable-major, ``Q[v, node]`` with v in (rho, rho u, rho v, rho w, rho e), the nodes of
  element 0 first, then element 1, and so on.
* Faces are numbered 0..5 = xi-, xi+, eta-, eta+, zeta-, zeta+.  The two face-local coordinates (s, t) are the
  two tangential reference coordinates in increasing axis order.
* Orientation code o (0..7) of face f of element e towards its neighbour face f' maps a point with local
  coordinates (s, t) on e's face to (s', t') on the neighbour's face: (u, v) = (t, s) if o & 4 else (s, t);
  s' = -u if o & 1 else u; t' = -v if o & 2 else v.
* Geometry of element e is a tensor-product Lagrange mapping of degree (M1, M2, M3) given by its values at
  equispaced reference nodes, array shape (K, M3+1, M2+1, M1+1, 3).
* Boundary tags: 0 = interior or periodic (has a neighbour), 1 = no-slip adiabatic wall, 2 = far field,
  3 = free-slip wall.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np

BC_NONE, BC_WALL, BC_FARFIELD, BC_FREESLIP, BC_OUTFLOW = 0, 1, 2, 3, 4
FAMILY_LG, FAMILY_LGL = 0, 1

# face f -> (normal axis, side) with side 0 at -1 and 1 at +1
FACE_AXIS = (0, 0, 1, 1, 2, 2)
FACE_SIDE = (0, 1, 0, 1, 0, 1)
TANGENTIAL = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


def orient_map(o: int, s, t):
    """Apply orientation code o to face-local coordinates (s, t) (see module docstring)."""
    u, v = (t, s) if (o & 4) else (s, t)
    return (-u if (o & 1) else u), (-v if (o & 2) else v)


@dataclasses.dataclass
class Mesh:
    """Hexahedral mesh: mapping nodes + face connectivity.  ``cmap(e, ref)`` is the continuous map the
    mapping nodes were sampled from (used only to sample input fields)."""

    K: int
    M: tuple
    gnodes: np.ndarray          # (K, M3+1, M2+1, M1+1, 3) float64
    nbr_elem: np.ndarray        # (K, 6) int64, -1 on boundary faces
    nbr_face: np.ndarray        # (K, 6) int8
    orient: np.ndarray          # (K, 6) int8
    bc: np.ndarray              # (K, 6) int32
    cmap: Optional[Callable] = None
    name: str = "mesh"

    def validate(self) -> None:
        K = self.K
        assert self.gnodes.shape == (K, self.M[2] + 1, self.M[1] + 1, self.M[0] + 1, 3)
        for e in range(K):
            for f in range(6):
                n = int(self.nbr_elem[e, f])
                if n < 0:
                    assert self.bc[e, f] != BC_NONE, (e, f)
                    continue
                g = int(self.nbr_face[e, f])
                assert int(self.nbr_elem[n, g]) == e and int(self.nbr_face[n, g]) == f, (e, f, n, g)
                o, ob = int(self.orient[e, f]), int(self.orient[n, g])
                for s, t in ((-1.0, -1.0), (1.0, -1.0), (-1.0, 1.0), (1.0, 1.0), (0.3, -0.7)):
                    s2, t2 = orient_map(o, s, t)
                    s3, t3 = orient_map(ob, s2, t2)
                    assert abs(s3 - s) < 1e-14 and abs(t3 - t) < 1e-14, (e, f, o, ob)


# --------------------------------------------------------------------------------------------------
# 1-D node sets used only to *sample* input fields at the solution nodes (library routines).
# --------------------------------------------------------------------------------------------------
def sample_nodes(order: int, family: int) -> np.ndarray:
    if family == FAMILY_LG:
        return np.polynomial.legendre.leggauss(order + 1)[0]
    if order == 0:
        raise ValueError("LGL needs order >= 1")
    inner = np.polynomial.legendre.Legendre.basis(order).deriv().roots() if order > 1 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def node_offsets(orders: np.ndarray) -> np.ndarray:
    npe = np.prod(np.asarray(orders, dtype=np.int64) + 1, axis=1)
    off = np.zeros(len(npe) + 1, dtype=np.int64)
    np.cumsum(npe, out=off[1:])
    return off


def node_coords(mesh: Mesh, orders: np.ndarray, family: int) -> np.ndarray:
    """Physical coordinates (3, n_nodes) of the solution nodes, from the continuous map ``mesh.cmap``."""
    orders = np.asarray(orders, dtype=np.int64)
    off = node_offsets(orders)
    out = np.empty((3, off[-1]))
    cache = {}
    for e in range(mesh.K):
        key = tuple(orders[e])
        if key not in cache:
            x1 = sample_nodes(key[0], family)
            x2 = sample_nodes(key[1], family)
            x3 = sample_nodes(key[2], family)
            Z, Y, X = np.meshgrid(x3, x2, x1, indexing="ij")
            cache[key] = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
        ref = cache[key]
        out[:, off[e]:off[e + 1]] = mesh.cmap(e, ref).T
    return out


# --------------------------------------------------------------------------------------------------
# Structured box meshes (optionally stretched, curved and periodic).
# --------------------------------------------------------------------------------------------------
def _equi(M: int) -> np.ndarray:
    return np.linspace(-1.0, 1.0, M + 1)


def _gnodes_from_cmap(K: int, M: Sequence[int], cmap) -> np.ndarray:
    Z, Y, X = np.meshgrid(_equi(M[2]), _equi(M[1]), _equi(M[0]), indexing="ij")
    ref = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    g = np.empty((K, M[2] + 1, M[1] + 1, M[0] + 1, 3))
    for e in range(K):
        g[e] = cmap(e, ref).reshape(M[2] + 1, M[1] + 1, M[0] + 1, 3)
    return g


def geometric_map(n: int, length: float, ratio: float):
    """Continuous index-space map s in [0, n] -> [0, length] whose cells grow by ``ratio``."""
    if abs(ratio - 1.0) < 1e-14:
        return lambda s: length * s / n
    h0 = length * (ratio - 1.0) / (ratio ** n - 1.0)
    return lambda s: h0 * (np.power(ratio, s) - 1.0) / (ratio - 1.0)


def box_mesh(n: Sequence[int], lo: Sequence[float], hi: Sequence[float], *, M=(1, 1, 1),
             periodic=(True, True, True), ratio=(1.0, 1.0, 1.0), bc_lo=(BC_FARFIELD,) * 3,
             bc_hi=(BC_FARFIELD,) * 3, wobble: float = 0.0, name: str = "box") -> Mesh:
    """Box of n[0] x n[1] x n[2] hexes; axis d stretched geometrically by ratio[d] towards lo[d].

    ``wobble`` adds a smooth periodic interior displacement (amplitude relative to the cell size) that
    makes the elements genuinely curved while keeping periodic faces matched.
    """
    nx, ny, nz = (int(v) for v in n)
    K = nx * ny * nz
    maps = [geometric_map(n[d], hi[d] - lo[d], ratio[d]) for d in range(3)]
    hmin = min((hi[d] - lo[d]) / n[d] for d in range(3))

    def cmap(e, ref):
        i = e % nx
        j = (e // nx) % ny
        k = e // (nx * ny)
        s1 = i + 0.5 * (ref[:, 0] + 1.0)
        s2 = j + 0.5 * (ref[:, 1] + 1.0)
        s3 = k + 0.5 * (ref[:, 2] + 1.0)
        x = lo[0] + maps[0](s1)
        y = lo[1] + maps[1](s2)
        z = lo[2] + maps[2](s3)
        if wobble:
            a = wobble * hmin
            p1, p2, p3 = 2 * np.pi * s1 / nx, 2 * np.pi * s2 / ny, 2 * np.pi * s3 / nz
            x = x + a * np.sin(p2) * np.sin(p3) * np.sin(p1)
            y = y + a * np.sin(p1) * np.sin(p3) * np.cos(p2 + 0.3) * np.sin(p2)
            z = z + a * np.sin(p1 + p2) * np.sin(p3) * np.sin(p1)
        return np.stack([x, y, z], axis=-1)

    gn = _gnodes_from_cmap(K, M, cmap)
    nbr = -np.ones((K, 6), dtype=np.int64)
    nf = np.zeros((K, 6), dtype=np.int8)
    orient = np.zeros((K, 6), dtype=np.int8)
    bc = np.zeros((K, 6), dtype=np.int32)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = i + nx * (j + ny * k)
                idx = [i, j, k]
                for f in range(6):
                    d, side = FACE_AXIS[f], FACE_SIDE[f]
                    m = list(idx)
                    m[d] += 1 if side else -1
                    if m[d] < 0 or m[d] >= n[d]:
                        if periodic[d]:
                            m[d] %= n[d]
                        else:
                            bc[e, f] = bc_hi[d] if side else bc_lo[d]
                            continue
                    nbr[e, f] = m[0] + nx * (m[1] + ny * m[2])
                    nf[e, f] = f ^ 1
    mesh = Mesh(K, tuple(int(v) for v in M), gn, nbr, nf, orient, bc, cmap, name)
    return mesh


# --------------------------------------------------------------------------------------------------
# Six-block cubed-sphere O-grid around a unit sphere.
# --------------------------------------------------------------------------------------------------
_PANELS = (  # (centre, t1, t2) with t1 x t2 = centre (right-handed element frames)
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
)


def _connect_by_corners(mesh_gn: np.ndarray, M: Sequence[int], period=None):
    """Link faces whose four corner points coincide (modulo ``period`` per axis when given) and derive the
    orientation codes from the corner correspondence."""
    K = mesh_gn.shape[0]
    scale = 1e6
    per = None if period is None else [None if p is None else int(round(p * scale)) for p in period]
    corners = {}
    nbr = -np.ones((K, 6), dtype=np.int64)
    nf = np.zeros((K, 6), dtype=np.int8)
    orient = np.zeros((K, 6), dtype=np.int8)
    local = ((-1, -1), (1, -1), (-1, 1), (1, 1))

    def quant(p):
        q = np.round(p * scale).astype(np.int64)
        if per is not None:
            for d in range(3):
                if per[d]:
                    q[..., d] = np.mod(q[..., d], per[d])
        return q

    def corner_pts(e, f):
        d, side = FACE_AXIS[f], FACE_SIDE[f]
        t1, t2 = TANGENTIAL[d]
        pts = []
        for s, t in local:
            ix = [0, 0, 0]
            ix[d] = M[d] if side else 0
            ix[t1] = M[t1] if s > 0 else 0
            ix[t2] = M[t2] if t > 0 else 0
            pts.append(mesh_gn[e, ix[2], ix[1], ix[0]])
        pts = np.array(pts)
        # the face centre disambiguates periodic directions with only two elements
        return quant(pts), quant(pts.mean(axis=0))

    pts_all = {}
    for e in range(K):
        for f in range(6):
            p, c = corner_pts(e, f)
            pts_all[(e, f)] = p
            corners.setdefault((tuple(sorted(tuple(q) for q in p)), tuple(c)), []).append((e, f))
    for key, lst in corners.items():
        if len(lst) == 1:
            continue
        assert len(lst) == 2, key
        (e, f), (g, h) = lst
        for a, b in (((e, f), (g, h)), ((g, h), (e, f))):
            pa, pb = pts_all[a], pts_all[b]
            found = None
            for o in range(8):
                ok = True
                for c, (s, t) in enumerate(local):
                    s2, t2 = orient_map(o, s, t)
                    cb = local.index((s2, t2))
                    if np.max(np.abs(pa[c] - pb[cb])) > 2:
                        ok = False
                        break
                if ok:
                    found = o
                    break
            assert found is not None, (a, b)
            nbr[a[0], a[1]] = b[0]
            nf[a[0], a[1]] = b[1]
            orient[a[0], a[1]] = found
    return nbr, nf, orient


def _rotations():
    """The 24 proper rotations of the reference cube as signed permutation matrices."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3))
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if np.linalg.det(R) > 0:
                out.append(R)
    return out


def reorient(mesh: Mesh, seed: int, period=None, orders: Optional[np.ndarray] = None):
    """Give every element a seeded random rotation of its reference frame (same physical mesh, new
    element frames and orientation codes).  Requires M1 = M2 = M3.  When ``orders`` is given, it is
    permuted with the frames so the discrete space stays the same; returns (mesh, orders)."""
    assert mesh.M[0] == mesh.M[1] == mesh.M[2]
    Mg = mesh.M[0]
    rng = np.random.default_rng(seed)
    rots = _rotations()
    pick = rng.integers(0, len(rots), size=mesh.K)
    eq = _equi(Mg)
    Z, Y, X = np.meshgrid(eq, eq, eq, indexing="ij")
    ref_new = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    gn = np.empty_like(mesh.gnodes)
    new_orders = None if orders is None else np.array(orders, copy=True)
    for e in range(mesh.K):
        R = rots[pick[e]]
        ref_old = ref_new @ R                      # xi_old = R^T xi_new
        idx = np.rint((ref_old + 1.0) * Mg / 2.0).astype(np.int64)
        gn[e] = mesh.gnodes[e][idx[:, 2], idx[:, 1], idx[:, 0]].reshape(gn[e].shape)
        if orders is not None:
            # new axis r runs along old axis perm[r]
            new_orders[e] = [orders[e][int(np.nonzero(R[r])[0][0])] for r in range(3)]
    old_cmap = mesh.cmap
    Rs = [rots[p] for p in pick]

    def cmap(e, ref):
        return old_cmap(e, ref @ Rs[e])

    nbr, nf, orient = _connect_by_corners(gn, mesh.M, period)
    bc = np.zeros_like(mesh.bc)
    # boundary tags follow the physical face: find the old face each new face came from
    for e in range(mesh.K):
        R = Rs[e]
        for f in range(6):
            if nbr[e, f] >= 0:
                continue
            d, side = FACE_AXIS[f], FACE_SIDE[f]
            n_new = np.zeros(3)
            n_new[d] = 1.0 if side else -1.0
            n_old = n_new @ R
            d_old = int(np.nonzero(n_old)[0][0])
            f_old = 2 * d_old + (1 if n_old[d_old] > 0 else 0)
            bc[e, f] = mesh.bc[e, f_old]
            assert bc[e, f] != BC_NONE
    out = Mesh(mesh.K, mesh.M, gn, nbr, nf, orient, bc, cmap, mesh.name + f"_rot{seed}")
    return out, new_orders


def ogrid_mesh(nt: int = 8, nr: int = 13, r_in: float = 1.0, r_out: float = 20.0, ratio: float = 1.25,
               M=(2, 2, 2), name: str = "ogrid") -> Mesh:
    """6 panels of nt x nt x nr hexes between spheres r_in and r_out, geometric radial spacing."""
    K = 6 * nt * nt * nr
    rmap = geometric_map(nr, r_out - r_in, ratio)
    P = [tuple(np.array(v, dtype=float) for v in p) for p in _PANELS]

    def cmap(e, ref):
        p = e // (nt * nt * nr)
        rem = e % (nt * nt * nr)
        i = rem % nt
        j = (rem // nt) % nt
        k = rem // (nt * nt)
        u = -1.0 + 2.0 * (i + 0.5 * (ref[:, 0] + 1.0)) / nt
        v = -1.0 + 2.0 * (j + 0.5 * (ref[:, 1] + 1.0)) / nt
        s = k + 0.5 * (ref[:, 2] + 1.0)
        a = np.tan(0.25 * np.pi * u)
        b = np.tan(0.25 * np.pi * v)
        c, t1, t2 = P[p]
        cube = c[None, :] + a[:, None] * t1[None, :] + b[:, None] * t2[None, :]
        dirn = cube / np.linalg.norm(cube, axis=1, keepdims=True)
        r = r_in + rmap(s)
        return dirn * r[:, None]

    gn = _gnodes_from_cmap(K, M, cmap)
    nbr, nf, orient = _connect_by_corners(gn, M)
    bc = np.zeros((K, 6), dtype=np.int32)
    for e in range(K):
        k = (e % (nt * nt * nr)) // (nt * nt)
        for f in range(6):
            if nbr[e, f] < 0:
                assert f in (4, 5), (e, f)
                bc[e, f] = BC_WALL if f == 4 else BC_FARFIELD
                assert (f == 4 and k == 0) or (f == 5 and k == nr - 1)
    mesh = Mesh(K, tuple(int(v) for v in M), gn, nbr, nf, orient, bc, cmap, name)
    return mesh


# --------------------------------------------------------------------------------------------------
# Orders and states.
# --------------------------------------------------------------------------------------------------
def uniform_orders(K: int, N: Sequence[int]) -> np.ndarray:
    return np.tile(np.asarray(N, dtype=np.int32)[None, :], (K, 1))


def random_orders(K: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(K, 3)).astype(np.int32)


def conserved(rho, u, v, w, p, gamma: float = 1.4) -> np.ndarray:
    """Stack a primitive field into the conserved input layout (rho, rho u, rho v, rho w, rho e)."""
    rho = np.asarray(rho, dtype=np.float64)
    E = np.asarray(p) / (gamma - 1.0) + 0.5 * rho * (np.asarray(u) ** 2 + np.asarray(v) ** 2 + np.asarray(w) ** 2)
    return np.stack([rho, rho * u, rho * v, rho * w, E]).astype(np.float64)


def freestream_state(n_nodes: int, mach: float, gamma: float = 1.4) -> np.ndarray:
    one = np.ones(n_nodes)
    return conserved(one, one, 0 * one, 0 * one, one / (gamma * mach * mach), gamma)


def box_wave_state(mesh: Mesh, orders, family: int, mach: float, gamma: float = 1.4,
                   amp: float = 1e-3, seed: int = 1) -> np.ndarray:
    """Smooth sinusoidal field times a seeded uniform (1 + amp*U(-1,1)) perturbation per nodal value."""
    x, y, z = node_coords(mesh, orders, family)
    pinf = 1.0 / (gamma * mach * mach)
    pi = np.pi
    rho = 1.0 + 0.1 * np.sin(pi * (x + y + z))
    u = 1.0 + 0.1 * np.sin(pi * y)
    v = 0.1 * np.sin(pi * z)
    w = 0.1 * np.sin(pi * x)
    p = pinf * (1.0 + 0.1 * np.cos(pi * (x - y + z)))
    Q = conserved(rho, u, v, w, p, gamma)
    if amp:
        rng = np.random.default_rng(seed)
        Q = Q * (1.0 + amp * rng.uniform(-1.0, 1.0, size=Q.shape))
    return Q


def perturbed_freestream(n_nodes: int, mach: float, amp: float, seed: int, gamma: float = 1.4) -> np.ndarray:
    Q = freestream_state(n_nodes, mach, gamma)
    rng = np.random.default_rng(seed)
    return Q * (1.0 + amp * rng.uniform(-1.0, 1.0, size=Q.shape))


def random_source(n_nodes: int, scale: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * rng.uniform(-1.0, 1.0, size=(5, n_nodes))


# --------------------------------------------------------------------------------------------------
# The workloads.
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Physics:
    mach: float = 0.2
    reynolds: float = 200.0
    prandtl: float = 0.72
    gamma: float = 1.4
    sutherland: float = 110.4 / 288.15
    cfl_adv: float = 0.5
    cfl_visc: float = 0.25
    family: int = FAMILY_LG
    viscosity: int = 0      # 0 Sutherland, 1 constant


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    orders: np.ndarray
    phys: Physics
    Q: np.ndarray
    S: Optional[np.ndarray] = None
    level_caps: Optional[list] = None

    @property
    def n_nodes(self) -> int:
        return int(node_offsets(self.orders)[-1])


def config_box(seed: int = 1, n: int = 4, N: int = 3) -> Workload:
    """Periodic [-1,1]^3 box of n^3 affine hexes, isotropic N, LGL, Mach 0.1, Re 100."""
    mesh = box_mesh((n, n, n), (-1, -1, -1), (1, 1, 1), M=(1, 1, 1), name=f"box{n}")
    orders = uniform_orders(mesh.K, (N, N, N))
    phys = Physics(mach=0.1, reynolds=100.0, family=FAMILY_LGL)
    Q = box_wave_state(mesh, orders, phys.family, phys.mach, seed=seed)
    return Workload(f"box{n}_N{N}_lgl", mesh, orders, phys, Q, None, [N, 1])


def plate_mesh(nx: int = 64, ny: int = 32, ratio: float = 1.1) -> Mesh:
    return box_mesh((nx, ny, 1), (0.0, 0.0, 0.0), (1.0, 0.5, 0.05), M=(2, 2, 1),
                    periodic=(False, False, True), ratio=(1.0, ratio, 1.0),
                    bc_lo=(BC_FARFIELD, BC_WALL, BC_NONE), bc_hi=(BC_FARFIELD, BC_FARFIELD, BC_NONE),
                    name=f"plate{nx}x{ny}")


def plate_mesh_inflow_outflow(nx: int = 64, ny: int = 32, ratio: float = 1.1, x_lead: float = 0.25) -> Mesh:
    """The plate mesh with the boundary layout of the paper's flat-plate case: uniform inflow (the far-field
    state) at x = 0, free slip on y = 0 ahead of the plate (x < x_lead), the no-slip adiabatic plate behind
    it, subsonic pressure outflow on the top and right sides."""
    m = plate_mesh(nx, ny, ratio)
    bc = m.bc.copy()
    for e in range(m.K):
        g = m.gnodes[e]
        xc = 0.5 * (g[..., 0].min() + g[..., 0].max())
        for f in range(6):
            if m.nbr_elem[e, f] >= 0:
                continue
            if f == 2:  # y = 0
                bc[e, f] = BC_FREESLIP if xc < x_lead else BC_WALL
            elif f in (1, 3):  # x = 1, y = 0.5
                bc[e, f] = BC_OUTFLOW
    out = dataclasses.replace(m, bc=bc, name=f"plate{nx}x{ny}_io")
    out.validate()
    return out


def config_plate(nx: int = 64, ny: int = 32, N=(6, 6, 1), seed: int = 2, amp: float = 1e-3) -> Workload:
    """Flat-plate boundary layer: stretched 64x32x1 hexes (ratio 1.1 to the wall), quadratic mapping,
    N=(6,6,1) Gauss nodes, Mach 0.2, Re_L 1e5; far-field start with a seeded perturbation."""
    mesh = plate_mesh(nx, ny)
    orders = uniform_orders(mesh.K, N)
    phys = Physics(mach=0.2, reynolds=1e5, family=FAMILY_LG)
    n_nodes = int(node_offsets(orders)[-1])
    Q = perturbed_freestream(n_nodes, phys.mach, amp, seed) if amp else freestream_state(n_nodes, phys.mach)
    return Workload(f"plate{nx}x{ny}_N{N[0]}{N[1]}{N[2]}", mesh, orders, phys, Q)


def config_batch(n: int = 64, kmin: int = 2000, kmax: int = 20000, seed: int = 4, lo: int = 2, hi: int = 5,
                 amp: float = 1e-3):
    """Independent steady problems: random boxes of kmin..kmax hexes (split into nx x ny x nz by seeded aspect
    draws), stretched toward a y = 0 no-slip wall by a ratio in [1, 1.15], far field on the other x / y
    sides, periodic in z, trilinear mapping; orders iid in [lo, hi] per direction (the maximum hi is present
    in every problem); Mach in [0.1, 0.4] and Re in [1e2, 1e4], all from the seed."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n):
        K = int(rng.integers(kmin, kmax + 1))
        a = rng.uniform(0.5, 2.0, size=3)
        nz = max(1, int(round((K / (a[0] * a[1])) ** (1 / 3) * a[2] ** 0)))
        base = max(1, int(round((K / nz) ** 0.5)))
        nx = max(1, int(round(base * a[0] / a[1])))
        ny = max(1, int(round(K / (nx * nz))))
        ratio = float(rng.uniform(1.0, 1.15))
        mesh = box_mesh((nx, ny, nz), (0.0, 0.0, 0.0), (1.0 * nx / max(nx, ny), 1.0 * ny / max(nx, ny), 0.1 * nz),
                        M=(1, 1, 1), periodic=(False, False, True), ratio=(1.0, ratio, 1.0),
                        bc_lo=(BC_FARFIELD, BC_WALL, BC_NONE), bc_hi=(BC_FARFIELD, BC_FARFIELD, BC_NONE),
                        name=f"batch{p}")
        orders = rng.integers(lo, hi + 1, size=(mesh.K, 3)).astype(np.int32)
        orders[int(rng.integers(0, mesh.K)), :] = hi
        mach = float(rng.uniform(0.1, 0.4))
        re = float(rng.uniform(1e2, 1e4))
        phys = Physics(mach=mach, reynolds=re, family=FAMILY_LG, cfl_adv=0.2, cfl_visc=0.2)
        n_nodes = int(node_offsets(orders)[-1])
        Q = perturbed_freestream(n_nodes, mach, amp, seed * 1000 + p)
        out.append(Workload(f"batch{p}_{nx}x{ny}x{nz}", mesh, orders, phys, Q))
    return out


def config_serve(n: int = 200, seed: int = 5, rate: float = 20.0, kmin: int = 1000, kmax: int = 50000,
                 lo: int = 1, hi: int = 7, re_lo: float = 1e2, re_hi: float = 1e4, tol: float = 1e-9,
                 ogrid_frac: float = 0.5):
    """A served stream of steady-solve requests: Poisson arrival times at 'rate' per second; each request a
    random stretched box as in config_batch (K ~ U{kmin..kmax}) or, with probability ogrid_frac, a six-block
    O-grid around the unit sphere (6 nt^2 nr ~ K hexes, outer radius 20, rotated frames); orders iid in
    [lo, hi] per direction; Mach in [0.1, 0.4], Re in [re_lo, re_hi]; far-field start.  Returns a list of
    (arrival time in seconds, Workload, tol), all from the seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(n):
        t += float(rng.exponential(1.0 / rate))
        K = int(rng.integers(kmin, kmax + 1))
        mach = float(rng.uniform(0.1, 0.4))
        re = float(rng.uniform(re_lo, re_hi))
        if rng.uniform() >= ogrid_frac:
            a = rng.uniform(0.5, 2.0, size=2)
            nz = max(1, int(round(K ** (1 / 3))))
            nx = max(1, int(round((K / nz) ** 0.5 * a[0] / a[1])))
            ny = max(1, int(round(K / (nx * nz))))
            ratio = float(rng.uniform(1.0, 1.15))
            mesh = box_mesh((nx, ny, nz), (0.0, 0.0, 0.0),
                            (1.0 * nx / max(nx, ny), 1.0 * ny / max(nx, ny), 0.1 * nz),
                            M=(1, 1, 1), periodic=(False, False, True), ratio=(1.0, ratio, 1.0),
                            bc_lo=(BC_FARFIELD, BC_WALL, BC_NONE), bc_hi=(BC_FARFIELD, BC_FARFIELD, BC_NONE),
                            name=f"serve{q}_box")
        else:
            nr = max(2, int(round((K / 6.0) ** (1 / 3) * rng.uniform(0.8, 1.25))))
            nt = max(1, int(round((K / (6.0 * nr)) ** 0.5)))
            mesh, _ = reorient(ogrid_mesh(nt, nr, r_out=20.0, ratio=1.25, name=f"serve{q}_ogrid"),
                               int(rng.integers(1 << 30)))
        orders = rng.integers(lo, hi + 1, size=(mesh.K, 3)).astype(np.int32)
        phys = Physics(mach=mach, reynolds=re, family=FAMILY_LG, cfl_adv=0.2, cfl_visc=0.2)
        n_nodes = int(node_offsets(orders)[-1])
        out.append((t, Workload(mesh.name, mesh, orders, phys, freestream_state(n_nodes, mach)), tol))
    return out


def config_ogrid(nt: int = 8, nr: int = 13, seed: int = 3, lo: int = 1, hi: int = 7, amp: float = 1e-3,
                 r_out: float = 20.0, ratio: float = 1.25, cfl: float = 0.2) -> Workload:
    """Six-block O-grid around the unit sphere (outer radius 20), quadratic mapping, iid orders in [lo,hi].
    Element frames are rotated with a seed, as a mesh generator would leave them, so the faces carry every
    orientation code.  Random low orders on curved elements need a smaller explicit step constant."""
    mesh, _ = reorient(ogrid_mesh(nt, nr, r_out=r_out, ratio=ratio), seed)
    orders = random_orders(mesh.K, lo, hi, seed)
    phys = Physics(mach=0.2, reynolds=200.0, family=FAMILY_LG, cfl_adv=cfl, cfl_visc=cfl)
    n_nodes = int(node_offsets(orders)[-1])
    Q = perturbed_freestream(n_nodes, phys.mach, amp, seed + 100)
    return Workload(f"ogrid{nt}x{nr}", mesh, orders, phys, Q)
