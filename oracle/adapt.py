"""Oracle of the truncation-error-driven anisotropic p-adaptation (test infrastructure only).

Plain Python / numpy, FP64, written from the paper's description (Sec. 3.3.2, computing the new polynomial
orders; the decoupled estimator, eq. AnisTruncError of Sec. 3.2.1; the order-jump rule eq. poljump2D of
Sec. 4.1.2 and the softened 3-D rule and wall conformity of Sec. 4.2.1).  Only ``tests/`` may import it; it
shares no code with the HIP library.

Per element, with reference orders P = (P1, P2, P3) and the decoupled directional truncation errors
tau_d(n) measured by the anisotropic 3V cycle for n < P_d (the element's infinity norm over nodes and
variables):

1. inner map: every combination N with measured orders n_min <= N_d < P_d in the directions that have
   estimates; tau(N) = tau_1(N_1) + tau_2(N_2) + tau_3(N_3);
2. if some N has tau(N) < tau_max, the one with the fewest degrees of freedom (N1+1)(N2+1)(N3+1) is chosen
   (ties: the lexicographically smallest triple);
3. otherwise each direction's tau_d is extrapolated to P_d <= n <= n_max_d by a least-squares fit of
   log tau_d(n) = a + b n over its measured orders (at least two), and the full map over n_min <= N_d <= n_max_d
   is searched the same way;
4. if no combination reaches tau_max, N_d = n_max_d in every direction with estimates.
A direction without estimates (P_d = 1, nothing to coarsen) keeps P_d and contributes nothing to the sum.

Afterwards the order-jump rule between face neighbours is enforced by raising the lower side until nothing
changes (a monotone fixed point, so the order of the sweeps does not matter), direction by direction through
the face orientation: rule 1, |N_i^+ - N_i^-| <= 1; rule 2, N_i^+ >= floor(2/3 N_i^-).  Optionally elements
that both touch a no-slip wall are made conforming across their common face (equal orders, the larger).

Multi-stage adaptation inside the FMG cycle (Sec. 3.3.4): stages at increasing orders P_1 < P_2 < ...; the
problem is converged at the current orders, its map estimated by the 3V cycle and the orders selected as above
but never above the next stage's order (the cap is applied before the jump rule); the adaptation ends at the
stage whose largest required order (before the cap) does not exceed the next stage's order, or at the last
stage.  The state follows every change of orders (per direction: interpolation up, L2 projection down), then
the adapted problem is solved to the final tolerance.
"""
from __future__ import annotations

import math

import numpy as np

BC_WALL = 1


def _fit(points):
    """Least-squares line through (n, log tau) for the given (n, tau) pairs, in ascending n: (a, b)."""
    m = len(points)
    sn = sl = snn = snl = 0.0
    for n, t in points:
        l = math.log(t)
        sn += n
        sl += l
        snn += n * n
        snl += n * l
    b = (m * snl - sn * sl) / (m * snn - sn * sn)
    a = (sl - b * sn) / m
    return a, b


def directional_table(P, tau_e, n_max, n_min):
    """tau_d(n) for every candidate order of each direction: list of dicts (None: direction without
    estimates), the inner and the extrapolated parts."""
    inner, full = [], []
    for d in range(3):
        meas = [(n, float(tau_e[d][n - 1])) for n in range(1, P[d]) if n - 1 < len(tau_e[d])
                and math.isfinite(float(tau_e[d][n - 1]))]
        if not meas:
            inner.append(None)
            full.append(None)
            continue
        tin = {n: t for n, t in meas if n >= n_min}
        tfull = dict(tin)
        pos = [(n, t) for n, t in meas if t > 0.0]
        if len(pos) >= 2:
            a, b = _fit(pos)
            for n in range(max(P[d], n_min), n_max[d] + 1):
                tfull[n] = math.exp(a + b * n)
        inner.append(tin)
        full.append(tfull)
    return inner, full


def _search(P, tables, tau_max):
    """Fewest-DOF combination with sum tau < tau_max (lexicographic tie-break), or None."""
    cand = []
    for d in range(3):
        cand.append([(P[d], 0.0)] if tables[d] is None else sorted(tables[d].items()))
    best = None
    for n1, t1 in cand[0]:
        for n2, t2 in cand[1]:
            for n3, t3 in cand[2]:
                tau = t1 + t2 + t3
                if not tau < tau_max:
                    continue
                key = ((n1 + 1) * (n2 + 1) * (n3 + 1), n1, n2, n3)
                if best is None or key < best:
                    best = key
    return None if best is None else [best[1], best[2], best[3]]


def element_orders(P, tau_e, tau_max, n_max, n_min=1):
    """New orders of one element (steps 1-4 above)."""
    inner, full = directional_table(P, tau_e, n_max, n_min)
    N = _search(P, inner, tau_max)
    if N is None:
        N = _search(P, full, tau_max)
    if N is None:
        N = [P[d] if inner[d] is None else n_max[d] for d in range(3)]
    return N


def face_directions(f, o):
    """Direction of the neighbour matching each of our directions across face f with orientation code o."""
    d = f // 2
    t1 = 1 if d == 0 else 0
    t2 = 1 if d == 2 else 2
    return d, t1, t2, (o & 4) != 0


def _neighbour_axes(h):
    dg = h // 2
    return dg, (1 if dg == 0 else 0), (1 if dg == 2 else 2)


def enforce_jumps(mesh, N, rule, wall_conforming=False):
    """Raise orders until the jump rule (and wall conformity) holds across every interior face."""
    N = np.array(N, dtype=np.int64).copy()
    wall = np.array([any(int(mesh.bc[e, f]) == BC_WALL and int(mesh.nbr_elem[e, f]) < 0 for f in range(6))
                     for e in range(mesh.K)])
    changed = True
    while changed:
        changed = False
        for e in range(mesh.K):
            for f in range(6):
                g = int(mesh.nbr_elem[e, f])
                if g < 0:
                    continue
                h = int(mesh.nbr_face[e, f])
                d, t1, t2, swap = face_directions(f, int(mesh.orient[e, f]))
                dg, s1, s2 = _neighbour_axes(h)
                pairs = [(d, dg), (t1, s2 if swap else s1), (t2, s1 if swap else s2)]
                for i, j in pairs:
                    need = N[e, i]
                    if rule == 1:
                        need = max(need, N[g, j] - 1)
                    elif rule == 2:
                        need = max(need, (2 * N[g, j]) // 3)
                    if wall_conforming and wall[e] and wall[g]:
                        need = max(need, N[g, j])
                    if need > N[e, i]:
                        N[e, i] = need
                        changed = True
    return N


def select_orders(mesh, orders, tau_map, tau_max, n_max, n_min=1, rule=1, wall_conforming=False, cap=None):
    """(new orders (K, 3), largest selected order before the cap) from the reference orders (K, 3) and the
    directional tau map [K][3][nt]; 'cap' (a stage's upper order) bounds the selection in every direction with
    estimates before the jump rule is enforced."""
    K = mesh.K
    out = np.zeros((K, 3), dtype=np.int64)
    for e in range(K):
        out[e] = element_orders([int(v) for v in orders[e]], tau_map[e], tau_max, list(n_max), n_min)
    max_required = int(out.max())
    if cap is not None:
        for e in range(K):
            for d in range(3):
                if out[e, d] > cap:
                    out[e, d] = cap
    if rule or wall_conforming:
        out = enforce_jumps(mesh, out, rule, wall_conforming)
    return out, max_required


def adapt_orders(mesh, orders, tau_map, tau_max, n_max, n_min=1, rule=1, wall_conforming=False, cap=None):
    """New orders (K, 3) (see select_orders)."""
    return select_orders(mesh, orders, tau_map, tau_max, n_max, n_min, rule, wall_conforming, cap)[0]


def multistage(ora, mesh, orders, stages, tau_max, n_max, n_min=1, rule=1, wall_conforming=False, conv=0.1,
               final_tol=1e-8, max_cycles=100, Q0=None, **mg):
    """Multi-stage adaptation from the first stage's orders, with the oracle's solver ('ora', an
    oracle.Oracle on 'mesh'); 'mg' are the multigrid parameters (the first solve may start with FMG, later
    ones continue V-cycling from the carried-over state).  Returns (orders, Q, reports, final cycles, final
    residual); a report per stage: dict(order, cycles, res, dof_before, dof_after, max_required, last)."""
    N = np.asarray(orders, dtype=np.int64).copy()
    Q = np.array(Q0, dtype=np.float64, copy=True)
    reports = []
    for i, P in enumerate(stages):
        prm = dict(mg)
        if i > 0:
            prm["fmg"] = 0
        Q, cyc, res, _ = ora.solve(N, Q, None, tol=conv * tau_max, max_cycles=max_cycles, **prm)
        tau, Q = ora.tau_3v(N, Q, None, **dict(prm, isolated=1))
        nxt = stages[i + 1] if i + 1 < len(stages) else None
        M, req = select_orders(mesh, N, tau, tau_max, n_max, n_min, rule, wall_conforming, nxt)
        last = nxt is None or req <= nxt
        dof0 = int(np.prod(N + 1, axis=1).sum())
        Q = ora.remap(N, M, Q)
        reports.append(dict(order=int(P), cycles=cyc, res=res, dof_before=dof0,
                            dof_after=int(np.prod(M + 1, axis=1).sum()), max_required=req, last=bool(last)))
        N = M
        if last:
            break
    prm = dict(mg, fmg=0)
    Q, cyc, res, _ = ora.solve(N, Q, None, tol=final_tol, max_cycles=max_cycles, **prm)
    return N, Q, reports, cyc, res
