"""Direct solutions the CADMM iteration must converge to (no iteration inside).

* ``kkt_reference``: the unconstrained minimum-effort problem of Sec. III-A
  (piecewise form, eq. ``continously_differentiable_constraints`` with
  continuity of orders 0..s-1, end states of eq. ``start_points_constraints``,
  interior positions pinned or free) solved as one equality-constrained QP
  through its KKT system, per axis.
* ``optimality_reference``: the square system of the optimality conditions of
  Sec. III-D.2 (degree 2p-1, end states to order p-1, positions at every knot,
  continuity to order 2p-2), per axis.  Its solution is the minimum-effort
  spline through the waypoints, so it must equal ``kkt_reference`` with pinned
  positions.
* ``constrained_reference``: the same QP plus the box rows and the velocity
  balls at the sample instants, handed to scipy's general constrained solver.

All three return monomial coefficients [S, 3, n] and the cost per trajectory.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize
import scipy.sparse
import scipy.sparse.linalg

from .cadmm import Problem, end_states, sample_times
from .polynomial import beta, cost_gram


def _np(x):
    return x.detach().cpu().numpy()


def _row(o, t, d):
    return _np(beta(o, np.float64(t), d))


def _traj_ranges(pr: Problem):
    for b in range(pr.B):
        yield b, int(pr.seg_offsets[b]), int(pr.seg_offsets[b + 1])


def _equality_rows(pr: Problem, b: int, s0: int, s1: int, a: int, cont_orders: int, pin: bool):
    """Rows (E, e) for one axis of one trajectory: end states, knot positions, continuity."""
    n, d, p = pr.n, pr.d, pr.p
    N = s1 - s0
    T = _np(pr.T)[s0:s1]
    P = _np(pr.P)[s0 + b: s1 + b + 1, a]
    ends = _np(end_states(pr))[b]        # [2, p, 3]
    rows, rhs = [], []

    def put(entries, val):
        r = np.zeros(N * n)
        for seg, vec in entries:
            r[seg * n:(seg + 1) * n] += vec
        rows.append(r)
        rhs.append(val)

    for o in range(p):
        put([(0, _row(o, 0.0, d))], ends[0, o, a])
        put([(N - 1, _row(o, T[N - 1], d))], ends[1, o, a])
    for k in range(N - 1):
        if pin:
            put([(k, _row(0, T[k], d))], P[k + 1])
            put([(k + 1, _row(0, 0.0, d))], P[k + 1])
        else:
            put([(k, _row(0, T[k], d)), (k + 1, -_row(0, 0.0, d))], 0.0)
        for o in range(1, cont_orders):
            put([(k, _row(o, T[k], d)), (k + 1, -_row(o, 0.0, d))], 0.0)
    return np.array(rows), np.array(rhs)


def _cost(pr: Problem, c: np.ndarray) -> np.ndarray:
    Q = _np(cost_gram(pr.T, pr.p, pr.d))
    per = np.einsum("sai,sij,saj->s", c, Q, c)
    J = np.zeros(pr.B)
    np.add.at(J, _np(pr.traj), per)
    return J


def kkt_reference(pr: Problem, pin=None):
    """Unconstrained optimum by the KKT system [2Q E^T; E 0][c; lam] = [0; e], per axis (sparse LU)."""
    pin = pr.fix_interior if pin is None else pin
    n = pr.n
    out = np.zeros((pr.S, 3, n))
    Qall = _np(cost_gram(pr.T, pr.p, pr.d))
    for b, s0, s1 in _traj_ranges(pr):
        N = s1 - s0
        Q = scipy.sparse.block_diag([2.0 * Qall[i] for i in range(s0, s1)])
        for a in range(3):
            E, e = _equality_rows(pr, b, s0, s1, a, pr.s, pin)
            m = E.shape[0]
            Es = scipy.sparse.csr_matrix(E)
            K = scipy.sparse.bmat([[Q, Es.T], [Es, None]], format="csc")
            rhs = np.concatenate([np.zeros(N * n), e])
            sol = scipy.sparse.linalg.spsolve(K, rhs)
            out[s0:s1, a, :] = sol[:N * n].reshape(N, n)
    return out, _cost(pr, out)


def optimality_reference(pr: Problem):
    """Square optimality-condition system of Sec. III-D.2 (pinned positions, continuity to 2p-2)."""
    n, p = pr.n, pr.p
    out = np.zeros((pr.S, 3, n))
    for b, s0, s1 in _traj_ranges(pr):
        for a in range(3):
            E, e = _equality_rows(pr, b, s0, s1, a, 2 * p - 1, True)
            assert E.shape[0] == E.shape[1], E.shape
            out[s0:s1, a, :] = np.linalg.solve(E, e).reshape(s1 - s0, n)
    return out, _cost(pr, out)


def constrained_reference(pr: Problem, tol: float = 1e-15, maxiter: int = 2000, vel_norm: int = 2):
    """Corridor- (box or polytope) and velocity-constrained optimum of one trajectory by scipy's SLSQP
    (tiny N only); the speed bound is ||v||_q <= vmax at the samples, q = vel_norm (2 or 4)."""
    assert pr.B == 1
    n, d, S = pr.n, pr.d, pr.S
    Q = _np(cost_gram(pr.T, pr.p, pr.d))
    nv = S * 3 * n

    def unpack(x):
        return x.reshape(S, 3, n)

    def f(x):
        c = unpack(x)
        return float(np.einsum("sai,sij,saj->", c, Q, c))

    def grad(x):
        c = unpack(x)
        return (2.0 * np.einsum("sij,saj->sai", Q, c)).reshape(-1)

    cons = []
    rows, rhs = [], []
    for a in range(3):
        E, e = _equality_rows(pr, 0, 0, S, a, pr.s, pr.fix_interior)
        for r, v in zip(E, e):
            full = np.zeros((S, 3, n))
            full[:, a, :] = r.reshape(S, n)
            rows.append(full.reshape(-1))
            rhs.append(v)
    cons.append(scipy.optimize.LinearConstraint(np.array(rows), np.array(rhs), np.array(rhs)))
    ts = _np(sample_times(pr))
    if pr.lo is not None:
        lo, hi = _np(pr.lo), _np(pr.hi)
        A, l, u = [], [], []
        for i in range(S):
            for j in range(pr.n_samples):
                bj = _row(0, ts[i, j], d)
                for a in range(3):
                    r = np.zeros((S, 3, n))
                    r[i, a, :] = bj
                    A.append(r.reshape(-1))
                    l.append(lo[i, a])
                    u.append(hi[i, a])
        cons.append(scipy.optimize.LinearConstraint(np.array(A), np.array(l), np.array(u)))
    if pr.faces is not None:
        F = _np(pr.faces)
        A, u = [], []
        for i in range(S):
            for j in range(pr.n_samples):
                bj = _row(0, ts[i, j], d)
                for k in range(F.shape[1]):
                    r = np.zeros((S, 3, n))
                    r[i] = F[i, k, :3, None] * bj[None, :]
                    A.append(r.reshape(-1))
                    u.append(F[i, k, 3])
        cons.append(scipy.optimize.LinearConstraint(np.array(A), -np.inf, np.array(u)))
    if pr.vmax is not None:
        vm = float(_np(pr.vmax)[0])
        D = []
        for i in range(S):
            for j in range(pr.n_samples):
                D.append((i, _row(1, ts[i, j], d)))

        q = vel_norm

        def vfun(x):
            c = unpack(x)
            return np.array([float((np.abs(c[i] @ r) ** q).sum()) for i, r in D])

        def vjac(x):
            c = unpack(x)
            J = np.zeros((len(D), nv))
            for k, (i, r) in enumerate(D):
                v = c[i] @ r
                g = np.zeros((S, 3, n))
                g[i] = (q * np.abs(v) ** (q - 1) * np.sign(v))[:, None] * r[None, :]
                J[k] = g.reshape(-1)
            return J

        cons.append(scipy.optimize.NonlinearConstraint(vfun, -np.inf, vm ** q, jac=vjac))
    # Feasible-ish start: the unconstrained optimum.
    x0, _ = kkt_reference(pr)
    res = scipy.optimize.minimize(f, x0.reshape(-1), jac=grad, method="SLSQP", constraints=cons,
                                  options={"ftol": tol, "maxiter": maxiter})
    c = unpack(res.x)
    return c, _cost(pr, c), res
