"""Independent reference solutions used to pin the oracle.

Nothing here runs HPR-QP: these are textbook solution methods for the same
convex QP (KKT enumeration, closed forms, bisection, a direct KKT solve) and
first-principles optimality checks of the subproblems of Algorithm 3.
"""
from __future__ import annotations

import itertools

import numpy as np


def kkt_enumerate(Q, c, L, U, A, l, u, tol=1e-9):
    """Brute-force active-set enumeration for a tiny convex QP.

    Every variable sits at L_j, at U_j or is free; every inequality row sits
    at l_i, at u_i or is inactive; equality rows (l_i == u_i) are always
    active.  For each pattern solve the linear KKT system
        Q x + c - A_act^T y_act - z_bnd = 0,  a_i x = bound_i,  x_j = bound_j
    (least squares, so PSD Q is handled), keep the points that are primal
    feasible with multipliers of the right sign
        y_i >= 0 at a lower bound, y_i <= 0 at an upper bound,
        z_j >= 0 at L_j,          z_j <= 0 at U_j,
    and return (obj, x, y, z) of the best one.
    """
    Q = np.asarray(Q, float); c = np.asarray(c, float)
    A = np.asarray(A, float).reshape(-1, len(c))
    n, m = len(c), A.shape[0]
    var_states = []
    for j in range(n):
        s = ["free"]
        if np.isfinite(L[j]): s.append("L")
        if np.isfinite(U[j]): s.append("U")
        var_states.append(s)
    row_states = []
    for i in range(m):
        if l[i] == u[i]:
            row_states.append(["eq"])
        else:
            s = ["off"]
            if np.isfinite(l[i]): s.append("l")
            if np.isfinite(u[i]): s.append("u")
            row_states.append(s)
    best = None
    for vs in itertools.product(*var_states):
        bnd = [j for j in range(n) if vs[j] != "free"]
        for rs in itertools.product(*row_states):
            act = [i for i in range(m) if rs[i] != "off"]
            na, nb = len(act), len(bnd)
            N = n + na + nb
            K = np.zeros((N, N)); rhs = np.zeros(N)
            # stationarity: Q x - A_act^T y - E^T z = -c
            K[:n, :n] = Q
            for a, i in enumerate(act):
                K[:n, n + a] = -A[i]
            for b, j in enumerate(bnd):
                K[j, n + na + b] = -1.0
            rhs[:n] = -c
            for a, i in enumerate(act):
                K[n + a, :n] = A[i]
                rhs[n + a] = l[i] if rs[i] in ("eq", "l") else u[i]
            for b, j in enumerate(bnd):
                K[n + na + b, j] = 1.0
                rhs[n + na + b] = L[j] if vs[j] == "L" else U[j]
            sol, *_ = np.linalg.lstsq(K, rhs, rcond=None)
            if np.linalg.norm(K @ sol - rhs) > 1e-8 * (1 + np.linalg.norm(rhs)):
                continue
            x = sol[:n]
            ok = np.all(x >= L - tol) and np.all(x <= U + tol)
            Ax = A @ x
            ok = ok and np.all(Ax >= l - tol) and np.all(Ax <= u + tol)
            y = np.zeros(m); z = np.zeros(n)
            for a, i in enumerate(act):
                y[i] = sol[n + a]
                if rs[i] == "l" and y[i] < -tol: ok = False
                if rs[i] == "u" and y[i] > tol: ok = False
            for b, j in enumerate(bnd):
                z[j] = sol[n + na + b]
                if vs[j] == "L" and z[j] < -tol: ok = False
                if vs[j] == "U" and z[j] > tol: ok = False
            if not ok:
                continue
            obj = 0.5 * x @ Q @ x + c @ x
            if best is None or obj < best[0] - 1e-12:
                best = (obj, x, y, z)
    return best


def diag_box_closed_form(d, c, L, U):
    """min 1/2 sum d_j x_j^2 + c'x over the box: x* = clip(-c/d, L, U)."""
    return np.clip(-c / d, L, U)


def diag_budget_bisect(d, c, L, U, total=1.0, iters=200):
    """min 1/2 sum d_j x_j^2 + c'x s.t. sum x = total, L <= x <= U.
    Stationarity gives x(nu) = clip((nu - c)/d, L, U), nondecreasing in nu;
    bisect sum x(nu) = total."""
    lo, hi = -1e6, 1e6
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.clip((mid - c) / d, L, U).sum() < total:
            lo = mid
        else:
            hi = mid
    nu = 0.5 * (lo + hi)
    return np.clip((nu - c) / d, L, U), nu


def equality_kkt(Q, c, A, b):
    """min 1/2 x'Qx + c'x s.t. Ax = b (Q PD): [[Q, -A^T], [A, 0]] [x; y] = [-c; b]."""
    n, m = Q.shape[0], A.shape[0]
    K = np.block([[Q, -A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-c, b]))
    return sol[:n], sol[n:]


def dense_metric_M(Q, A, sigma, lamA, lamQ):
    """Assemble the metric M of Algorithm 3 ("eq:metric-M") densely in the
    coordinates (y, omega, x), where w = V omega and the columns of V are an
    orthonormal basis of Range(Q) (the z-block of M is zero).

    T_1 = S + S_sGS with S = sigma diag(S_y, S_w), S_y = lamA I - A A^T,
    S_w = Q (lamQ I - Q), and S_sGS1 = sigma^2 A Q (sigma Q^2 + Q + sigma S_w)^{-1} Q A^T
    with the inverse taken on Range(Q).
    """
    n = Q.shape[0]; m = A.shape[0]
    ev, V = np.linalg.eigh(Q)
    V = V[:, ev > 1e-10 * max(1.0, ev.max())]
    r = V.shape[1]
    AQ = np.hstack([A.T, -Q @ V])                    # A_Q (y, omega) = A^T y - Q V omega
    Sy = lamA * np.eye(m) - A @ A.T
    Sw = V.T @ (Q @ (lamQ * np.eye(n) - Q)) @ V
    S = sigma * np.block([[Sy, np.zeros((m, r))], [np.zeros((r, m)), Sw]])
    Wop = V.T @ (sigma * Q @ Q + Q + sigma * Q @ (lamQ * np.eye(n) - Q)) @ V
    Winv = V @ np.linalg.inv(Wop) @ V.T
    S1 = sigma ** 2 * A @ Q @ Winv @ Q @ A.T
    Ssgs = np.zeros((m + r, m + r)); Ssgs[:m, :m] = S1
    top = sigma * AQ.T @ AQ + S + Ssgs
    M = np.block([[top, AQ.T], [AQ, np.eye(n) / sigma]])
    return M, V


def kkt_residual_numpy(Q, c, L, U, A, l, u, x, y, z):
    """max(eta_p, eta_d, eta_gap) computed directly with numpy (dense)."""
    Ax = A @ x; Qx = Q @ x; ATy = A.T @ y
    bvec = np.maximum(np.where(np.isinf(l), 0, np.abs(l)), np.where(np.isinf(u), 0, np.abs(u)))
    eta_p = np.max(np.abs(Ax - np.clip(Ax, l, u)), initial=0.0) / (1 + max(np.max(bvec, initial=0), np.max(np.abs(Ax), initial=0)))
    eta_d = np.max(np.abs(-Qx + ATy + z - c)) / (1 + max(np.max(np.abs(c)), np.max(np.abs(ATy)), np.max(np.abs(Qx))))
    P = 0.5 * x @ Qx + c @ x
    def supp(v, lo, hi):
        s = 0.0
        for vi, a, b in zip(v, lo, hi):
            if vi > 0: s += a * vi
            elif vi < 0: s += b * vi
        return s
    D = -0.5 * x @ Qx + supp(y, l, u) + supp(z, L, U)
    return max(eta_p, eta_d, abs(P - D) / (1 + max(abs(P), abs(D)))), P, D
