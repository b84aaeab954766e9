"""Seeded synthetic convex-QP instances for HPR-QP.

This module only *generates* problem data (numpy + scipy.sparse); it holds
none of the solver's arithmetic.  Both the CPU oracle (``oracle/``) and the
GPU library (``paper_2507_02470_amd``) consume the :class:`QP` objects built
here, and neither of them is imported by this module.

Problem form (paper, Section 1, problem "QP-primal"):

    min  1/2 <x, Q x> + <c, x> + lambda ||x||_1   s.t.  l <= A x <= u,   L <= x <= U

with Q self-adjoint PSD given either as an explicit CSR matrix, as the
Kronecker product B (x) C applied matrix-free, as diag(d) + F F^T, as the
Gram matrix Ahat^T Ahat of a sparse Ahat (applied matrix-free), or as 0;
lambda = ``l1_weight`` (0 for the CQP "QP-primal-0").  Infinite bounds are
IEEE +-inf.

Workloads (all seeded with ``numpy.random.default_rng``):

* ``make_small_ccqp``   tiny random CCQP (n=200, m=100), explicit sparse Q.
* ``make_random_large`` OSQP-style "random" class at scale (n=1e6, m=5e5).
* ``make_kron``          matrix-free Q = B (x) C with assignment constraints
                         (the QAP-relaxation structure of Section 4.5).
* ``make_qap``           the synthetic QAP relaxation of Section 4.5, Q = 2(Bhat (x)
                         Ahat - I (x) S - T (x) I), S and T from ``qap_st``.
* ``make_portfolio``     portfolio-style QP, Q = F F^T + D, budget + sector rows.
* ``make_portfolio_family`` a fixed portfolio instance plus per-sample
                         perturbations of c and of the sector bounds.
* ``make_tiny``          very small random QPs for brute-force checks.
* ``make_lasso``         Lasso 1/2||Ahat x - bhat||^2 + lambda ||x||_1 (Section
                         4.4), Q = Ahat^T Ahat matrix-free, c = -Ahat^T bhat, m = 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

QKINDS = ("zero", "csr", "kron", "lowrank", "gram")


@dataclass
class QP:
    n: int
    m: int
    qkind: str
    c: np.ndarray
    L: np.ndarray
    U: np.ndarray
    a_rowptr: np.ndarray
    a_col: np.ndarray
    a_val: np.ndarray
    l: np.ndarray
    u: np.ndarray
    q_rowptr: Optional[np.ndarray] = None
    q_col: Optional[np.ndarray] = None
    q_val: Optional[np.ndarray] = None
    kron_B: Optional[np.ndarray] = None   # p x p (Q = B (x) C)
    kron_C: Optional[np.ndarray] = None   # s x s
    kron_S: Optional[np.ndarray] = None   # s x s (QAP relaxation: Q = B (x) C - I (x) S - T (x) I)
    kron_T: Optional[np.ndarray] = None   # p x p
    lr_d: Optional[np.ndarray] = None     # n
    lr_F: Optional[np.ndarray] = None     # n x r, row-major
    gram_rowptr: Optional[np.ndarray] = None   # Ahat (p x n) CSR, Q = Ahat^T Ahat
    gram_col: Optional[np.ndarray] = None
    gram_val: Optional[np.ndarray] = None
    gram_p: int = 0
    l1_weight: float = 0.0                # lambda of phi(x) = lambda ||x||_1 + box
    meta: dict = field(default_factory=dict)

    # ---- convenience (data plumbing only) ----
    @property
    def a_nnz(self) -> int:
        return int(self.a_rowptr[-1])

    @property
    def q_nnz(self) -> int:
        return 0 if self.q_rowptr is None else int(self.q_rowptr[-1])

    def A_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.a_val, self.a_col, self.a_rowptr), shape=(self.m, self.n))

    def Q_dense(self) -> np.ndarray:
        """Dense Q (small instances only; used by tests)."""
        if self.qkind == "zero":
            return np.zeros((self.n, self.n))
        if self.qkind == "csr":
            return sp.csr_matrix((self.q_val, self.q_col, self.q_rowptr),
                                 shape=(self.n, self.n)).toarray()
        if self.qkind == "kron":
            Q = np.kron(self.kron_B, self.kron_C)
            if self.kron_S is not None:
                Q -= np.kron(np.eye(self.kron_B.shape[0]), self.kron_S)
            if self.kron_T is not None:
                Q -= np.kron(self.kron_T, np.eye(self.kron_C.shape[0]))
            return Q
        if self.qkind == "lowrank":
            return np.diag(self.lr_d) + self.lr_F @ self.lr_F.T
        if self.qkind == "gram":
            Ah = self.Ahat_scipy().toarray()
            return Ah.T @ Ah
        raise ValueError(self.qkind)

    def Ahat_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.gram_val, self.gram_col, self.gram_rowptr), shape=(self.gram_p, self.n))

    def copy(self) -> "QP":
        import copy as _c
        return _c.deepcopy(self)


def _csr_arrays(M: sp.spmatrix):
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    return (np.ascontiguousarray(M.indptr, dtype=np.int32),
            np.ascontiguousarray(M.indices, dtype=np.int32),
            np.ascontiguousarray(M.data, dtype=np.float64))


def _bernoulli_sparse(rng, rows, cols, density):
    """rows x cols matrix, each entry nonzero with prob `density`, N(0,1) values."""
    mask = rng.random((rows, cols)) < density
    vals = rng.standard_normal((rows, cols))
    return sp.csr_matrix(np.where(mask, vals, 0.0))


def from_dense(Q, c, L, U, A, l, u, qkind="csr") -> QP:
    """Build a QP from dense arrays (tests and small cases)."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    n = len(c)
    if A.size == 0:
        A = np.zeros((0, n))
    m = A.shape[0]
    ar, ac, av = _csr_arrays(sp.csr_matrix(A))
    kw = {}
    if qkind == "csr":
        qr, qc, qv = _csr_arrays(sp.csr_matrix(np.asarray(Q, dtype=np.float64)))
        kw = dict(q_rowptr=qr, q_col=qc, q_val=qv)
    elif qkind != "zero":
        raise ValueError("from_dense supports csr/zero")
    return QP(n=n, m=m, qkind=qkind, c=np.asarray(c, float).copy(), L=np.asarray(L, float).copy(),
              U=np.asarray(U, float).copy(), a_rowptr=ar, a_col=ac, a_val=av,
              l=np.asarray(l, float).reshape(m).copy(), u=np.asarray(u, float).reshape(m).copy(), **kw)


# ---------------------------------------------------------------------------
# Tiny small-CCQP workload: n=200, m=100
# ---------------------------------------------------------------------------
def make_small_ccqp(seed: int = 1000, n: int = 200, m: int = 100, nb: int = 50,
                    density: float = 0.05) -> QP:
    """Q = B^T B + 0.01 I (B nb x n, 5% N(0,1)); A m x n at 5% N(0,1);
    x0 ~ U(-5,5); first half rows equality l=u=A x0, second half l=-inf,
    u = A x0 + U(0,1); box [-10,10]; c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    B = _bernoulli_sparse(rng, nb, n, density)
    Q = (B.T @ B + 0.01 * sp.identity(n)).tocsr()
    A = _bernoulli_sparse(rng, m, n, density)
    x0 = rng.uniform(-5.0, 5.0, n)
    Ax0 = A @ x0
    half = m // 2
    l = np.empty(m); u = np.empty(m)
    l[:half] = Ax0[:half]; u[:half] = Ax0[:half]
    l[half:] = -np.inf; u[half:] = Ax0[half:] + rng.uniform(0.0, 1.0, m - half)
    c = rng.standard_normal(n)
    qr, qc, qv = _csr_arrays(Q)
    ar, ac, av = _csr_arrays(A)
    return QP(n=n, m=m, qkind="csr", c=c, L=np.full(n, -10.0), U=np.full(n, 10.0),
              a_rowptr=ar, a_col=ac, a_val=av, l=l, u=u, q_rowptr=qr, q_col=qc, q_val=qv,
              meta=dict(workload="small_ccqp", seed=seed, x_feasible=x0))


# ---------------------------------------------------------------------------
# Large random class: n=1e6, m=5e5, ~10 nnz/row in A, Q = D + S
# ---------------------------------------------------------------------------
def make_random_large(seed: int = 1001, n: int = 1_000_000, m: int = 500_000,
                      nnz_per_row: int = 10, pairs_per_row: int = 2) -> QP:
    """A: `nnz_per_row` uniformly random columns per row, N(0,1) values.
    Q = D + S, D ~ U(0.1,1) diagonal, S symmetric with `pairs_per_row`
    random off-diagonal pairs per row (N(0,1)) and diagonal sum|offdiag|+1e-3,
    so S is diagonally dominant (PSD) and nnz(Q) ~ 5 n.
    x0 ~ U(0,10) (inside the box [0,10]); half the rows equality l=u=A x0,
    the other half l=-inf, u = A x0 + U(0,1); c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(m, dtype=np.int64), nnz_per_row)
    cols = rng.integers(0, n, size=m * nnz_per_row, dtype=np.int64)
    vals = rng.standard_normal(m * nnz_per_row)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sum_duplicates()
    # symmetric off-diagonal part
    i = np.repeat(np.arange(n, dtype=np.int64), pairs_per_row)
    j = rng.integers(0, n - 1, size=n * pairs_per_row, dtype=np.int64)
    j = j + (j >= i)                       # j != i
    v = rng.standard_normal(n * pairs_per_row)
    S = sp.coo_matrix((np.concatenate([v, v]), (np.concatenate([i, j]), np.concatenate([j, i]))),
                      shape=(n, n)).tocsr()
    S.sum_duplicates()
    rowabs = np.asarray(abs(S).sum(axis=1)).ravel()
    D = rng.uniform(0.1, 1.0, n)
    Q = (S + sp.diags(rowabs + 1e-3 + D)).tocsr()
    x0 = rng.uniform(0.0, 10.0, n)
    Ax0 = A @ x0
    half = m // 2
    l = np.empty(m); u = np.empty(m)
    l[:half] = Ax0[:half]; u[:half] = Ax0[:half]
    l[half:] = -np.inf; u[half:] = Ax0[half:] + rng.uniform(0.0, 1.0, m - half)
    c = rng.standard_normal(n)
    qr, qc, qv = _csr_arrays(Q)
    ar, ac, av = _csr_arrays(A)
    return QP(n=n, m=m, qkind="csr", c=c, L=np.zeros(n), U=np.full(n, 10.0),
              a_rowptr=ar, a_col=ac, a_val=av, l=l, u=u, q_rowptr=qr, q_col=qc, q_val=qv,
              meta=dict(workload="random_large", seed=seed, x_feasible=x0))


def shuffle_row_entries(qp: QP, seed: int) -> QP:
    """A copy of `qp` whose CSR rows (A, and Q when explicit) list their
    entries in a random order: the same matrices, unsorted column indices."""
    rng = np.random.default_rng(seed)
    out = qp.copy()

    def shuffle(rp, col, val):
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        order = np.lexsort((rng.random(len(col)), rows))
        return np.ascontiguousarray(col[order]), np.ascontiguousarray(val[order])

    out.a_col, out.a_val = shuffle(qp.a_rowptr, qp.a_col, qp.a_val)
    if qp.qkind == "csr":
        out.q_col, out.q_val = shuffle(qp.q_rowptr, qp.q_col, qp.q_val)
    out.meta = dict(qp.meta, shuffled_columns=seed)
    return out


# ---------------------------------------------------------------------------
# Matrix-free Kronecker Q = B (x) C with assignment constraints
# ---------------------------------------------------------------------------
def assignment_A(d: int):
    """Row sums and column sums of a d x d matrix X stored column-major
    (x[i + d*j] = X[i, j]): rows 0..d-1 are sum_j X[i,j], rows d..2d-1 are
    sum_i X[i,j]."""
    n = d * d
    idx = np.arange(n, dtype=np.int64)
    i = idx % d
    j = idx // d
    rows = np.concatenate([i, d + j])
    cols = np.concatenate([idx, idx])
    A = sp.csr_matrix((np.ones(2 * n), (rows, cols)), shape=(2 * d, n))
    return A


def make_kron(seed: int = 1002, d: int = 300) -> QP:
    """B, C = G G^T / d with G ~ N(0,1) d x d (each PSD); Q = B (x) C, n = d^2;
    assignment equalities l = u = 1; box [0,1]; c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((d, d)); Bm = G1 @ G1.T / d
    G2 = rng.standard_normal((d, d)); Cm = G2 @ G2.T / d
    Bm = 0.5 * (Bm + Bm.T); Cm = 0.5 * (Cm + Cm.T)
    n = d * d
    A = assignment_A(d)
    ar, ac, av = _csr_arrays(A)
    c = rng.standard_normal(n)
    return QP(n=n, m=2 * d, qkind="kron", c=c, L=np.zeros(n), U=np.ones(n),
              a_rowptr=ar, a_col=ac, a_val=av, l=np.ones(2 * d), u=np.ones(2 * d),
              kron_B=Bm, kron_C=Cm,
              meta=dict(workload="kron_assignment", seed=seed, d=d,
                        x_feasible=np.full(n, 1.0 / d)))


def qap_st(Ahat: np.ndarray, Bhat: np.ndarray):
    """The matrices S, T of the QAP relaxation of Section 4.5 (problem data).

    Ahat = V_A diag(alpha) V_A^T with alpha descending, Bhat = V_B diag(beta)
    V_B^T with beta ascending; (s, t) is an optimal solution of the LP
    max { sum(s) + sum(t) : s_i + t_j <= alpha_i beta_j for all i, j }, and
    S = V_A diag(s) V_A^T, T = V_B diag(t) V_B^T.  The LP is the dual of the
    assignment problem with costs alpha_i beta_j, whose optimum pairs alpha_i
    with beta_i (rearrangement inequality); one optimal (s, t) is the pair of
    potentials  t_1 = 0,  t_{k+1} = t_k + alpha_k (beta_{k+1} - beta_k),
    s_i = alpha_i beta_i - t_i  (feasible because alpha is descending and
    beta ascending).  The LP has other optimal solutions; this one is fixed
    here.  Returns (S, T, s, t, alpha, beta)."""
    al, VA = np.linalg.eigh(0.5 * (Ahat + Ahat.T))
    be, VB = np.linalg.eigh(0.5 * (Bhat + Bhat.T))
    al, VA = al[::-1], VA[:, ::-1]              # descending
    d = len(al)
    t = np.zeros(d)
    for k in range(d - 1):
        t[k + 1] = t[k] + al[k] * (be[k + 1] - be[k])
    s = al * be - t
    S = (VA * s) @ VA.T
    T = (VB * t) @ VB.T
    return 0.5 * (S + S.T), 0.5 * (T + T.T), s, t, al, be


def make_qap(seed: int = 1007, d: int = 256) -> QP:
    """The synthetic QAP relaxation of Section 4.5: d points uniform in the
    unit square, Ahat their Euclidean distance matrix, Bhat symmetric with
    U[0,1) entries and zero diagonal; the CQP
        min <vec X, Qhat vec X>  s.t.  X e = e, X^T e = e, vec X >= 0,
        Qhat = Bhat (x) Ahat - I (x) S - T (x) I   (S, T from qap_st),
    written as 1/2 <x, Q x> with Q = 2 Qhat (so the objective is the paper's)
    and c = 0.  n = d^2, m = 2d."""
    rng = np.random.default_rng(seed)
    pts = rng.random((d, 2))
    Ah = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    Ub = np.triu(rng.random((d, d)), 1)
    Bh = Ub + Ub.T
    S, T, s, t, al, be = qap_st(Ah, Bh)
    n = d * d
    A = assignment_A(d)
    ar, ac, av = _csr_arrays(A)
    return QP(n=n, m=2 * d, qkind="kron", c=np.zeros(n), L=np.zeros(n), U=np.full(n, np.inf),
              a_rowptr=ar, a_col=ac, a_val=av, l=np.ones(2 * d), u=np.ones(2 * d),
              kron_B=2.0 * Bh, kron_C=Ah, kron_S=2.0 * S, kron_T=2.0 * T,
              meta=dict(workload="qap_relaxation", seed=seed, d=d, Ahat=Ah, Bhat=Bh, s=s, t=t,
                        alpha=al, beta=be))


# ---------------------------------------------------------------------------
# Portfolio-style QP, Q = F F^T + D
# ---------------------------------------------------------------------------
def make_portfolio(seed: int, n: Optional[int] = None, nmin: int = 50, nmax: int = 2000,
                   rank: int = 10, nsectors: int = 20, sector_density: float = 0.05) -> QP:
    """n ~ U{nmin..nmax} (unless given); F n x rank ~ N(0, 0.1) (std);
    D ~ U(0.01, 0.1); A = budget row (all ones, l = u = 1) + `nsectors`
    membership rows (entries 1 with prob 5%, l = -inf, u ~ U(0.2, 0.5));
    box [0, 0.3]; c = -mu with mu ~ N(0.05, 0.02) (std)."""
    rng = np.random.default_rng(seed)
    if n is None:
        n = int(rng.integers(nmin, nmax + 1))
    F = rng.normal(0.0, 0.1, (n, rank))
    D = rng.uniform(0.01, 0.1, n)
    member = rng.random((nsectors, n)) < sector_density
    A = np.vstack([np.ones((1, n)), member.astype(np.float64)])
    m = nsectors + 1
    l = np.empty(m); u = np.empty(m)
    l[0] = 1.0; u[0] = 1.0
    l[1:] = -np.inf; u[1:] = rng.uniform(0.2, 0.5, nsectors)
    mu = rng.normal(0.05, 0.02, n)
    ar, ac, av = _csr_arrays(sp.csr_matrix(A))
    return QP(n=n, m=m, qkind="lowrank", c=-mu, L=np.zeros(n), U=np.full(n, 0.3),
              a_rowptr=ar, a_col=ac, a_val=av, l=l, u=u,
              lr_d=D, lr_F=np.ascontiguousarray(F),
              meta=dict(workload="portfolio", seed=seed, x_feasible=np.full(n, 1.0 / n)))


def make_portfolio_batch(count: int = 4096, seed0: int = 10_000, **kw) -> list:
    """Instance i is ``make_portfolio(seed0 + i)``."""
    return [make_portfolio(seed0 + i, **kw) for i in range(count)]


def make_portfolio_family_base(seed: int = 1004, n: int = 1000) -> QP:
    """The fixed parametric-family instance (n = 1000, m = 21)."""
    return make_portfolio(seed, n=n)


def portfolio_family_sample(base: QP, seed: int) -> tuple:
    """One member of the family: c = c0 + N(0, 0.01), sector upper bounds
    u = u0 * U(0.8, 1.2) (budget row unchanged).  Returns (c, l, u)."""
    rng = np.random.default_rng(seed)
    c = base.c + rng.normal(0.0, 0.01, base.n)
    u = base.u.copy()
    u[1:] = base.u[1:] * rng.uniform(0.8, 1.2, base.m - 1)
    return c, base.l.copy(), u


def family_member(base: QP, seed: int) -> QP:
    c, l, u = portfolio_family_sample(base, seed)
    q = base.copy()
    q.c, q.l, q.u = c, l, u
    q.meta = dict(base.meta, sample_seed=seed)
    return q


# ---------------------------------------------------------------------------
# Tiny random QPs (brute-force checks)
# ---------------------------------------------------------------------------
def make_tiny(seed: int, n: int = 4, m: int = 2, psd_rank: Optional[int] = None,
              n_eq: int = 1, box: float = 2.0, qkind: str = "csr") -> QP:
    """Random tiny QP with a strictly feasible-ish point x0 in the box.
    Q = G G^T (+ 0.1 I unless psd_rank is given, then rank-deficient PSD)."""
    rng = np.random.default_rng(seed)
    if qkind == "zero":
        Q = np.zeros((n, n))
    else:
        r = n if psd_rank is None else psd_rank
        G = rng.standard_normal((n, r))
        Q = G @ G.T + (0.1 * np.eye(n) if psd_rank is None else 0.0)
        Q = 0.5 * (Q + Q.T)
    A = rng.standard_normal((m, n)) if m > 0 else np.zeros((0, n))
    x0 = rng.uniform(-0.5 * box, 0.5 * box, n)
    Ax0 = A @ x0
    l = np.empty(m); u = np.empty(m)
    for i in range(m):
        if i < n_eq:
            l[i] = u[i] = Ax0[i]
        else:
            kind = rng.integers(0, 3)
            lo = Ax0[i] - rng.uniform(0.1, 1.0)
            hi = Ax0[i] + rng.uniform(0.1, 1.0)
            l[i], u[i] = [(lo, hi), (-np.inf, hi), (lo, np.inf)][kind]
    L = np.full(n, -box); U = np.full(n, box)
    # make a couple of bounds infinite to exercise the +-inf paths
    if n >= 3:
        L[n - 1] = -np.inf
    c = rng.standard_normal(n) * 2.0
    return from_dense(Q, c, L, U, A, l, u, qkind=qkind)


def power_start(k: int, seed: int = 0) -> np.ndarray:
    """Seeded N(0,1) start vector for the power method (length k)."""
    return np.random.default_rng(seed).standard_normal(k)

def rescale(qp: QP, seed: int, decades: float = 2.0) -> QP:
    """The same QP after a change of variables x = S x' and a scaling R of the
    rows of A, with S, R diagonal and entries 10^U(-decades, decades): a badly
    scaled instance with the same optimal value (dense; small instances)."""
    rng = np.random.default_rng(seed)
    Q, A = qp.Q_dense(), qp.A_scipy().toarray()
    s = 10.0 ** rng.uniform(-decades, decades, qp.n)
    r = 10.0 ** rng.uniform(-decades, decades, qp.m)
    out = from_dense(s[:, None] * Q * s[None, :], s * qp.c, qp.L / s, qp.U / s,
                     r[:, None] * A * s[None, :], r * qp.l, r * qp.u)
    out.meta = dict(workload=qp.meta.get("workload"), rescaled=seed)
    return out


def make_lasso_rows(seed: int = 1008, p: int = 200_000, q: int = 5_000_000, per_row: int = 1000,
                    lam_frac: float = 0.2) -> QP:
    """The random Lasso of make_lasso at the sizes of the paper's large random
    Lasso table (p = 2e5 .. 6e5 rows, q = 5e6 .. 1e7 columns), built row by
    row so that it fits in memory and time: every row of Ahat holds `per_row`
    columns drawn uniformly (repeats dropped, so slightly fewer) with N(0, 1)
    values; bhat, x_true and lambda as in make_lasso.  The paper does not
    print the density; 1000 per row (2e8 nonzeros at p = 2e5) is what its
    run times on the A100 allow (a denser Ahat would not fit its 80 GB)."""
    rng = np.random.default_rng(seed)
    cols = rng.integers(0, q, size=(p, per_row), dtype=np.int32)
    cols.sort(axis=1)
    keep = np.ones(cols.shape, dtype=bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    rp = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rp[1:])
    ci = cols[keep]
    del cols, keep
    vv = rng.standard_normal(ci.size)
    Ah = sp.csr_matrix((vv, ci, rp.astype(np.int32)), shape=(p, q))
    xt = np.where(rng.random(q) < 0.5, 0.0, rng.standard_normal(q) / np.sqrt(q))
    bh = Ah @ xt + rng.standard_normal(p)
    g = np.asarray(Ah.T @ bh).ravel()
    return QP(n=q, m=0, qkind="gram", c=-g, L=np.full(q, -np.inf), U=np.full(q, np.inf),
              a_rowptr=np.zeros(1, dtype=np.int32), a_col=np.zeros(0, dtype=np.int32),
              a_val=np.zeros(0), l=np.zeros(0), u=np.zeros(0),
              gram_rowptr=rp.astype(np.int32), gram_col=ci, gram_val=vv, gram_p=p,
              l1_weight=lam_frac * np.abs(g).max(),
              meta=dict(workload="lasso", seed=seed, p=p, q=q, per_row=per_row, bhat=bh))


def make_lasso(seed: int = 1005, p: int = 200, q: int = 600, density: float = 0.15,
               lam_frac: float = 0.2) -> QP:
    """Lasso  min 1/2 ||Ahat x - bhat||^2 + lambda ||x||_1  (Section 4.4) as the
    CCQP  1/2 <x, Ahat^T Ahat x> - <Ahat^T bhat, x> + lambda ||x||_1, m = 0,
    no box (the constant 1/2 ||bhat||^2 is dropped).  The random class the
    paper scales up: Ahat p x q with `density` N(0,1) entries, bhat = Ahat
    x_true + noise, x_true with half of its entries zero and the rest
    N(0, 1/q), noise N(0, 1), lambda = lam_frac ||Ahat^T bhat||_inf."""
    rng = np.random.default_rng(seed)
    Ah = sp.random(p, q, density=density, format="csr", random_state=rng,
                   data_rvs=lambda k: rng.standard_normal(k))
    xt = np.where(rng.random(q) < 0.5, 0.0, rng.standard_normal(q) / np.sqrt(q))
    bh = Ah @ xt + rng.standard_normal(p)
    g = np.asarray(Ah.T @ bh).ravel()
    rp, ci, vv = _csr_arrays(Ah)
    qp = QP(n=q, m=0, qkind="gram", c=-g, L=np.full(q, -np.inf), U=np.full(q, np.inf),
            a_rowptr=np.zeros(1, dtype=np.int32), a_col=np.zeros(0, dtype=np.int32),
            a_val=np.zeros(0), l=np.zeros(0), u=np.zeros(0),
            gram_rowptr=rp, gram_col=ci, gram_val=vv, gram_p=p, l1_weight=lam_frac * np.abs(g).max(),
            meta=dict(workload="lasso", seed=seed, p=p, q=q, density=density, bhat=bh))
    return qp
