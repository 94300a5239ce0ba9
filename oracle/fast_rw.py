"""Precomputed-eigenvector ("fast") random walker (oracle; test infrastructure only).

Sec. II-B.  With E = Q (Lambda + gamma I)^{-1} Q^T (eq. (7)) split into blocks
[E_s, R; R^T, E_n] (eqs. (8)-(9)) and the auxiliary unknown F = (L + gamma I) U (eqs. (10)-(13)),
left-multiplying by E gives U_n = R^T F_s + gamma E_n P_n (eq. (15)), and eliminating U_n from
eq. (11) gives the S x S seed system  (I - B R^T) F_s = L_s U_s + gamma (U_s + B E_n P_n)  (eq. (17)).

gamma = 0 (the paragraph after eq. (17)): L has the null vector g, so E L = I - g g^T and eq. (14)
must be altered; the paper points to first computing g_n^T U_n (the column sums of U_n) and using
them to obtain F_s, without giving the equations.  Reading used here (derived from the same
equations): write U = E F + g c^T with c^T = g^T U, where E = Q' Lambda'^{-1} Q'^T is built from the
eigenpairs other than the null pair.  Then, with F_n = 0 (eq. (13) with gamma = 0):

    U_n = R^T F_s + g_n c^T,                 R^T = Q'_n Lambda'^{-1} Q'_s^T
    (I - B R^T) F_s - B g_n c^T = L_s U_s    (eq. (11) with U_n substituted)
    g_s^T F_s = 0                            (g^T F = g^T L U = 0 and F_n = 0)

an (S+1) x (S+1) bordered system in (F_s, c).  It is exact when Q holds all N eigenvectors, and the
rows of U sum to 1 for any truncation.

Normalized Laplacian (Sec. II-C): every quantity is taken in hat variables, L -> L_hat,
U_s -> D_s^{1/2} U_s, g -> D^{1/2} 1 / ||D^{1/2} 1||, and U = D^{-1/2} U_hat at the end.
A node with d = 0 (no edges at all) gets U = 0.

Exact mode.  R^T carries Lambda'^{-1}, so when the graph has weakly coupled regions (eigenvalues
1e-9 .. 1e-17 above zero) the bordered system has entries of size 1/lambda and its FP64 solution
loses up to all of its digits.  With exact=True the seed-side steps (B Q'_n, B R^T, the bordered
solve and Y = Lambda'^{-1} Q'_s^T F_s) are carried out on the given FP64 inputs in 100-digit decimal
arithmetic (each FP64 input converts exactly; a condition number up to 1e20 still leaves about 80
correct digits, far below FP64's resolution), Y and c are rounded once to FP64, and only the final
reconstruction Q'_n Y + g_n c^T runs in FP64.  exact="rational" carries out the same steps in exact
rational arithmetic (Python fractions): no rounding at all, but its cost grows steeply with S; it
pins the decimal evaluation.  Both evaluate the same equations, in the same order, without FP64
rounding in the ill-conditioned part; the bordered solve is Gaussian elimination with partial
pivoting (largest magnitude), which in exact arithmetic gives the exact solution whatever pivots it
takes.
"""
from __future__ import annotations

import decimal
from decimal import Decimal
from fractions import Fraction

import numpy as np

from .eigen import insert_null
from .exact_rw import one_hot, seed_split


def _seed_blocks(graph, seed_node):
    M = graph.M().tocsr()
    N = graph.N
    s, n = seed_split(N, seed_node)
    Ms_rows = M[s]                       # S x N
    Ms = Ms_rows[:, s]                   # L_s  (seed-seed block)
    B_full = Ms_rows.tolil(copy=True)    # B with the seed columns zeroed, kept N wide
    B_full[:, s] = 0.0
    B_full = B_full.tocsr()
    return M, s, n, Ms, B_full


def _exact_solve(A, b):
    """Gaussian elimination with partial pivoting (largest magnitude) in the entries' own arithmetic
    (rationals or 100-digit decimals); A n x n, b n x k."""
    n = len(A)
    A = [row[:] for row in A]
    b = [row[:] for row in b]
    for k in range(n):
        p = max(range(k, n), key=lambda i: abs(A[i][k]))
        if A[p][k] == 0:
            raise np.linalg.LinAlgError("singular bordered system")
        A[k], A[p] = A[p], A[k]
        b[k], b[p] = b[p], b[k]
        inv = 1 / A[k][k]
        for i in range(k + 1, n):
            f = A[i][k] * inv
            if f == 0:
                continue
            Ai, Ak = A[i], A[k]
            for j in range(k + 1, n):
                if Ak[j] != 0:
                    Ai[j] -= f * Ak[j]
            bi, bk = b[i], b[k]
            for j in range(len(bi)):
                bi[j] -= f * bk[j]
            Ai[k] = A[k][k] * 0
    x = [[b[0][0] * 0] * len(b[0]) for _ in range(n)]
    for k in range(n - 1, -1, -1):
        for j in range(len(b[0])):
            acc = b[k][j]
            for i in range(k + 1, n):
                if A[k][i] != 0:
                    acc -= A[k][i] * x[i][j]
            x[k][j] = acc / A[k][k]
    return x


def _coeffs_exact(graph, Qp, lp, ghat, s, Ms, B, Uhat_s, C, number=Fraction):
    F = number
    S, mp = s.size, Qp.shape[1]
    Bc = B.tocsr()
    Qs = [[F(float(v)) for v in row] for row in Qp[s]]
    inv_l = [1 / F(float(v)) for v in lp]
    BQn = []                                          # B Q'_n, exactly
    Bg = []                                           # B g_n, exactly
    for i in range(S):
        lo, hi = Bc.indptr[i], Bc.indptr[i + 1]
        cols, vals = Bc.indices[lo:hi], Bc.data[lo:hi]
        row = [F(0)] * mp
        gsum = F(0)
        for t, bv in zip(cols, vals):
            fb = F(float(bv))
            gsum += fb * F(float(ghat[t]))
            qt = Qp[t]
            for j in range(mp):
                row[j] += fb * F(float(qt[j]))
        BQn.append(row)
        Bg.append(gsum)
    A = [[BQn[i][j] * inv_l[j] for j in range(mp)] for i in range(S)]      # B Q'_n Lambda'^{-1}
    K = [[(F(1) if i == k else F(0)) - sum(A[i][j] * Qs[k][j] for j in range(mp)) for k in range(S)]
         + [-Bg[i]] for i in range(S)]
    K.append([F(float(ghat[v])) for v in s] + [F(0)])
    Msc = Ms.tocsr()
    rhs = []
    for i in range(S):
        lo, hi = Msc.indptr[i], Msc.indptr[i + 1]
        acc = [F(0)] * C
        for t, mv in zip(Msc.indices[lo:hi], Msc.data[lo:hi]):
            for c in range(C):
                if Uhat_s[t, c] != 0:
                    acc[c] += F(float(mv)) * F(float(Uhat_s[t, c]))
        rhs.append(acc)
    rhs.append([F(0)] * C)
    sol = _exact_solve(K, rhs)
    Fs, c = sol[:S], sol[S]
    Y = np.array([[float(inv_l[j] * sum(Qs[k][j] * Fs[k][cc] for k in range(S))) for cc in range(C)]
                  for j in range(mp)])
    return Y, np.array([float(v) for v in c])


def fast_rw_coeffs(graph, Q, lam, seed_node, seed_label, C, m=None, exact=False):
    """Solve the gamma = 0 bordered system.  Returns (Qp, Y, c) such that the hat-variable
    probabilities at a non-seed node i are  Qp[i] @ Y + ghat[i] * c."""
    m = Q.shape[1] if m is None else m
    ghat = graph.ghat()
    Qm, lm = insert_null(np.asarray(Q, dtype=np.float64)[:, :m], np.asarray(lam, dtype=np.float64)[:m], ghat)
    Qp, lp = Qm[:, 1:], lm[1:]                       # Q', Lambda' (null pair removed)
    M, s, n, Ms, B = _seed_blocks(graph, seed_node)
    S = s.size
    Uhat_s = graph.hat_scale()[s][:, None] * one_hot(seed_label, C)
    if exact == "rational":
        Y, c = _coeffs_exact(graph, Qp, lp, ghat, s, Ms, B, Uhat_s, C, Fraction)
        return Qp, Y, c
    if exact:
        with decimal.localcontext() as ctx:
            ctx.prec = 100
            ctx.Emin, ctx.Emax = -999999, 999999
            Y, c = _coeffs_exact(graph, Qp, lp, ghat, s, Ms, B, Uhat_s, C, Decimal)
        return Qp, Y, c
    Qs = Qp[s]                                       # Q'_s
    BQn = B @ Qp                                     # B Q'_n      (S x m')
    BRt = BQn @ (Qs / lp[None, :]).T                 # B R^T = B Q'_n Lambda'^{-1} Q'_s^T   (S x S)
    Bg = B @ ghat                                    # B g_n
    K = np.zeros((S + 1, S + 1))
    K[:S, :S] = np.eye(S) - BRt
    K[:S, S] = -Bg
    K[S, :S] = ghat[s]
    rhs = np.zeros((S + 1, C))
    rhs[:S] = Ms @ Uhat_s
    sol = np.linalg.solve(K, rhs)                   # LU with partial pivoting (LAPACK gesv)
    Fs, c = sol[:S], sol[S]
    Y = (Qs.T @ Fs) / lp[:, None]                    # Lambda'^{-1} Q'_s^T F_s
    return Qp, Y, c


def fast_rw(graph, Q, lam, seed_node, seed_label, C, m=None, rows=None, exact=False):
    """Label probabilities U (N x C, or len(rows) x C) of the gamma = 0 fast random walker."""
    Qp, Y, c = fast_rw_coeffs(graph, Q, lam, seed_node, seed_label, C, m, exact=exact)
    ghat = graph.ghat()
    hs = graph.hat_scale()
    N = graph.N
    rows = np.arange(N) if rows is None else np.asarray(rows, dtype=np.int64)
    Uhat = Qp[rows] @ Y + np.outer(ghat[rows], c)
    with np.errstate(divide="ignore", invalid="ignore"):
        U = np.where(hs[rows, None] > 0, Uhat / hs[rows, None], 0.0)
    # seed rows are fixed (eq. (1)): one-hot
    seed_node = np.asarray(seed_node)
    lab = np.asarray(seed_label)
    pos = {int(v): k for k, v in enumerate(seed_node)}
    for r, i in enumerate(rows):
        k = pos.get(int(i))
        if k is not None:
            U[r] = 0.0
            U[r, lab[k]] = 1.0
    return U


def fast_rw_prior(graph, Q, lam, seed_node, seed_label, C, gamma, prior, m=None):
    """gamma > 0 fast random walker, eqs. (15) and (17) as printed, in the variables of the
    operator graph.M() (with the normalized Laplacian this applies the prior in hat variables,
    P_hat = D^{1/2} P, as the substitution of Sec. II-C prescribes).  The stored basis is read as in the
    gamma = 0 case: the analytic null vector g (the zero-eigenvalue eigenvector of Sec. II-B) takes the
    place of the stored column closest to it, with eigenvalue 0, and the other columns are made
    orthogonal to it (insert_null); E = Q (Lambda + gamma I)^{-1} Q^T then includes the null pair."""
    m = Q.shape[1] if m is None else m
    Q, lam = insert_null(np.asarray(Q, dtype=np.float64)[:, :m], np.asarray(lam, dtype=np.float64)[:m],
                         graph.ghat())
    M, s, n, Ms, B = _seed_blocks(graph, seed_node)
    hs = graph.hat_scale()
    Uhat_s = hs[s][:, None] * one_hot(seed_label, C)
    Phat = hs[:, None] * np.asarray(prior, dtype=np.float64)
    Phat_n = Phat.copy()
    Phat_n[s] = 0.0                                   # P_n, embedded N wide
    inv = 1.0 / (lam + gamma)
    Qs = Q[s]
    # E_n P_n = Q_n (Lambda + gamma)^{-1} Q_n^T P_n
    QnTPn = Q.T @ Phat_n
    EnPn = Q @ (inv[:, None] * QnTPn)                 # evaluated on all rows; only rows n are used
    EnPn[s] = 0.0
    BRt = (B @ Q) @ (Qs * inv[None, :]).T             # B R^T,  R^T = Q_n (Lambda+gamma)^{-1} Q_s^T
    S = s.size
    lhs = np.eye(S) - BRt
    rhs = Ms @ Uhat_s + gamma * (Uhat_s + B @ EnPn)
    Fs = np.linalg.solve(lhs, rhs)
    Uhat = Q @ (inv[:, None] * (Qs.T @ Fs)) + gamma * EnPn   # eq. (15) on the non-seed rows
    with np.errstate(divide="ignore", invalid="ignore"):
        U = np.where(hs[:, None] > 0, Uhat / hs[:, None], 0.0)
    U[s] = one_hot(seed_label, C)
    return U
