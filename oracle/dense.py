"""The smoothing problem's definition written out densely (tiny k only).

TEST INFRASTRUCTURE: see the package docstring.

Section II-A stacks the evolution and observation equations into one linear
least-squares problem.  With A the block matrix whose block rows are, in order,

    G_0 u_0                     (observation 0)
    H_1 u_1 - F_1 u_0           (evolution 1)
    G_1 u_1                     (observation 1)
    ...
    H_k u_k - F_k u_{k-1}       (evolution k)
    G_k u_k                     (observation k)

b = (o_0, c_1, o_1, ..., c_k, o_k) and cov(e) block diagonal with blocks
(C_0, K_1, C_1, ..., K_k, C_k) (eq. structure-of-cov-e; the paper calls C_i L_i),
the estimate is the generalized least-squares minimizer
(eq. nonlinear-generalized-least-squares with linear A)

    u_hat = argmin_u (A u - b)^T W (A u - b),   W = cov(e)^{-1},

i.e. u_hat = (A^T W A)^{-1} A^T W b, and its covariance is
cov(u_hat) = (A^T W A)^{-1} = (R^T R)^{-1} for any thin QR of U A (Section IV).
Nothing here factors W: the normal-equation form needs no choice of U.
"""
from __future__ import annotations

import numpy as np


def _block(cov, diag):
    return np.diag(cov) if diag else np.asarray(cov)


def assemble(p):
    """Dense (A, b, cov_e) of problem p, rows ordered as in Section II-A."""
    k, n, m = p.k, p.n, p.m
    N = (k + 1) * n
    rows, rhs, covs = [], [], []
    eye = np.eye(n)
    for i in range(k + 1):
        if i >= 1:
            blk = np.zeros((n, N))
            blk[:, (i - 1) * n:i * n] = -p.F[i - 1]
            blk[:, i * n:(i + 1) * n] = eye if p.H is None else p.H[i - 1]
            rows.append(blk)
            rhs.append(p.c[i - 1])
            covs.append(_block(p.K[i - 1], p.K_diag))
        if m:
            blk = np.zeros((m, N))
            blk[:, i * n:(i + 1) * n] = p.G[i]
            rows.append(blk)
            rhs.append(p.o[i])
            covs.append(_block(p.C[i], p.C_diag))
    A = np.vstack(rows)
    b = np.concatenate(rhs)
    tot = A.shape[0]
    cov_e = np.zeros((tot, tot))
    at = 0
    for cblk in covs:
        d = cblk.shape[0]
        cov_e[at:at + d, at:at + d] = cblk
        at += d
    return A, b, cov_e


def normal_matrix(p):
    """(J, h) = (A^T W A, A^T W b) with W = cov(e)^{-1}."""
    A, b, cov_e = assemble(p)
    WA = np.linalg.solve(cov_e, A)
    Wb = np.linalg.solve(cov_e, b)
    return A.T @ WA, A.T @ Wb


def smooth(p):
    """u_hat [k+1][n], Sigma [k+1][n][n], full S = (A^T W A)^{-1} and the
    weighted residual (A u_hat - b)^T W (A u_hat - b)."""
    J, h = normal_matrix(p)
    S = np.linalg.inv(J)
    u = np.linalg.solve(J, h)
    k, n = p.k, p.n
    sig = np.stack([S[i * n:(i + 1) * n, i * n:(i + 1) * n] for i in range(k + 1)])
    A, b, cov_e = assemble(p)
    r = A @ u - b
    resid2 = float(r @ np.linalg.solve(cov_e, r))
    return dict(u=u.reshape(k + 1, n), cov=sig, S=S, resid2=resid2)


def objective_terms(p, u):
    """Per-step terms of the objective (A u - b)^T W (A u - b) of Section II-A
    at u [k+1][n]: for step i, r_i^T K_i^{-1} r_i with the evolution residual
    r_i = H_i u_i - F_i u_{i-1} - c_i (i >= 1), plus s_i^T C_i^{-1} s_i with the
    observation residual s_i = G_i u_i - o_i.  W is block diagonal, so the
    objective is the sum of these terms.  Vectorized over steps (any k)."""
    k, n, m = p.k, p.n, p.m
    u = np.asarray(u, dtype=np.float64).reshape(k + 1, n)
    terms = np.zeros(k + 1)
    if k > 0:
        Hu = u[1:] if p.H is None else np.einsum("tij,tj->ti", p.H, u[1:])
        r = Hu - np.einsum("tij,tj->ti", p.F, u[:-1]) - p.c
        if p.K_diag:
            terms[1:] += np.sum(r * r / p.K, axis=1)
        else:
            terms[1:] += np.einsum("ti,ti->t", r, np.linalg.solve(p.K, r[..., None])[..., 0])
    if m:
        s = np.einsum("tij,tj->ti", p.G, u) - p.o
        if p.C_diag:
            terms += np.sum(s * s / p.C, axis=1)
        else:
            terms += np.einsum("ti,ti->t", s, np.linalg.solve(p.C, s[..., None])[..., 0])
    return terms


def whitened(p):
    """(U A, U b) with U = L^{-1} for the Cholesky factor cov(e) = L L^T.

    Any U with U^T U = cov(e)^{-1} gives the same estimate; this one is used for
    dense QR factors of U A (and of U A P for a block-column permutation P).
    """
    A, b, cov_e = assemble(p)
    L = np.linalg.cholesky(cov_e)
    UA = np.linalg.solve(L, A)
    Ub = np.linalg.solve(L, b)
    return UA, Ub


def smooth_lstsq(p):
    """u_hat by a QR-based least-squares solve of min ||U A u - U b||."""
    UA, Ub = whitened(p)
    u, *_ = np.linalg.lstsq(UA, Ub, rcond=None)
    return u.reshape(p.k + 1, p.n)


def permuted_R(p, order):
    """R of a thin QR of U A P, where P lists the block columns in ``order``
    (a permutation of 0..k).  Returns (R, Qt_Ub) with R of size (k+1)n."""
    n = p.n
    UA, Ub = whitened(p)
    cols = np.concatenate([np.arange(i * n, (i + 1) * n) for i in order])
    q, r = np.linalg.qr(UA[:, cols])
    return r, q.T @ Ub


def assemble_general(gp):
    """Dense (A, b, cov_e) of a problem with per-step dimensions (Section II-A:
    u_i in R^{n_i}, H_i l_i x n_i, F_i l_i x n_{i-1}, G_i m_i x n_i), block rows
    in the order observation 0, evolution 1, observation 1, ..., and block
    column i at offset n_0 + ... + n_{i-1}."""
    k = gp.k
    off = np.concatenate([[0], np.cumsum(gp.n)])
    N = int(off[-1])
    rows, rhs, covs = [], [], []
    for i in range(k + 1):
        if i >= 1:
            blk = np.zeros((gp.l[i - 1], N))
            blk[:, off[i - 1]:off[i]] = -gp.F[i - 1]
            blk[:, off[i]:off[i + 1]] = gp.H[i - 1]
            rows.append(blk)
            rhs.append(gp.c[i - 1])
            covs.append(gp.K[i - 1])
        if gp.m[i]:
            blk = np.zeros((gp.m[i], N))
            blk[:, off[i]:off[i + 1]] = gp.G[i]
            rows.append(blk)
            rhs.append(gp.o[i])
            covs.append(gp.C[i])
    A = np.vstack(rows)
    b = np.concatenate(rhs)
    cov_e = np.zeros((A.shape[0], A.shape[0]))
    at = 0
    for cblk in covs:
        d = cblk.shape[0]
        cov_e[at:at + d, at:at + d] = cblk
        at += d
    return A, b, cov_e, off


def smooth_general(gp):
    """u_hat_i, Sigma_i = cov(u_hat_i) and the lag-one blocks cov(u_hat_i,
    u_hat_{i+1}) of a per-step-dimension problem: (A^T W A)^{-1} A^T W b and
    (A^T W A)^{-1} written out densely (tiny k only)."""
    A, b, cov_e, off = assemble_general(gp)
    J = A.T @ np.linalg.solve(cov_e, A)
    h = A.T @ np.linalg.solve(cov_e, b)
    S = np.linalg.inv(J)
    u = np.linalg.solve(J, h)
    k = gp.k
    us = [u[off[i]:off[i + 1]] for i in range(k + 1)]
    cov = [S[off[i]:off[i + 1], off[i]:off[i + 1]] for i in range(k + 1)]
    lag1 = [S[off[i]:off[i + 1], off[i + 1]:off[i + 2]] for i in range(k)]
    return dict(u=us, cov=cov, lag1=lag1, J=J)
