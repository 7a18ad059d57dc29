"""Textbook Kalman filter + Rauch-Tung-Striebel smoother (test pin only).

Written independently of the oracle: covariance-form predict/update with the
Joseph-form covariance update, then the RTS backward pass.  With a proper prior
N(mu_0, P_0) on u_0 and H_i = I, its smoothed means and covariances equal the
generalized least-squares estimate of Section II-A in which the prior enters as
an observation of u_0 with G_0 = I, o_0 = mu_0 and covariance P_0 (Section II-B
notes that these recursions need the prior).
"""
import numpy as np


def _cov(x, diag):
    return np.diag(x) if diag else x


def kf_rts(p):
    k, n = p.k, p.n
    assert p.H is None, "H = I only"
    assert p.m == n and np.allclose(p.G[0], np.eye(n)), "prior enters as G_0 = I"
    xf = np.zeros((k + 1, n))
    Pf = np.zeros((k + 1, n, n))
    xp = np.zeros((k + 1, n))
    Pp = np.zeros((k + 1, n, n))
    xf[0] = p.o[0]
    Pf[0] = _cov(p.C[0], p.C_diag)
    I = np.eye(n)
    for i in range(1, k + 1):
        F = p.F[i - 1]
        xp[i] = F @ xf[i - 1] + p.c[i - 1]
        Pp[i] = F @ Pf[i - 1] @ F.T + _cov(p.K[i - 1], p.K_diag)
        G = p.G[i]
        R = _cov(p.C[i], p.C_diag)
        S = G @ Pp[i] @ G.T + R
        Kg = np.linalg.solve(S, G @ Pp[i]).T
        xf[i] = xp[i] + Kg @ (p.o[i] - G @ xp[i])
        IKG = I - Kg @ G
        Pf[i] = IKG @ Pp[i] @ IKG.T + Kg @ R @ Kg.T
    xs = xf.copy()
    Ps = Pf.copy()
    for i in range(k - 1, -1, -1):
        Cg = np.linalg.solve(Pp[i + 1], p.F[i] @ Pf[i]).T
        xs[i] = xf[i] + Cg @ (xs[i + 1] - xp[i + 1])
        Ps[i] = Pf[i] + Cg @ (Ps[i + 1] - Pp[i + 1]) @ Cg.T
    return xs, Ps
