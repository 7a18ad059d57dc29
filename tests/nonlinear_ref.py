"""A nonlinear tracking model and a CPU reference of the Gauss-Newton /
Levenberg-Marquardt iteration -- TEST INFRASTRUCTURE.

Model (n = 4: position x, y and velocity vx, vy; m = 2):
    evolution    p_i = p_{i-1} + dt v_{i-1},  v_i = v_{i-1} - dt kappa |v_{i-1}| v_{i-1}
    observation  range sqrt(x^2 + y^2) and bearing atan2(y, x)
The reference solves every linear problem with the sequential oracle
(oracle/seq.py) and evaluates the objective with the dense definition
(oracle/dense.py); its iteration logic restates the library driver's
globalization (step halving, or lambda / 10 after an accepted and x 10 after a
rejected Levenberg-Marquardt step) so that both take the same decisions.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

DT, KAPPA = 0.1, 0.05


def f_np(up):
    x, y, vx, vy = up.T
    s = np.sqrt(vx * vx + vy * vy)
    fv = np.stack([x + DT * vx, y + DT * vy, vx - DT * KAPPA * s * vx, vy - DT * KAPPA * s * vy], axis=1)
    k = up.shape[0]
    F = np.zeros((k, 4, 4))
    F[:, 0, 0] = F[:, 1, 1] = 1.0
    F[:, 0, 2] = F[:, 1, 3] = DT
    inv = 1.0 / np.maximum(s, 1e-300)
    F[:, 2, 2] = 1.0 - DT * KAPPA * (s + vx * vx * inv)
    F[:, 2, 3] = -DT * KAPPA * vx * vy * inv
    F[:, 3, 2] = -DT * KAPPA * vx * vy * inv
    F[:, 3, 3] = 1.0 - DT * KAPPA * (s + vy * vy * inv)
    return fv, F


def g_np(u):
    x, y = u[:, 0], u[:, 1]
    r2 = x * x + y * y
    r = np.sqrt(r2)
    gv = np.stack([r, np.arctan2(y, x)], axis=1)
    G = np.zeros((u.shape[0], 2, 4))
    G[:, 0, 0], G[:, 0, 1] = x / r, y / r
    G[:, 1, 0], G[:, 1, 1] = -y / r2, x / r2
    return gv, G


class TorchModel:
    """The same model on device tensors (float64)."""

    def f(self, up):
        import torch
        x, y, vx, vy = up.unbind(1)
        s = torch.sqrt(vx * vx + vy * vy)
        fv = torch.stack([x + DT * vx, y + DT * vy, vx - DT * KAPPA * s * vx, vy - DT * KAPPA * s * vy], 1)
        F = torch.zeros((up.shape[0], 4, 4), dtype=up.dtype, device=up.device)
        F[:, 0, 0] = 1.0
        F[:, 1, 1] = 1.0
        F[:, 0, 2] = DT
        F[:, 1, 3] = DT
        inv = 1.0 / torch.clamp(s, min=1e-300)
        F[:, 2, 2] = 1.0 - DT * KAPPA * (s + vx * vx * inv)
        F[:, 2, 3] = -DT * KAPPA * vx * vy * inv
        F[:, 3, 2] = -DT * KAPPA * vx * vy * inv
        F[:, 3, 3] = 1.0 - DT * KAPPA * (s + vy * vy * inv)
        return fv, F

    def g(self, u):
        import torch
        x, y = u[:, 0], u[:, 1]
        r2 = x * x + y * y
        r = torch.sqrt(r2)
        gv = torch.stack([r, torch.atan2(y, x)], 1)
        G = torch.zeros((u.shape[0], 2, 4), dtype=u.dtype, device=u.device)
        G[:, 0, 0] = x / r
        G[:, 0, 1] = y / r
        G[:, 1, 0] = -y / r2
        G[:, 1, 1] = x / r2
        return gv, G


def make_data(seed: int, k: int, dense_cov: bool, spread: float = 1.0):
    """Seeded trajectory, observations, noise covariances and a perturbed
    initial guess (positions stay at x > 0, away from the bearing's branch cut)."""
    rng = np.random.default_rng(seed)
    n, m = 4, 2
    u = np.zeros((k + 1, n))
    u[0] = [20.0, 0.0, 1.0, 0.6]
    q = np.array([1e-4, 1e-4, 4e-4, 4e-4])
    for i in range(1, k + 1):
        fv, _ = f_np(u[i - 1:i])
        u[i] = fv[0] + np.sqrt(q) * rng.standard_normal(n)
    rvar = np.array([0.04, 1e-4])
    gv, _ = g_np(u)
    o = gv + np.sqrt(rvar) * rng.standard_normal((k + 1, m))
    if dense_cov:
        Kb = np.diag(q) + 2e-5 * np.ones((n, n))
        Cb = np.diag(rvar) + 1e-5 * np.ones((m, m))
        K = np.broadcast_to(Kb, (k, n, n)).copy()
        C = np.broadcast_to(Cb, (k + 1, m, m)).copy()
    else:
        K = np.broadcast_to(q, (k, n)).copy()
        C = np.broadcast_to(rvar, (k + 1, m)).copy()
    c = np.zeros((k, n))
    u0 = u + spread * np.array([0.5, 0.5, 0.1, 0.1]) * rng.standard_normal((k + 1, n))
    return dict(truth=u, u0=u0, c=c, K=K, o=o, C=C, K_diag=not dense_cov, C_diag=not dense_cov, n=n, m=m, k=k)


def _lin(u, d):
    fv, F = f_np(u[:-1])
    gv, G = g_np(u)
    return fv + d["c"] - u[1:], d["o"] - gv, F, G


def _problem(d, F, G, c, o, C, m):
    return SimpleNamespace(k=d["k"], n=d["n"], m=m, H=None, F=F, c=c, K=d["K"], G=G, o=o, C=C,
                           K_diag=d["K_diag"], C_diag=d["C_diag"])


def objective(d, u):
    from oracle import dense
    c, o, F, G = _lin(u, d)
    p = _problem(d, F, G, c, o, d["C"], d["m"])
    return float(dense.objective_terms(p, np.zeros_like(u)).sum())


def reference(d, method="lm", max_iter=50, ftol=1e-12, xtol=1e-10, lam0=1e-3):
    """The iteration of smooth_nonlinear on the CPU (sequential oracle)."""
    from oracle import seq
    k, n, m = d["k"], d["n"], d["m"]
    u = d["u0"].copy()
    J = objective(d, u)
    hist, it, conv, lam = [J], 0, False, lam0
    while it < max_iter and not conv:
        c, o, F, G = _lin(u, d)
        if method == "gn":
            delta = seq.smooth(_problem(d, F, G, c, o, d["C"], m), want_cov=False)["u"]
            alpha, ok = 1.0, False
            while alpha > 1e-12:
                u_try = u + alpha * delta
                J_try = objective(d, u_try)
                if J_try < J:
                    ok = True
                    break
                alpha *= 0.5
            if not ok:
                conv = True
                break
            step = alpha * np.abs(delta).max()
        else:
            Ga = np.concatenate([G, np.broadcast_to(np.eye(n), (k + 1, n, n))], axis=1)
            oa = np.concatenate([o, np.zeros((k + 1, n))], axis=1)
            ok = False
            while lam <= 1e16:
                if d["C_diag"]:
                    Ca = np.concatenate([d["C"], np.full((k + 1, n), 1.0 / lam)], axis=1)
                else:
                    Ca = np.zeros((k + 1, m + n, m + n))
                    Ca[:, :m, :m] = d["C"]
                    Ca[:, m:, m:] = np.eye(n) / lam
                delta = seq.smooth(_problem(d, F, Ga, c, oa, Ca, m + n), want_cov=False)["u"]
                u_try = u + delta
                J_try = objective(d, u_try)
                if J_try < J:
                    ok = True
                    lam = max(lam / 10.0, 1e-12)
                    break
                lam *= 10.0
            if not ok:
                conv = True
                break
            step = np.abs(delta).max()
        dec = J - J_try
        u, J = u_try, J_try
        it += 1
        hist.append(J)
        if dec <= ftol * max(J, 1e-300) or step <= xtol * (1.0 + np.abs(u).max()):
            conv = True
    return dict(u=u, objective=J, iterations=it, converged=conv, history=hist)


def gradient(d, u):
    """Gradient of the nonlinear objective, J'(u) = -2 A(u)^T W r(u), from the
    Jacobians and residuals (the linear problem's rhs is -r)."""
    from oracle import dense
    c, o, F, G = _lin(u, d)
    p = _problem(d, F, G, c, o, d["C"], d["m"])
    A, b, cov_e = dense.assemble(p)
    return (-2.0 * A.T @ np.linalg.solve(cov_e, b)).reshape(u.shape)
