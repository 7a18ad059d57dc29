"""Nonlinear smoothing by Gauss-Newton or Levenberg-Marquardt iterations, each
a linear smoothing problem solved by the odd-even smoother without covariances
(Section II-B; the NC mode of Section V-D).

The model is H_i u_i = f_i(u_{i-1}) + c_i + eps_i for i = 1..k (cov(eps_i) =
K_i) and o_i = g_i(u_i) + delta_i for i = 0..k (cov(delta_i) = C_i).  At the
iterate u~ the correction d solves the linear problem with F_i = df_i/du(u~_{i-1}),
G_i = dg_i/du(u~_i) and the residuals as right-hand sides:

    H_i d_i - F_i d_{i-1} ~ f_i(u~_{i-1}) + c_i - H_i u~_i   (K_i)
    G_i d_i               ~ o_i - g_i(u~_i)                  (C_i)

The model's functions and Jacobians are evaluated for all steps at once, on
the device, by the caller's ``model`` object; the library solves every linear
problem (ks_smooth) and evaluates every objective value (ks_objective) in its
own kernels.  The plan stays resident across iterations; only its inputs
change.

Globalization:
* ``method="gn"``: Gauss-Newton with step halving until the objective
  decreases;
* ``method="lm"``: Levenberg-Marquardt, the Jacobian of every step stacked
  with sqrt(lambda) I (observation rows d_i ~ 0 of variance 1/lambda, so the
  linear problems have m + n observation rows), lambda divided by 10 after an
  accepted step and multiplied by 10 after a rejected one.

    model.f(u_prev [k, n]) -> (f [k, n], F [k, n, n])
    model.g(u [k+1, n])    -> (g [k+1, m], G [k+1, m, n])
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import torch

from . import ks


@dataclass
class NonlinearResult:
    u: torch.Tensor                      # [k+1, n] final iterate
    objective: float                     # ||U(A(u) - b)||^2 at u
    iterations: int                      # accepted steps
    converged: bool
    history: List[float] = field(default_factory=list)   # objective after each accepted step
    cov: Optional[torch.Tensor] = None   # covariance blocks of the last linearization


class _Linearization:
    """Residuals and Jacobians of the model at one iterate."""

    def __init__(self, model, u, H, c, o):
        fv, self.F = model.f(u[:-1])
        gv, self.G = model.g(u)
        Hu = u[1:] if H is None else torch.bmm(H, u[1:, :, None])[..., 0]
        self.c = (fv + c - Hu).contiguous()     # evolution right-hand side of the correction
        self.o = (o - gv).contiguous()          # observation right-hand side
        self.F = self.F.contiguous()
        self.G = self.G.contiguous()


def smooth_nonlinear(model, u0: torch.Tensor, H, c, K, o, C, K_diag: bool, C_diag: bool, *,
                     method: str = "lm", max_iter: int = 50, ftol: float = 1e-12, xtol: float = 1e-10,
                     lam0: float = 1e-3, want_cov: bool = False) -> NonlinearResult:
    if method not in ("gn", "lm"):
        raise ValueError(f"method must be 'gn' or 'lm', got {method!r}")
    k, n = u0.shape[0] - 1, u0.shape[1]
    m = o.shape[1]
    dev = u0.device
    plan = ks.Plan(k, n, m, K_diag, C_diag, device=dev)
    lm_plan = None
    if method == "lm":
        if not ks.supported(n, m + n):
            plan.close()
            raise ks.KsError(ks.KS_E_ARG, f"Levenberg-Marquardt needs m + n = {m + n} observation rows "
                                          f"for n = {n}; use method='gn'")
        lm_plan = ks.Plan(k, n, m + n, K_diag, C_diag, device=dev)
        G_aug = torch.zeros((k + 1, m + n, n), dtype=torch.float64, device=dev)
        G_aug[:, m:, :] = torch.eye(n, dtype=torch.float64, device=dev)
        o_aug = torch.zeros((k + 1, m + n), dtype=torch.float64, device=dev)
        if C_diag:
            C_aug = torch.empty((k + 1, m + n), dtype=torch.float64, device=dev)
            C_aug[:, :m] = C
        else:
            C_aug = torch.zeros((k + 1, m + n, m + n), dtype=torch.float64, device=dev)
            C_aug[:, :m, :m] = C
    try:
        u = u0.clone().contiguous()
        lin = _Linearization(model, u, H, c, o)
        J = plan.objective(None, None, lin.c, K, None, lin.o, C)
        history, it, converged, lam = [J], 0, False, lam0
        d = torch.empty_like(u)
        while it < max_iter and not converged:
            if method == "gn":
                plan.smooth(H, lin.F, lin.c, K, lin.G, lin.o, C, u_out=d)
                alpha, accepted = 1.0, False
                while alpha > 1e-12:
                    u_try = (u + alpha * d).contiguous()
                    lin_try = _Linearization(model, u_try, H, c, o)
                    J_try = plan.objective(None, None, lin_try.c, K, None, lin_try.o, C)
                    if J_try < J:
                        accepted = True
                        break
                    alpha *= 0.5
                if not accepted:
                    converged = True   # no decrease along the Gauss-Newton direction: stationary
                    break
                step = alpha * float(d.abs().max())
            else:
                G_aug[:, :m, :] = lin.G
                o_aug[:, :m] = lin.o
                accepted = False
                while lam <= 1e16:
                    if C_diag:
                        C_aug[:, m:] = 1.0 / lam
                    else:
                        C_aug[:, m:, m:] = torch.eye(n, dtype=torch.float64, device=dev) / lam
                    lm_plan.smooth(H, lin.F, lin.c, K, G_aug, o_aug, C_aug, u_out=d)
                    u_try = (u + d).contiguous()
                    lin_try = _Linearization(model, u_try, H, c, o)
                    J_try = plan.objective(None, None, lin_try.c, K, None, lin_try.o, C)
                    if J_try < J:
                        accepted = True
                        lam = max(lam / 10.0, 1e-12)
                        break
                    lam *= 10.0
                if not accepted:
                    converged = True
                    break
                step = float(d.abs().max())
            decrease = J - J_try
            u, lin, J = u_try, lin_try, J_try
            it += 1
            history.append(J)
            if decrease <= ftol * max(J, 1e-300) or step <= xtol * (1.0 + float(u.abs().max())):
                converged = True
        cov = None
        if want_cov:
            _, cov = plan.smooth_cov(H, lin.F, lin.c, K, lin.G, lin.o, C)
        return NonlinearResult(u=u, objective=J, iterations=it, converged=converged, history=history, cov=cov)
    finally:
        plan.close()
        if lm_plan is not None:
            lm_plan.close()
