"""Problems with per-step dimensions (Section II-A: u_i in R^{n_i}, H_i
l_i x n_i full rank and possibly rectangular, F_i l_i x n_{i-1}, G_i m_i x n_i
with m_i >= 0) solved by the uniform-dimension kernels through an exact
embedding.

The embedding picks the smallest supported state dimension n >= max(n_i, l_i)
whose observation class holds m = max_i (m_i + n - n_i), and gives state i the
n - n_i padding components z_i:

* evolution i: the l_i rows [H_i 0] [u_i; z_i] - [F_i 0] [u_{i-1}; z_{i-1}] ~ c_i
  with covariance K_i, then n - l_i zero rows of unit variance;
* observation i: the m_i rows G_i u_i ~ o_i with covariance C_i, the n - n_i rows
  z_i ~ 0 of unit variance, then zero rows up to m.

A padding component appears in its own pinning row only, so A^T W A is block
diagonal between padding and real components: the estimate, its covariance
blocks (Section IV) and the lag-one blocks of the real components are exactly
those of the original problem.  Zero rows change no Householder reflector.
Placing the blocks is data movement only; every arithmetic step runs in the
library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import torch

from . import ks

STATE_CLASSES = (1, 2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48)


def embedding_dims(gp) -> tuple:
    """(n, m) of the uniform problem that embeds gp."""
    need = max(max(gp.n), max(gp.l) if gp.l else 0)
    for n in STATE_CLASSES:
        if n < need:
            continue
        m = max(mi + n - ni for mi, ni in zip(gp.m, gp.n))
        if ks.supported(n, m):
            return n, m
    raise ks.KsError(ks.KS_E_ARG, f"no kernel class embeds state dimensions up to {need} "
                                  f"with the observation rows needed")


def embed(gp, n: int, m: int):
    """Uniform arrays (numpy, dense covariances) of the embedded problem.  Steps
    are placed in groups of equal block shapes (one fancy-indexed copy per
    group, not per step)."""
    k = gp.k
    H = np.zeros((k, n, n)); F = np.zeros((k, n, n)); c = np.zeros((k, n))
    K = np.broadcast_to(np.eye(n), (k, n, n)).copy()
    G = np.zeros((k + 1, m, n)); o = np.zeros((k + 1, m))
    C = np.broadcast_to(np.eye(m), (k + 1, m, m)).copy()
    groups = {}
    for t in range(k):
        groups.setdefault((gp.l[t], gp.n[t + 1], gp.n[t]), []).append(t)
    for (li, ni, np_), ts in groups.items():
        ts = np.asarray(ts)
        H[ts, :li, :ni] = np.stack([gp.H[t] for t in ts])
        F[ts, :li, :np_] = np.stack([gp.F[t] for t in ts])
        c[ts, :li] = np.stack([gp.c[t] for t in ts])
        K[ts, :li, :li] = np.stack([gp.K[t] for t in ts])
    groups = {}
    for i in range(k + 1):
        groups.setdefault((gp.m[i], gp.n[i]), []).append(i)
    for (mi, ni), idx in groups.items():
        idx = np.asarray(idx)
        if mi:
            G[idx, :mi, :ni] = np.stack([gp.G[i] for i in idx])
            o[idx, :mi] = np.stack([gp.o[i] for i in idx])
            C[idx, :mi, :mi] = np.stack([gp.C[i] for i in idx])
        pad = np.arange(n - ni)
        G[idx[:, None], mi + pad[None, :], ni + pad[None, :]] = 1.0
    return H, F, c, K, G, o, C


@dataclass
class GeneralResult:
    n: List[int]
    u_pad: torch.Tensor       # [k+1, n_embed]
    cov_pad: torch.Tensor     # [k+1, n_embed, n_embed]
    lag1_pad: torch.Tensor    # [k, n_embed, n_embed]

    def u(self, i: int) -> torch.Tensor:
        return self.u_pad[i, :self.n[i]]

    def cov(self, i: int) -> torch.Tensor:
        return self.cov_pad[i, :self.n[i], :self.n[i]]

    def lag1(self, i: int) -> torch.Tensor:
        """cov(u_hat_i, u_hat_{i+1}), n_i x n_{i+1}."""
        return self.lag1_pad[i, :self.n[i], :self.n[i + 1]]


def smooth_general(gp, device=None, fp32: bool = False) -> GeneralResult:
    """States, covariance blocks and lag-one blocks of a per-step-dimension
    problem (gen.GeneralProblem layout)."""
    n, m = embedding_dims(gp)
    arrays = embed(gp, n, m)
    dev = ks._device(device)
    H, F, c, K, G, o, C = (torch.from_numpy(a).to(dev) for a in arrays)
    plan = ks.Plan(gp.k, n, m, False, False, device=dev, fp32=fp32)
    try:
        u, cov, lag1 = plan.smooth_cov_lag1(H, F, c, K, G, o, C)
    finally:
        plan.close()
    return GeneralResult(n=list(gp.n), u_pad=u, cov_pad=cov, lag1_pad=lag1)
