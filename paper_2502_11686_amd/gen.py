"""Seeded synthetic inputs for linear Kalman smoothing problems.

This module draws model matrices, noise covariances and a simulated trajectory,
and packs them in the step-major layout that both the library and the CPU oracle
accept.  It holds none of the smoother's arithmetic (no whitening, no QR, no
solves): it only samples a linear dynamic system of the form of Section II-A
(evolution equation H_i u_i = F_i u_{i-1} + c_i + eps_i for i = 1..k,
observation equation o_i = G_i u_i + delta_i for i = 0..k) with
cov(eps_i) = K_i and cov(delta_i) = C_i (the paper calls the latter L_i).

Array layout (all float64, C-contiguous, step-major):

    H, F : [k][n][n]      entry t belongs to evolution step i = t + 1
    c    : [k][n]
    K    : [k][n][n] (dense) or [k][n] (diagonal variances)
    G    : [k+1][m][n]
    o    : [k+1][m]
    C    : [k+1][m][m] (dense) or [k+1][m] (diagonal variances)

H is None when every H_i is the identity.

The workload recipes follow the paper's benchmark problems (Section V-B:
orthonormal-ish F, H = I, synthetic observations) widened to the shapes of the
five workloads this library is measured on (see ``workload``).  Every draw comes
from a numpy Generator seeded with SeedSequence(1000 + workload_id); batched and
served problems draw from ``.spawn()``-ed children in order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    k: int
    n: int
    m: int
    F: np.ndarray
    c: np.ndarray
    K: np.ndarray
    G: np.ndarray
    o: np.ndarray
    C: np.ndarray
    K_diag: bool
    C_diag: bool
    H: Optional[np.ndarray] = None
    u_true: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def steps(self) -> int:
        """Number of smoothed states, k + 1."""
        return self.k + 1

    def arrays(self):
        """The seven inputs in ABI order (H may be None)."""
        return self.H, self.F, self.c, self.K, self.G, self.o, self.C


# --------------------------------------------------------------------------
# elementary samplers
# --------------------------------------------------------------------------

def haar_orthogonal(rng: np.random.Generator, count: int, n: int) -> np.ndarray:
    """count independent Haar-distributed n x n orthogonal matrices.

    QR of a Gaussian matrix with the signs of diag(R) folded into Q
    (Mezzadri, Notices AMS 2007).
    """
    z = rng.standard_normal((count, n, n))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diagonal(r, axis1=1, axis2=2))
    d[d == 0] = 1.0
    return q * d[:, None, :]


def loguniform(rng: np.random.Generator, lo: float, hi: float, size) -> np.ndarray:
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def spd_dense(rng: np.random.Generator, count: int, d: int) -> np.ndarray:
    """count SPD matrices L L^T + 0.1 I with L having N(0, 1) entries."""
    L = rng.standard_normal((count, d, d))
    return L @ np.swapaxes(L, 1, 2) + 0.1 * np.eye(d)[None]


def contracting_F(rng: np.random.Generator, count: int, n: int) -> np.ndarray:
    """F = Q diag(U[0.95, 1]) Q^T with Q Haar; count independent draws."""
    q = haar_orthogonal(rng, count, n)
    lam = rng.uniform(0.95, 1.0, size=(count, n))
    return (q * lam[:, None, :]) @ np.swapaxes(q, 1, 2)


def _noise(rng: np.random.Generator, cov: np.ndarray, diag: bool, shape) -> np.ndarray:
    z = rng.standard_normal(shape)
    if diag:
        return np.sqrt(cov) * z
    chol = np.linalg.cholesky(cov)
    return np.einsum("tij,tj->ti", chol, z)


# --------------------------------------------------------------------------
# problem builder
# --------------------------------------------------------------------------

def make_problem(rng: np.random.Generator, k: int, n: int, m: int, *,
                 F_mode: str = "per_step", cov: str = "diag",
                 H_mode: str = "identity", c_scale: float = 1.0,
                 var_range=(1e-2, 1.0)) -> Problem:
    """Sample one smoothing problem with k evolution steps (k + 1 states).

    F_mode  'const'    one F = Q diag(U[0.95,1]) Q^T for every step
            'per_step' an independent such F_i per step
    cov     'diag'     K_i, C_i diagonal with log-uniform variances in var_range
            'dense'    K_i, C_i = L L^T + 0.1 I, L Gaussian
    H_mode  'identity' H_i = I (H is None)
            'random'   H_i = Q_i diag(U[1, 2]) with Q_i Haar (well conditioned)
    """
    if k < 0 or n < 1 or m < 0:
        raise ValueError("need k >= 0, n >= 1, m >= 0")
    if F_mode == "const":
        F = np.broadcast_to(contracting_F(rng, 1, n), (k, n, n)).copy()
    elif F_mode == "per_step":
        F = contracting_F(rng, k, n) if k else np.zeros((0, n, n))
    else:
        raise ValueError(F_mode)
    G = rng.standard_normal((k + 1, m, n)) / np.sqrt(n)
    if cov == "diag":
        K = loguniform(rng, *var_range, size=(k, n))
        C = loguniform(rng, *var_range, size=(k + 1, m))
        K_diag = C_diag = True
    elif cov == "dense":
        K = spd_dense(rng, k, n) if k else np.zeros((0, n, n))
        C = spd_dense(rng, k + 1, m) if m else np.zeros((k + 1, 0, 0))
        K_diag = C_diag = False
    else:
        raise ValueError(cov)
    if H_mode == "identity":
        H = None
    elif H_mode == "random":
        q = haar_orthogonal(rng, k, n) if k else np.zeros((0, n, n))
        H = q * rng.uniform(1.0, 2.0, size=(k, 1, n))
    else:
        raise ValueError(H_mode)
    c = c_scale * rng.standard_normal((k, n))

    # simulated truth: u_0 ~ N(0, I), then the evolution recurrence
    eps = _noise(rng, K, K_diag, (k, n))
    delta = _noise(rng, C, C_diag, (k + 1, m))
    u = np.empty((k + 1, n))
    u[0] = rng.standard_normal(n)
    for i in range(1, k + 1):
        rhs = F[i - 1] @ u[i - 1] + c[i - 1] + eps[i - 1]
        u[i] = rhs if H is None else np.linalg.solve(H[i - 1], rhs)
    o = np.einsum("tij,tj->ti", G, u) + delta
    return Problem(k=k, n=n, m=m, F=np.ascontiguousarray(F), c=c, K=K, G=G, o=o,
                   C=C, K_diag=K_diag, C_diag=C_diag, H=H, u_true=u)


def paper_shaped(rng: np.random.Generator, k: int, n: int) -> Problem:
    """The paper's own benchmark shape (Section V-B): n = m, fixed random
    orthonormal F and G, H = I, K = L = I and random observations."""
    q = haar_orthogonal(rng, 2, n)
    F = np.broadcast_to(q[0], (k, n, n)).copy()
    G = np.broadcast_to(q[1], (k + 1, n, n)).copy()
    return Problem(k=k, n=n, m=n, F=F, c=np.zeros((k, n)), K=np.ones((k, n)),
                   G=G, o=rng.standard_normal((k + 1, n)), C=np.ones((k + 1, n)),
                   K_diag=True, C_diag=True)


# --------------------------------------------------------------------------
# the five measured workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    0: "single problem, n=4, m=2, k=1000, constant F, diagonal covariances",
    1: "single long trajectory, n=6, m=3, k=100000, per-step F, dense covariances",
    2: "large blocks, n=48, m=24, k=20000, per-step F, diagonal covariances",
    3: "512 uneven problems, k log-uniform [64,16384], n in {4,8,16,32}, m=n/2",
    4: "served requests, k log-uniform [100,200000], n in {6,12,24}, m=n/2",
}


def rng_for(workload_id: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(1000 + workload_id))


def workload(workload_id: int, *, k: Optional[int] = None) -> Problem:
    """Single-problem workloads 0, 1, 2 (k may be overridden for small cases)."""
    rng = rng_for(workload_id)
    if workload_id == 0:
        return make_problem(rng, 1000 if k is None else k, 4, 2, F_mode="const", cov="diag")
    if workload_id == 1:
        return make_problem(rng, 100000 if k is None else k, 6, 3, F_mode="per_step", cov="dense")
    if workload_id == 2:
        return make_problem(rng, 20000 if k is None else k, 48, 24, F_mode="per_step", cov="diag")
    raise ValueError("workloads 3 and 4 are multi-problem: use batch_workload / serving_requests")


def batch_shapes(count: int = 512, k_range=(64, 16384), n_choices=(4, 8, 16, 32),
                 workload_id: int = 3):
    """(k, n) of each problem of the batched workload, in order."""
    rng = rng_for(workload_id)
    ks = np.rint(loguniform(rng, k_range[0], k_range[1], size=count)).astype(np.int64)
    ns = rng.choice(np.asarray(n_choices), size=count)
    return [(int(a), int(b)) for a, b in zip(ks, ns)]


def batch_workload(count: int = 512, k_range=(64, 16384), n_choices=(4, 8, 16, 32),
                   workload_id: int = 3):
    """Problems of the batched workload (diagonal covariances, per-step F, m = n/2)."""
    shapes = batch_shapes(count, k_range, n_choices, workload_id)
    children = np.random.SeedSequence(1000 + workload_id).spawn(count)
    out = []
    for (k, n), ss in zip(shapes, children):
        out.append(make_problem(np.random.default_rng(ss), k, n, n // 2,
                                F_mode="per_step", cov="diag"))
    return out


def serving_requests(count: int, rate_hz: float, k_range=(100, 200000),
                     n_choices=(6, 12, 24), fp32_fraction: float = 0.5,
                     workload_id: int = 4, k_cap: Optional[int] = None):
    """Request descriptors for the serving workload: (arrival_s, k, n, fp32, seed).

    Poisson arrivals at rate_hz; k log-uniform; n uniform over n_choices; the
    precision form of each request is a seeded Bernoulli(fp32_fraction).  The
    problem itself is built lazily with ``request_problem``.
    """
    rng = rng_for(workload_id)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps)
    ks = np.rint(loguniform(rng, k_range[0], k_range[1], size=count)).astype(np.int64)
    if k_cap is not None:
        ks = np.minimum(ks, k_cap)
    ns = rng.choice(np.asarray(n_choices), size=count)
    fp32 = rng.uniform(size=count) < fp32_fraction
    seeds = rng.integers(0, 2**63 - 1, size=count)
    return [dict(arrival_s=float(a), k=int(b), n=int(c), fp32=bool(d), seed=int(e))
            for a, b, c, d, e in zip(t, ks, ns, fp32, seeds)]


def request_problem(req: dict) -> Problem:
    rng = np.random.default_rng(req["seed"])
    n = req["n"]
    return make_problem(rng, req["k"], n, n // 2, F_mode="per_step", cov="dense")


@dataclass
class GeneralProblem:
    """A problem with per-step dimensions (Section II-A): u_i has n[i]
    components; evolution step i = 1..k has l[i-1] equations with H[i-1]
    (l x n_i), F[i-1] (l x n_{i-1}), c[i-1], K[i-1] (l x l, dense); state i has
    m[i] >= 0 observations with G[i] (m_i x n_i), o[i], C[i] (m_i x m_i, dense).
    Every entry of the lists is a float64 numpy array."""
    n: list
    l: list
    m: list
    H: list
    F: list
    c: list
    K: list
    G: list
    o: list
    C: list

    @property
    def k(self) -> int:
        return len(self.n) - 1


def make_general_problem(rng: np.random.Generator, k: int, n_choices=(2, 3, 4, 5),
                         m_extra: int = 1) -> GeneralProblem:
    """Random dimensions per step: n_i from n_choices, l_i in n_i - 1 .. n_i + 1
    (at least 1: H_i rectangular either way, full rank), m_i from
    max(0, n_i - l_i) to n_i + m_extra (zero allowed when H_i has full column rank),
    m_0 = n_0; full column rank overall with probability one.  Dense SPD
    covariances, Haar-based H_i, Gaussian F_i, a simulated trajectory."""
    n = [int(rng.choice(n_choices)) for _ in range(k + 1)]
    l, m = [], [n[0]]
    for i in range(1, k + 1):
        li = max(1, n[i] + int(rng.integers(-1, 2)))
        l.append(li)
        m.append(int(rng.integers(max(0, n[i] - li), n[i] + m_extra + 1)))
    H, F, c, K, G, o, C = [], [], [], [], [], [], []
    u = [rng.standard_normal(n[0])]
    for i in range(1, k + 1):
        li, ni, np_ = l[i - 1], n[i], n[i - 1]
        q = haar_orthogonal(rng, 1, max(li, ni))[0]
        Hi = q[:li, :ni] * rng.uniform(1.0, 2.0, size=(1, ni))
        Fi = rng.standard_normal((li, np_)) / np.sqrt(np_) * 0.9
        Ki = spd_dense(rng, 1, li)[0]
        # a state and the forcing c_i that make the evolution rows hold up to noise
        ui = rng.standard_normal(ni)
        ci = Hi @ ui - Fi @ u[-1] - np.linalg.cholesky(Ki) @ rng.standard_normal(li)
        H.append(Hi); F.append(Fi); c.append(ci); K.append(Ki); u.append(ui)
    for i in range(k + 1):
        mi, ni = m[i], n[i]
        Gi = rng.standard_normal((mi, ni)) / np.sqrt(ni)
        Ci = spd_dense(rng, 1, mi)[0] if mi else np.zeros((0, 0))
        noise = np.linalg.cholesky(Ci) @ rng.standard_normal(mi) if mi else np.zeros(0)
        G.append(Gi); C.append(Ci); o.append(Gi @ u[i] + noise)
    return GeneralProblem(n=n, l=l, m=m, H=H, F=F, c=c, K=K, G=G, o=o, C=C)
