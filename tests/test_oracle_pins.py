"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

The sequential oracle (oracle/seq.py) and the dense definition (oracle/dense.py)
are pinned to references other than themselves:

* the dense definition against a textbook Kalman filter + RTS smoother in the
  proper-prior special case, and against a QR-based least-squares solve;
* the sequential oracle against the dense definition over a sweep of k, n, m,
  covariance layouts and H, with both of its covariance forms (the RTS
  recursion in square-root form over R, and the RTS recursion in information
  form over the model matrices, which shares no step with it), and the two
  forms against each other on long problems;
* both against closed forms (k = 0), invariants (symmetry, positive
  definiteness, zero gradient of the objective at u_hat, residual identity) and
  a Monte Carlo estimate of cov(u_hat).
"""
import numpy as np
import pytest

from oracle import dense, seq
from paper_2502_11686_amd import gen
from tests.kalman_rts import kf_rts


def rel_state_err(u, ref):
    return np.max(np.abs(u - ref)) / max(np.max(np.abs(ref)), 1e-300)


def rel_cov_err(S, ref):
    num = np.linalg.norm(S - ref, axis=(1, 2))
    den = np.linalg.norm(ref, axis=(1, 2))
    return float(np.max(num / den))


def small(seed, k, n, m, cov="diag", H_mode="identity", F_mode="per_step"):
    rng = np.random.default_rng(seed)
    return gen.make_problem(rng, k, n, m, F_mode=F_mode, cov=cov, H_mode=H_mode)


def with_prior(p, seed):
    """Make the observation of u_0 a proper prior N(mu_0, P_0) (needs m = n)."""
    rng = np.random.default_rng(seed)
    n = p.n
    p.G[0] = np.eye(n)
    p.o[0] = rng.standard_normal(n)
    if p.C_diag:
        p.C[0] = gen.loguniform(rng, 0.1, 2.0, n)
    else:
        p.C[0] = gen.spd_dense(rng, 1, n)[0]
    return p


# ---------------------------------------------------------------- dense pins

@pytest.mark.parametrize("cov", ["diag", "dense"])
@pytest.mark.parametrize("k,n", [(0, 3), (1, 2), (5, 3), (12, 4)])
def test_dense_definition_equals_kalman_rts(k, n, cov):
    p = with_prior(small(10 + k, k, n, n, cov=cov), 99)
    d = dense.smooth(p)
    xs, Ps = kf_rts(p)
    assert rel_state_err(d["u"], xs) < 1e-10
    assert rel_cov_err(d["cov"], Ps) < 1e-9


@pytest.mark.parametrize("k,n,m", [(0, 2, 3), (4, 3, 2), (9, 2, 1)])
def test_dense_definition_equals_qr_lstsq(k, n, m):
    p = small(20 + k, k, n, m, cov="dense")
    assert rel_state_err(dense.smooth(p)["u"], dense.smooth_lstsq(p)) < 1e-10


# ------------------------------------------------------ sequential vs dense

SHAPES = [(1, 1), (2, 1), (4, 2), (3, 3), (6, 3), (4, 5)]
KS = list(range(0, 20)) + [31, 32, 33, 63, 64, 100]


@pytest.mark.parametrize("n,m", SHAPES)
def test_sequential_matches_dense_sweep(n, m):
    worst_u = worst_s = 0.0
    for k in KS:
        if (k + 1) * m < n:
            continue  # rank deficient: covered by test_rank_deficiency
        for cov in ("diag", "dense"):
            for H_mode in ("identity", "random"):
                p = small(1000 * n + 10 * m + k, k, n, m, cov=cov, H_mode=H_mode)
                d = dense.smooth(p)
                for from_rts in (False, True):  # square-root RTS over R; information-form RTS
                    o = seq.smooth(p, want_lag1=True, rts=from_rts)
                    worst_u = max(worst_u, rel_state_err(o["u"], d["u"]))
                    worst_s = max(worst_s, rel_cov_err(o["cov"], d["cov"]))
                    assert abs(o["resid2"] - d["resid2"]) <= 1e-9 * max(1.0, d["resid2"])
                    nn = p.n
                    for i in range(k):
                        lag = d["S"][i * nn:(i + 1) * nn, (i + 1) * nn:(i + 2) * nn]
                        assert np.linalg.norm(o["lag1"][i] - lag) <= 1e-9 * np.linalg.norm(lag) + 1e-14
    assert worst_u < 1e-11, worst_u
    assert worst_s < 1e-10, worst_s


def test_sequential_matches_kalman_rts_long():
    p = with_prior(small(7, 400, 4, 4, cov="dense"), 5)
    xs, Ps = kf_rts(p)
    for from_rts in (False, True):
        o = seq.smooth(p, rts=from_rts)
        assert rel_state_err(o["u"], xs) < 1e-9
        assert rel_cov_err(o["cov"], Ps) < 1e-8


@pytest.mark.parametrize("n,m,cov,H_mode", [(6, 3, "dense", "identity"), (4, 2, "diag", "random"),
                                            (12, 6, "dense", "random"), (24, 12, "diag", "identity")])
def test_rts_recursion_agrees_with_selected_inversion(n, m, cov, H_mode):
    """The oracle's two covariance forms, the square-root RTS recursion over R
    and the information-form RTS recursion over the model matrices, on
    problems too long for the dense definition.  These problems are well
    conditioned (cond(A^T W A) below 1e6), so the information form, whose
    error grows with that condition number, agrees to 1e-11."""
    p = small(77 + n, 3000 if n <= 12 else 400, n, m, cov=cov, H_mode=H_mode)
    a = seq.smooth(p, want_lag1=True)
    b = seq.smooth(p, want_lag1=True, rts=True)
    assert np.array_equal(a["u"], b["u"])
    assert rel_cov_err(a["cov"], b["cov"]) < 1e-11
    scale = np.sqrt(np.linalg.norm(a["cov"][:-1], axis=(1, 2)) * np.linalg.norm(a["cov"][1:], axis=(1, 2)))
    assert np.max(np.linalg.norm(a["lag1"] - b["lag1"], axis=(1, 2)) / scale) < 1e-11


def test_k0_closed_form():
    rng = np.random.default_rng(3)
    p = gen.make_problem(rng, 0, 3, 5, cov="dense")
    L = np.linalg.cholesky(p.C[0])
    Gw = np.linalg.solve(L, p.G[0])
    ow = np.linalg.solve(L, p.o[0])
    J = Gw.T @ Gw
    u0 = np.linalg.solve(J, Gw.T @ ow)
    o = seq.smooth(p)
    assert rel_state_err(o["u"][0], u0) < 1e-12
    assert rel_cov_err(o["cov"], np.linalg.inv(J)[None]) < 1e-12


# ---------------------------------------------------------------- invariants

def gradient_blocks(p, u):
    """Blocks of A^T W (A u - b), computed step by step with K^{-1}, C^{-1}."""
    k, n = p.k, p.n
    g = np.zeros((k + 1, n))
    cov = lambda x, d: np.diag(x) if d else x
    for i in range(k + 1):
        if p.m:
            r = p.G[i] @ u[i] - p.o[i]
            g[i] += p.G[i].T @ np.linalg.solve(cov(p.C[i], p.C_diag), r)
        if i >= 1:
            H = np.eye(n) if p.H is None else p.H[i - 1]
            r = H @ u[i] - p.F[i - 1] @ u[i - 1] - p.c[i - 1]
            w = np.linalg.solve(cov(p.K[i - 1], p.K_diag), r)
            g[i] += H.T @ w
            g[i - 1] -= p.F[i - 1].T @ w
    return g


@pytest.mark.parametrize("wid", [0])
def test_invariants_full_workload0(wid):
    p = gen.workload(wid)
    o = seq.smooth(p)
    S = o["cov"]
    assert np.array_equal(S, np.swapaxes(S, 1, 2))
    np.linalg.cholesky(S)  # raises if any block is not positive definite
    g = gradient_blocks(p, o["u"])
    scale = np.max(np.abs(gradient_blocks(p, np.zeros_like(o["u"]))))
    assert np.max(np.abs(g)) < 1e-11 * scale


def test_gradient_zero_dense_covariances():
    p = gen.workload(1, k=2000)
    o = seq.smooth(p, want_cov=False)
    g = gradient_blocks(p, o["u"])
    scale = np.max(np.abs(gradient_blocks(p, np.zeros_like(o["u"]))))
    assert np.max(np.abs(g)) < 1e-11 * scale


def test_monte_carlo_covariance_and_unbiasedness():
    """cov(u_hat) over repeated noise draws matches Sigma (Section IV), and
    E[u_hat] = u (the estimator is unbiased, Section II-A).

    The model (F, G, K, C) and the true trajectory stay fixed; each draw makes
    fresh data b = A u + e with e ~ N(0, cov(e)), i.e. c_i = u_i - F_i u_{i-1}
    - eps_i and o_i = G_i u_i + delta_i."""
    rng = np.random.default_rng(11)
    p = gen.make_problem(rng, 6, 2, 1, cov="dense")
    base = seq.smooth(p)
    u = p.u_true
    LK = np.linalg.cholesky(p.K)
    LC = np.linalg.cholesky(p.C)
    draws = 4000
    est = np.zeros((draws, p.k + 1, p.n))
    r = np.random.default_rng(12)
    for t in range(draws):
        eps = np.einsum("tij,tj->ti", LK, r.standard_normal((p.k, p.n)))
        dlt = np.einsum("tij,tj->ti", LC, r.standard_normal((p.k + 1, p.m)))
        q = gen.Problem(k=p.k, n=p.n, m=p.m, F=p.F, K=p.K, G=p.G, C=p.C,
                        K_diag=False, C_diag=False, H=None,
                        c=u[1:] - np.einsum("tij,tj->ti", p.F, u[:-1]) - eps,
                        o=np.einsum("tij,tj->ti", p.G, u) + dlt)
        est[t] = seq.smooth(q, want_cov=False)["u"]
    mean = est.mean(axis=0)
    for i in range(p.k + 1):
        Sig = base["cov"][i]
        d = np.linalg.solve(np.linalg.cholesky(Sig), mean[i] - u[i])
        assert np.linalg.norm(d) * np.sqrt(draws) < 5.0  # mean within ~5 sigma
        emp = np.cov(est[:, i, :].T)
        assert np.linalg.norm(emp - Sig) <= 0.12 * np.linalg.norm(Sig)


# ------------------------------------------------------------- error paths

def test_rank_deficiency():
    rng = np.random.default_rng(1)
    p = gen.make_problem(rng, 0, 3, 2)  # k = 0 with m < n
    assert seq.smooth(p, check=False)["status"] == seq.E_RANK
    p = gen.make_problem(rng, 5, 2, 1)
    p.G[:] = 0.0  # nothing observes the states
    assert seq.smooth(p, check=False)["status"] == seq.E_RANK


def test_not_spd():
    rng = np.random.default_rng(2)
    p = gen.make_problem(rng, 4, 2, 1)
    p.K[2, 1] = -1.0
    assert seq.smooth(p, check=False)["status"] == seq.E_NOT_SPD
    p = gen.make_problem(rng, 4, 2, 2, cov="dense")
    p.C[1] = -np.eye(2)
    assert seq.smooth(p, check=False)["status"] == seq.E_NOT_SPD


def test_objective_terms_scalar_closed_form():
    """k = 1, n = m = 1: the objective written out by hand,
    (g0 u0 - o0)^2/C0 + (h u1 - f u0 - c)^2/K + (g1 u1 - o1)^2/C1."""
    p = small(31, 1, 1, 1, cov="diag", H_mode="random")
    u = np.array([[0.7], [-1.3]])
    h, f, c, K = p.H[0, 0, 0], p.F[0, 0, 0], p.c[0, 0], p.K[0, 0]
    g0, g1, o0, o1, C0, C1 = p.G[0, 0, 0], p.G[1, 0, 0], p.o[0, 0], p.o[1, 0], p.C[0, 0], p.C[1, 0]
    t0 = (g0 * 0.7 - o0) ** 2 / C0
    t1 = (h * -1.3 - f * 0.7 - c) ** 2 / K + (g1 * -1.3 - o1) ** 2 / C1
    terms = dense.objective_terms(p, u)
    assert np.allclose(terms, [t0, t1], rtol=1e-14, atol=0)


@pytest.mark.parametrize("cov,H_mode", [("diag", "identity"), ("dense", "random")])
def test_objective_terms_sum_to_assembled_quadratic(cov, H_mode):
    """The per-step terms add up to (Au - b)^T cov(e)^{-1} (Au - b) of the
    assembled problem, and at u_hat to its minimum, with
    J(u_hat + d) - J(u_hat) = d^T A^T W A d for any d."""
    p = small(32, 9, 3, 2, cov=cov, H_mode=H_mode)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((p.k + 1, p.n))
    A, b, cov_e = dense.assemble(p)
    r = A @ u.ravel() - b
    assert np.isclose(dense.objective_terms(p, u).sum(), r @ np.linalg.solve(cov_e, r), rtol=1e-12)
    ref = dense.smooth(p)
    J0 = dense.objective_terms(p, ref["u"]).sum()
    assert np.isclose(J0, ref["resid2"], rtol=1e-10)
    d = rng.standard_normal(A.shape[1])
    Ad = A @ d
    J1 = dense.objective_terms(p, ref["u"] + d.reshape(p.k + 1, p.n)).sum()
    assert np.isclose(J1 - J0, Ad @ np.linalg.solve(cov_e, Ad), rtol=1e-9)


def _uniform_as_general(p):
    n, m, k = p.n, p.m, p.k
    H = [np.eye(n) if p.H is None else p.H[t] for t in range(k)]
    K = [np.diag(p.K[t]) if p.K_diag else p.K[t] for t in range(k)]
    C = [np.diag(p.C[i]) if p.C_diag else p.C[i] for i in range(k + 1)]
    return gen.GeneralProblem(n=[n] * (k + 1), l=[n] * k, m=[m] * (k + 1), H=H, F=list(p.F), c=list(p.c),
                              K=K, G=list(p.G), o=list(p.o), C=C)


def test_general_oracle_reduces_to_uniform():
    p = small(41, 7, 3, 2, cov="dense", H_mode="random")
    ref = dense.smooth(p)
    g = dense.smooth_general(_uniform_as_general(p))
    assert np.allclose(np.stack(g["u"]), ref["u"], rtol=0, atol=1e-12 * np.abs(ref["u"]).max())
    assert np.allclose(np.stack(g["cov"]), ref["cov"], rtol=1e-10, atol=1e-14)


def _objective_per_step(gp, us):
    """sum_i r_i^T K_i^{-1} r_i + s_i^T C_i^{-1} s_i, written step by step."""
    J = 0.0
    for i in range(gp.k + 1):
        if i >= 1:
            r = gp.H[i - 1] @ us[i] - gp.F[i - 1] @ us[i - 1] - gp.c[i - 1]
            J += r @ np.linalg.solve(gp.K[i - 1], r)
        if gp.m[i]:
            s = gp.G[i] @ us[i] - gp.o[i]
            J += s @ np.linalg.solve(gp.C[i], s)
    return J


def test_general_oracle_against_per_step_objective():
    """u_hat zeroes the gradient of the objective written per step, and
    Sigma = (Hessian / 2)^{-1}, both by central differences (the objective is
    quadratic, so second differences are exact up to rounding)."""
    gp = gen.make_general_problem(np.random.default_rng(42), 5)
    ref = dense.smooth_general(gp)
    off = np.concatenate([[0], np.cumsum(gp.n)])
    N = int(off[-1])
    x0 = np.concatenate(ref["u"])

    def f(x):
        return _objective_per_step(gp, [x[off[i]:off[i + 1]] for i in range(gp.k + 1)])

    h = 1e-3
    E = np.eye(N) * h
    grad = np.array([(f(x0 + E[a]) - f(x0 - E[a])) / (2 * h) for a in range(N)])
    assert np.abs(grad).max() < 1e-6 * max(1.0, f(x0))
    Hs = np.empty((N, N))
    for a in range(N):
        for b in range(N):
            Hs[a, b] = (f(x0 + E[a] + E[b]) - f(x0 + E[a] - E[b]) - f(x0 - E[a] + E[b]) + f(x0 - E[a] - E[b])) / (4 * h * h)
    S = np.linalg.inv(Hs / 2)
    for i in range(gp.k + 1):
        blk = S[off[i]:off[i + 1], off[i]:off[i + 1]]
        assert np.allclose(ref["cov"][i], blk, rtol=1e-5, atol=1e-7 * np.abs(blk).max())
    for i in range(gp.k):
        blk = S[off[i]:off[i + 1], off[i + 1]:off[i + 2]]
        assert np.allclose(ref["lag1"][i], blk, rtol=1e-5, atol=1e-6 * np.abs(S).max())


def test_general_oracle_unobserved_step_is_the_infinite_variance_limit():
    """m_i = 0 equals observing u_i with a variance going to infinity."""
    gp = gen.make_general_problem(np.random.default_rng(43), 6)
    i = 3  # unobserved, with an evolution block of full column rank (l_i = n_i + 1)
    rng = np.random.default_rng(1)
    li = gp.n[i] + 1
    gp.l[i - 1] = li
    gp.H[i - 1] = rng.standard_normal((li, gp.n[i]))
    gp.F[i - 1] = rng.standard_normal((li, gp.n[i - 1]))
    gp.c[i - 1] = rng.standard_normal(li)
    gp.K[i - 1] = np.eye(li)
    gp.m[i], gp.G[i], gp.o[i], gp.C[i] = 0, np.zeros((0, gp.n[i])), np.zeros(0), np.zeros((0, 0))
    ref = dense.smooth_general(gp)
    rng = np.random.default_rng(2)
    big = gen.GeneralProblem(**{f: list(getattr(gp, f)) for f in ("n", "l", "m", "H", "F", "c", "K", "G", "o", "C")})
    big.m[i] = 2
    big.G[i] = rng.standard_normal((2, gp.n[i]))
    big.o[i] = rng.standard_normal(2)
    big.C[i] = 1e14 * np.eye(2)
    lim = dense.smooth_general(big)
    for t in range(gp.k + 1):
        assert np.allclose(lim["u"][t], ref["u"][t], rtol=0, atol=1e-8 * max(1.0, np.abs(ref["u"][t]).max()))
        assert np.allclose(lim["cov"][t], ref["cov"][t], rtol=1e-8, atol=1e-10)
