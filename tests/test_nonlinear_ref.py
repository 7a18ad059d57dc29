"""Pins of the CPU reference of the Gauss-Newton / Levenberg-Marquardt
iteration (tests/nonlinear_ref.py) against what the mathematics fixes: the
model's Jacobians against finite differences, and the limit point against a
zero gradient of the nonlinear objective (Section II-B)."""
import numpy as np
import pytest

from tests import nonlinear_ref as nl


def test_jacobians_match_finite_differences():
    rng = np.random.default_rng(3)
    u = np.array([[20.0, 1.0, 1.0, 0.6]]) + 0.1 * rng.standard_normal((1, 4))
    _, F = nl.f_np(u)
    _, G = nl.g_np(u)
    h = 1e-6
    for j in range(4):
        e = np.zeros((1, 4))
        e[0, j] = h
        fd_f = (nl.f_np(u + e)[0] - nl.f_np(u - e)[0]) / (2 * h)
        fd_g = (nl.g_np(u + e)[0] - nl.g_np(u - e)[0]) / (2 * h)
        assert np.allclose(fd_f[0], F[0][:, j], atol=1e-8)
        assert np.allclose(fd_g[0], G[0][:, j], atol=1e-8)


def test_gradient_matches_finite_differences():
    d = nl.make_data(11, 12, dense_cov=True)
    u = d["u0"]
    g = nl.gradient(d, u)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(u.shape)
    h = 1e-5
    fd = (nl.objective(d, u + h * v) - nl.objective(d, u - h * v)) / (2 * h)
    assert np.isclose(fd, np.sum(g * v), rtol=1e-6)


@pytest.mark.parametrize("dense_cov", [False, True])
def test_reference_reaches_a_stationary_point(dense_cov):
    d = nl.make_data(12, 30, dense_cov=dense_cov)
    g0 = np.abs(nl.gradient(d, d["u0"])).max()
    res = {}
    for method in ("gn", "lm"):
        r = nl.reference(d, method=method)
        assert r["converged"]
        assert all(b <= a for a, b in zip(r["history"], r["history"][1:]))
        assert np.abs(nl.gradient(d, r["u"])).max() <= 1e-7 * g0
        res[method] = r
    # both globalizations reach the same minimum from the same start
    assert np.allclose(res["gn"]["u"], res["lm"]["u"], rtol=0, atol=1e-7)
