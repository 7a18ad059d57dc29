"""GPU: Gauss-Newton and Levenberg-Marquardt smoothing of a nonlinear model
(Section II-B), every linear problem solved by ks_smooth (no covariances) and
every objective value by ks_objective, against the same iteration on the CPU
with the sequential oracle (tests/nonlinear_ref.py, pinned on the CPU to a
zero gradient at its limit point)."""
import numpy as np
import pytest
import torch

from paper_2502_11686_amd import nonlinear
from tests import nonlinear_ref as nl

pytestmark = pytest.mark.gpu


def _dev(d, key):
    return torch.from_numpy(np.ascontiguousarray(d[key])).to("cuda")


@pytest.mark.parametrize("method", ["gn", "lm"])
@pytest.mark.parametrize("k,dense_cov,spread", [(200, False, 1.0), (1500, True, 8.0), (20000, False, 16.0)])
def test_nonlinear_matches_cpu_iteration(method, k, dense_cov, spread):
    d = nl.make_data(100 + k, k, dense_cov=dense_cov, spread=spread)
    res = nonlinear.smooth_nonlinear(nl.TorchModel(), _dev(d, "u0"), None, _dev(d, "c"), _dev(d, "K"),
                                     _dev(d, "o"), _dev(d, "C"), d["K_diag"], d["C_diag"], method=method)
    ref = nl.reference(d, method=method)
    assert res.converged and ref["converged"]
    u = res.u.cpu().numpy()
    scale = np.abs(ref["u"]).max()
    assert np.max(np.abs(u - ref["u"])) <= 1e-8 * scale
    assert np.isclose(res.objective, ref["objective"], rtol=1e-10)
    # the first accepted steps (far from ties) take the same decisions
    nh = min(3, len(ref["history"]), len(res.history))
    assert np.allclose(res.history[:nh], ref["history"][:nh], rtol=1e-9)
    if k <= 1500:
        g = nl.gradient(d, u)
        assert np.abs(g).max() <= 1e-6 * np.abs(nl.gradient(d, d["u0"])).max()


def test_nonlinear_final_covariance():
    """want_cov returns the covariance blocks of the last linearization."""
    d = nl.make_data(7, 300, dense_cov=True, spread=2.0)
    res = nonlinear.smooth_nonlinear(nl.TorchModel(), _dev(d, "u0"), None, _dev(d, "c"), _dev(d, "K"),
                                     _dev(d, "o"), _dev(d, "C"), d["K_diag"], d["C_diag"], want_cov=True)
    from oracle import seq
    ref = nl.reference(d)
    c, o, F, G = nl._lin(ref["u"], d)
    lin = seq.smooth(nl._problem(d, F, G, c, o, d["C"], d["m"]), want_cov=True)
    S = res.cov.cpu().numpy()
    err = np.max(np.linalg.norm(S - lin["cov"], axis=(1, 2)) / np.linalg.norm(lin["cov"], axis=(1, 2)))
    assert err < 1e-7, err
