"""Host logic of the per-step-dimension embedding (no GPU): the embedded
uniform problem has the original problem's estimate and covariance blocks
(dense definition on both sides), and the chosen kernel class holds it."""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import dense
from paper_2502_11686_amd import gen, general, ks


@pytest.mark.parametrize("seed,k,n_choices,m_extra", [(0, 9, (2, 3, 4, 5), 1), (1, 0, (3,), 1),
                                                      (2, 6, (1, 2), 1), (3, 5, (10, 14), 0)])
def test_embedding_is_exact(seed, k, n_choices, m_extra):
    gp = gen.make_general_problem(np.random.default_rng(seed), k, n_choices, m_extra)
    n, m = general.embedding_dims(gp)
    assert n >= max(gp.n) and ks.supported(n, m)
    H, F, c, K, G, o, C = general.embed(gp, n, m)
    p = SimpleNamespace(k=gp.k, n=n, m=m, H=H, F=F, c=c, K=K, G=G, o=o, C=C, K_diag=False, C_diag=False)
    emb = dense.smooth(p)
    ref = dense.smooth_general(gp)
    for i in range(gp.k + 1):
        ni = gp.n[i]
        assert np.allclose(emb["u"][i][:ni], ref["u"][i], rtol=0, atol=1e-10 * max(1, np.abs(ref["u"][i]).max()))
        assert np.allclose(emb["cov"][i][:ni, :ni], ref["cov"][i], rtol=1e-9, atol=1e-12)
        # padding components are decoupled: unit variance, no correlation with real ones
        assert np.allclose(emb["cov"][i][ni:, ni:], np.eye(n - ni), atol=1e-12)
        assert np.allclose(emb["cov"][i][:ni, ni:], 0.0, atol=1e-12)


def test_embedding_rejects_what_no_class_holds():
    gp = gen.make_general_problem(np.random.default_rng(5), 3, (40,), 1)
    gp.m[0] = 60
    gp.G[0] = np.zeros((60, gp.n[0]))
    gp.o[0] = np.zeros(60)
    gp.C[0] = np.eye(60)
    with pytest.raises(ks.KsError):
        general.embedding_dims(gp)
