"""Pins of oracle/dense.py permuted_R (no GPU).

permuted_R(p, order) returns the R factor of a thin QR of U A P (P: the block
columns taken in ``order``) and Q^T U b.  It is the expected value of the GPU
test that compares R-factor block rows, so it is pinned here to facts that do
not depend on how it is computed:

* the normal equations: R^T R = P^T (A^T W A) P and R^T (Q^T U b) = P^T A^T W b
  for every QR of U A P, with (A^T W A, A^T W b) from dense.normal_matrix
  (itself pinned to a Kalman filter + RTS smoother and to a least-squares
  solve in test_oracle_pins.py);
* the structure of Section III (Fig. R-structures, drawn for k = 50): in the
  odd-even order the block row of a column eliminated at level l has at most
  two off-diagonal blocks, on the columns i - 2^l and i + 2^l, both eliminated
  later; level l eliminates ceil(N_l / 2) columns, N_l = floor((k+1) / 2^l),
  and the last level one;
* planted mistakes in a copy of the function (order ignored, columns of a
  block reversed, rows out of step with the right-hand side, a wrong whitening
  factor, right-hand side not rotated) each fail one of the pins.
"""
import inspect

import numpy as np
import pytest

from oracle import dense
from paper_2502_11686_amd import gen


def level(i):
    """Level at which original column i is eliminated: ctz(i + 1)."""
    return ((i + 1) & -(i + 1)).bit_length() - 1


def odd_even_order(k):
    return sorted(range(k + 1), key=lambda i: (level(i), i))


def perm_cols(n, order):
    return np.concatenate([np.arange(i * n, (i + 1) * n) for i in order])


def check_normal_equations(p, order, R, qtb):
    J, h = dense.normal_matrix(p)
    cols = perm_cols(p.n, order)
    Jp = J[np.ix_(cols, cols)]
    scale = np.linalg.norm(J)
    assert np.allclose(R, np.triu(R), rtol=0, atol=0), "R is not upper triangular"
    assert np.linalg.norm(R.T @ R - Jp) < 1e-12 * scale, "R^T R != P^T A^T W A P"
    assert np.linalg.norm(R.T @ qtb - h[cols]) < 1e-11 * max(1.0, np.linalg.norm(h)), \
        "R^T Q^T U b != P^T A^T W b"


def check_odd_even_structure(p, order, R):
    n, k = p.n, p.k
    pos = {c: q for q, c in enumerate(order)}
    for q, i in enumerate(order):
        l = level(i)
        rows = slice(q * n, (q + 1) * n)
        diag = np.linalg.norm(R[rows, q * n:(q + 1) * n])
        nbrs = {i - (1 << l), i + (1 << l)} & set(range(k + 1))
        for c in nbrs:  # neighbours are eliminated after i
            assert pos[c] > q and level(c) > l, (i, c)
        for c in range(k + 1):
            if pos[c] <= q or c in nbrs:
                continue
            blk = R[rows, pos[c] * n:(pos[c] + 1) * n]
            assert np.linalg.norm(blk) < 1e-12 * diag, f"block ({i}, {c}) should be zero"


@pytest.mark.parametrize("k,n,m,cov,H", [(50, 2, 1, "diag", "identity"), (50, 3, 2, "dense", "random"),
                                         (37, 3, 2, "dense", "random"), (64, 4, 2, "diag", "identity"),
                                         (20, 4, 4, "dense", "random"), (0, 3, 3, "diag", "identity")])
def test_permuted_R_normal_equations_and_structure(k, n, m, cov, H):
    p = gen.make_problem(np.random.default_rng(300 + k + n), k, n, m, cov=cov, H_mode=H)
    order = odd_even_order(k)
    R, qtb = dense.permuted_R(p, order)
    assert R.shape == ((k + 1) * n, (k + 1) * n) and qtb.shape == ((k + 1) * n,)
    check_normal_equations(p, order, R, qtb)
    check_odd_even_structure(p, order, R)


def test_permuted_R_natural_order_is_block_bidiagonal():
    """In the natural order (the sequential smoother's) each block row has one
    off-diagonal block, on the next column."""
    k, n = 30, 3
    p = gen.make_problem(np.random.default_rng(5), k, n, 2, cov="dense", H_mode="random")
    order = list(range(k + 1))
    R, qtb = dense.permuted_R(p, order)
    check_normal_equations(p, order, R, qtb)
    for i in range(k + 1):
        rows = slice(i * n, (i + 1) * n)
        diag = np.linalg.norm(R[rows, i * n:(i + 1) * n])
        for c in range(i + 2, k + 1):
            assert np.linalg.norm(R[rows, c * n:(c + 1) * n]) < 1e-12 * diag


@pytest.mark.parametrize("k", [0, 1, 2, 7, 50, 63, 64, 100, 1000, 100000])
def test_columns_per_level(k):
    """Level l eliminates ceil(N_l / 2) columns, N_l = floor((k+1) / 2^l); the
    last level, L = floor(log2(k+1)), one (Section III recursion)."""
    counts = {}
    for i in range(k + 1):
        counts[level(i)] = counts.get(level(i), 0) + 1
    L = (k + 1).bit_length() - 1
    assert max(counts) == L and counts[L] == 1
    for l in range(L + 1):
        Nl = (k + 1) >> l
        assert counts[l] == (Nl + 1) // 2, (k, l)


# ------------------------------------------------------------ planted mistakes

def _mutant(replacements):
    """A copy of permuted_R (and of whitened, which it calls) with textual
    replacements applied, compiled in a copy of the oracle module's namespace."""
    ns = dict(vars(dense))
    for fn in (dense.whitened, dense.permuted_R):
        src = inspect.getsource(fn)
        for old, new in replacements:
            src = src.replace(old, new)
        exec(compile(src, "<mutant>", "exec"), ns)
    return ns["permuted_R"]


MUTANTS = {
    "order ignored": [("for i in order", "for i in sorted(order)")],
    "block columns reversed": [("np.arange(i * n, (i + 1) * n)", "np.arange(i * n, (i + 1) * n)[::-1]")],
    "rows out of step with rhs": [("UA, Ub = whitened(p)", "UA, Ub = whitened(p); UA = UA[::-1]")],
    "whitening by L^T": [("L = np.linalg.cholesky(cov_e)", "L = np.linalg.cholesky(cov_e).T")],
    "rhs not rotated": [("return r, q.T @ Ub", "return r, Ub[:r.shape[0]]")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_in_permuted_R_is_caught(name):
    for old, _ in MUTANTS[name]:
        assert sum(inspect.getsource(f).count(old) for f in (dense.whitened, dense.permuted_R)) == 1, old
    fn = _mutant(MUTANTS[name])
    p = gen.make_problem(np.random.default_rng(11), 50, 3, 2, cov="dense", H_mode="random")
    order = odd_even_order(p.k)
    R, qtb = fn(p, order)
    with pytest.raises(AssertionError):
        check_normal_equations(p, order, R, qtb)
        check_odd_even_structure(p, order, R)


def test_unmutated_copy_passes():
    fn = _mutant([])
    p = gen.make_problem(np.random.default_rng(11), 50, 3, 2, cov="dense", H_mode="random")
    order = odd_even_order(p.k)
    R, qtb = fn(p, order)
    check_normal_equations(p, order, R, qtb)
    check_odd_even_structure(p, order, R)
